"""The C-ABI conventions on the GPU: results that do not fit the caller's
capacity (the TM_ECAPACITY case: the count says how many there were, the
best `capacity` by key are written), device memory from a registered
allocator (torch's caching allocator), and rotated tables cached per angle
grid on one model used with several grids in turn."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05576_amd as P

    P.lib()
    return P


def _c2(index=0):
    import paper_2112_05576_amd as P

    sc = synth.scene_for_config(2, index)
    cfg = sc.config
    L = cfg["levels"]
    return P, sc, cfg, L


def test_detect_capacity_overflow():
    P, sc, cfg, L = _c2(0)
    case("capacity overflow C2 image 0")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    full = P.detect(gm, pyr, sp)
    assert len(full) >= 2, len(full)
    for cap in (1, len(full) - 1):
        with pytest.raises(P.TMError) as e:
            P.detect(gm, pyr, sp, capacity=cap)
        assert e.value.status == P.TM_ECAPACITY
        # deterministic truncation: the best `cap` of the full result, bit for bit
        assert e.value.poses.tobytes() == full[:cap].tobytes()
    # the raw count: every match is counted, only `cap` are written
    out = torch.full((3, P.tm.POSE_WORDS), -7, dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.detect_async(gm, pyr, sp, out[:1], n)
    assert int(n.item()) == len(full)
    assert int(out[1, 0].item()) == -7  # nothing written past the capacity
    # exactly at the capacity: no error
    assert P.detect(gm, pyr, sp, capacity=len(full)).tobytes() == full.tobytes()
    # batches: the same per pair
    imgs = [torch.from_numpy(synth.scene_for_config(2, i).image).cuda() for i in range(3)]
    b = P.Batch([gm], imgs, L, cfg["tau_s"], sp, capacity=1)
    b.run()
    with pytest.raises(P.TMError) as e:
        b.results()
    assert e.value.status == P.TM_ECAPACITY
    for i, im in enumerate(imgs):
        pyr.update(im)
        ref = P.detect(gm, pyr, sp)
        assert e.value.poses[i].tobytes() == ref[:1].tobytes()


def test_torch_allocator():
    """Handles take their memory from torch's caching allocator once it is
    registered: a counting wrapper around it sees every handle allocate and
    free all it took; results are those of hipMalloc'd handles; handles made
    after switching back take nothing from it."""
    import ctypes

    from paper_2112_05576_amd import tm

    P, sc, cfg, L = _c2(1)
    case("torch caching allocator")
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    gm0 = P.Model(sc.model, L, cfg["tau_m"])
    pyr0 = P.Pyramid(sc.image, L, cfg["tau_s"])
    ref = P.detect(gm0, pyr0, sp)
    img = torch.from_numpy(sc.image).cuda()
    live = {}

    def alloc(nbytes, ctx, stream):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        live[p] = int(nbytes)
        return p

    def free(ptr, ctx, stream):
        live.pop(int(ptr))
        torch.cuda.caching_allocator_delete(int(ptr))

    a = tm.AllocatorC(tm._ALLOC_FN(alloc), tm._FREE_FN(free), None)
    assert P.lib().tm_set_allocator(ctypes.byref(a)) == 0
    try:
        gm = P.Model(sc.model, L, cfg["tau_m"])
        m_bytes = sum(live.values())
        assert m_bytes > 0  # the model's points and directions
        pyr = P.Pyramid(img, L, cfg["tau_s"])
        assert sum(live.values()) - m_bytes >= 640 * 480 * 9  # the pyramid's levels and fields
        got = P.detect(gm, pyr, sp)
        assert got.tobytes() == ref.tobytes()
        b = P.Batch([gm], [img], L, cfg["tau_s"], sp)
        b.run(graph=True)
        assert b.results()[0].tobytes() == ref.tobytes()
        torch.cuda.synchronize()
        b.free()
        pyr.free()
        gm.free()
        assert not live, live  # every block handed back
    finally:
        assert P.lib().tm_set_allocator(None) == 0
    # the binding's own registration: torch's caching allocator as it is
    P.use_torch_allocator(True)
    try:
        gm = P.Model(sc.model, L, cfg["tau_m"])
        pyr = P.Pyramid(img, L, cfg["tau_s"])
        assert P.detect(gm, pyr, sp).tobytes() == ref.tobytes()
        pyr.free()
        gm.free()
    finally:
        P.use_torch_allocator(False)
    # handles made after switching back take nothing from the wrapper
    pyr2 = P.Pyramid(img, L, cfg["tau_s"])
    assert not live
    assert P.detect(gm0, pyr2, sp).tobytes() == ref.tobytes()


def test_tables_cached_per_grid():
    """One model searched with two angle grids in turn, and on two streams at
    once: every result equals that of a fresh model with one grid."""
    P, sc, cfg, L = _c2(2)
    case("rotated tables per grid")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
    pyr_b = P.Pyramid(sc.image, L, cfg["tau_s"])
    grids = [P.SearchParams(theta_step_top=1.0), P.SearchParams(theta_step_top=2.0),
             P.SearchParams(theta_step_top=1.0, theta_min=-30.0, theta_range=60.0)]
    ref = []
    for sp in grids:
        fresh = P.Model(sc.model, L, cfg["tau_m"])
        ref.append(P.detect(fresh, pyr, sp))
    for rep in range(2):
        for sp, r in zip(grids, ref):
            assert P.detect(gm, pyr, sp).tobytes() == r.tobytes()
    # two streams, two grids, one model
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [torch.empty((8, P.tm.POSE_WORDS), dtype=torch.int32, device="cuda") for _ in range(2)]
    ns = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    for it in range(4):
        P.detect_async(gm, pyr, grids[it % 2], outs[0], ns[0], stream=s1)
        P.detect_async(gm, pyr_b, grids[(it + 1) % 2], outs[1], ns[1], stream=s2)
    torch.cuda.synchronize()
    got0 = P.poses_to_numpy(outs[0], int(ns[0].item()))
    got1 = P.poses_to_numpy(outs[1], int(ns[1].item()))
    assert got0.tobytes() == ref[1].tobytes() and got1.tobytes() == ref[0].tobytes()


def test_fp16_batch_pyramid_keeps_fp16_at_the_top_only():
    """An FP16 batch stores FP16 directions at its searched level only: the
    top level's field equals a single FP16 pyramid's bit for bit, the lower
    levels have none (null in tm_pyramid_level, TM_EINVAL on a field read),
    and their uint8 images are still there."""
    import ctypes

    P, sc, cfg, L = _c2(3)
    case("FP16 batch pyramid levels")
    img = torch.from_numpy(sc.image).cuda()
    model = P.Model(sc.model, L, cfg["tau_m"])
    b = P.Batch([model], [img], L, cfg["tau_s"], P.SearchParams(theta_step_top=cfg["theta_step_top"]),
                precision=P.TM_FP16)
    b.run()
    single = P.Pyramid(img, L, cfg["tau_s"], precision=P.TM_FP16)
    torch.cuda.synchronize()
    h = ctypes.c_void_p()
    assert P.lib().tm_batch_pyramid(b._h, 0, ctypes.byref(h)) == 0
    pyr = P.Pyramid.__new__(P.Pyramid)
    pyr._h, pyr.levels, pyr.precision = h, L, P.TM_FP16
    try:
        gi, gf = pyr.read(L - 1)
        si, sf = single.read(L - 1)
        torch.cuda.synchronize()
        assert torch.equal(gi, si) and gf.view(torch.int16).equal(sf.view(torch.int16))
        for l in range(L - 1):
            w, hh, prec = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            a, f = ctypes.c_void_p(), ctypes.c_void_p(1)
            assert P.lib().tm_pyramid_level(h, l, ctypes.byref(w), ctypes.byref(hh), ctypes.byref(a), ctypes.byref(f),
                                            ctypes.byref(prec)) == 0
            assert a.value and not f.value
            with pytest.raises(P.TMError) as e:
                pyr.read(l)
            assert e.value.status == P.tm.TM_EINVAL
            im = torch.empty((hh.value, w.value), dtype=torch.uint8, device="cuda")
            assert P.lib().tm_pyramid_read(h, l, ctypes.c_void_p(im.data_ptr()), None, None) == 0
            torch.cuda.synchronize()
            assert torch.equal(im, single.read(l)[0])
    finally:
        pyr._h = ctypes.c_void_p()  # owned by the batch
        single.free()
