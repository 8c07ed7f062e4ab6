"""tm_detect_static, the detection for callers that cannot allocate: its
results equal tm_detect's bit for bit on two calls in a row (a 640x480
four-level detection, then a smaller 128x128 one-level detection with another
model), in FP32 and FP16; it calls no allocator (a counting allocator
registered for the handles sees tm_detect grow the pyramid's workspace and
tm_detect_static take nothing); a detection needing more scratch than the
static array holds is refused with TM_ECAPACITY before anything runs."""
import ctypes

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


def _run(P, fn, gm, pyr, sp, cap):
    out = torch.full((cap, P.tm.POSE_WORDS), -1, dtype=torch.int32, device="cuda")
    n = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    fn(gm, pyr, sp, out, n)
    torch.cuda.synchronize()
    m = int(n.item())
    return m, P.poses_to_numpy(out, min(m, cap)).copy()


@pytest.mark.parametrize("precision", [0, 1])
def test_static_detection_equals_detect(precision):
    import paper_2112_05576_amd as P

    for ci in (2, 1):  # the second call: a smaller image and another model
        sc = synth.scene_for_config(ci, 0)
        cfg = sc.config
        L = cfg["levels"]
        case(f"tm_detect_static C{ci} precision={precision}")
        gm = P.Model(sc.model, L, cfg["tau_m"])
        pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=precision)
        sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
        ref = _run(P, P.detect_async, gm, pyr, sp, sp.max_matches)
        got = _run(P, P.detect_static_async, gm, pyr, sp, sp.max_matches)
        assert ref[0] >= 1
        assert got[0] == ref[0] and got[1].tobytes() == ref[1].tobytes()
        # a capacity below the count: the same truncation and count as tm_detect
        if ref[0] >= 2:
            r1 = _run(P, P.detect_async, gm, pyr, sp, 1)
            g1 = _run(P, P.detect_static_async, gm, pyr, sp, 1)
            assert g1[0] == r1[0] == ref[0] and g1[1].tobytes() == r1[1].tobytes()


def test_static_detection_calls_no_allocator():
    import paper_2112_05576_amd as P
    from paper_2112_05576_amd import tm

    calls = []

    def alloc(nbytes, ctx, stream):
        calls.append(int(nbytes))
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))

    def free(ptr, ctx, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = tm.AllocatorC(tm._ALLOC_FN(alloc), tm._FREE_FN(free), None)
    sc = synth.scene_for_config(2, 1)
    cfg = sc.config
    L = cfg["levels"]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    case("tm_detect_static allocates nothing")
    assert P.lib().tm_set_allocator(ctypes.byref(a)) == 0
    try:
        gm = P.Model(sc.model, L, cfg["tau_m"])
        pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
        built = len(calls)
        assert built >= 2  # the model's and the pyramid's memory came from the allocator
        got = _run(P, P.detect_static_async, gm, pyr, sp, sp.max_matches)
        got2 = _run(P, P.detect_static_async, gm, pyr, sp, sp.max_matches)
        assert len(calls) == built  # nothing allocated by the static detections
        ref = _run(P, P.detect_async, gm, pyr, sp, sp.max_matches)
        assert len(calls) > built  # tm_detect grew the pyramid's workspace and cached a table
        assert got[1].tobytes() == ref[1].tobytes() and got2[1].tobytes() == ref[1].tobytes()
        pyr.free()
        gm.free()
    finally:
        assert P.lib().tm_set_allocator(None) == 0


def test_static_detection_refuses_oversized():
    import paper_2112_05576_amd as P

    case("tm_detect_static over the static array")
    sc = synth.scene_for_config(1, 0)
    gm = P.Model(sc.model, 2, 30.0)
    img = torch.full((4096, 4096), 40, dtype=torch.uint8, device="cuda")
    pyr = P.Pyramid(img, 2, 30.0)  # top level 2048 x 2048: its selection scratch alone exceeds the array
    sp = P.SearchParams(theta_step_top=5.0)
    out = torch.full((8, P.tm.POSE_WORDS), -1, dtype=torch.int32, device="cuda")
    n = torch.full((1,), -5, dtype=torch.int32, device="cuda")
    with pytest.raises(P.TMError) as e:
        P.detect_static_async(gm, pyr, sp, out, n)
    assert e.value.status == P.TM_ECAPACITY and "static array" in str(e.value)
    torch.cuda.synchronize()
    assert int(n.item()) == -5 and int(out.min().item()) == -1  # nothing ran
