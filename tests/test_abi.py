"""The C-ABI library loads, exports every entry point that include/tm.h
declares, and rejects invalid arguments before touching a device (these
calls need no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2112_05576_amd import tm

    if not os.path.exists(tm.LIB_PATH):
        from paper_2112_05576_amd import build

        build.build(verbose=False)
    return tm.lib()


def test_every_declared_symbol_is_exported(L):
    from paper_2112_05576_amd import tm

    names = _declared()
    assert len(names) >= 19
    out = subprocess.run(["nm", "-D", "--defined-only", tm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(tm_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)
    # nothing else leaks out of the C ABI
    assert exported == set(names)


def test_invalid_arguments_fail_before_the_device(L):
    from paper_2112_05576_amd import tm

    vp = ctypes.c_void_p
    out = vp()
    pp = tm.PyrParamsC(4, 30.0, tm.TM_FP32)
    assert L.tm_build_model(None, 64, 64, 64, ctypes.byref(pp), None, ctypes.byref(out)) == tm.TM_EINVAL
    assert b"null image" in L.tm_last_error()
    fake = vp(0x1000)  # never dereferenced: validation fails first
    bad = tm.PyrParamsC(0, 30.0, tm.TM_FP32)
    assert L.tm_build_pyramid(fake, 64, 64, 64, ctypes.byref(bad), None, ctypes.byref(out)) == tm.TM_EINVAL
    bad = tm.PyrParamsC(4, -1.0, tm.TM_FP32)
    assert L.tm_build_pyramid(fake, 64, 64, 64, ctypes.byref(bad), None, ctypes.byref(out)) == tm.TM_EINVAL
    bad = tm.PyrParamsC(4, 30.0, 7)
    assert L.tm_build_pyramid(fake, 64, 64, 64, ctypes.byref(bad), None, ctypes.byref(out)) == tm.TM_EINVAL
    bad = tm.PyrParamsC(4, 30.0, tm.TM_FP32, 2)  # neither pyramid source
    assert L.tm_build_pyramid(fake, 64, 64, 64, ctypes.byref(bad), None, ctypes.byref(out)) == tm.TM_EINVAL
    assert b"source" in L.tm_last_error()
    assert L.tm_build_model(fake, 64, 64, 64, ctypes.byref(bad), None, ctypes.byref(out)) == tm.TM_EINVAL
    assert L.tm_build_pyramid(fake, 64, 64, 32, ctypes.byref(pp), None, ctypes.byref(out)) == tm.TM_EINVAL
    # 4 levels need at least 3 * 2^3 = 24 pixels a side
    assert L.tm_build_pyramid(fake, 23, 64, 64, ctypes.byref(pp), None, ctypes.byref(out)) == tm.TM_EINVAL
    assert b"too small" in L.tm_last_error()
    sp = tm.SearchParams().c()
    assert L.tm_detect(None, None, ctypes.byref(sp), fake, 8, fake, None) == tm.TM_EINVAL
    assert L.tm_select(None, None, None, 4, 4, 1, 1, 0, 0.5, 1.0, None, 8, None, None) == tm.TM_EINVAL
    assert L.tm_select(fake, fake, fake, 4, 4, 1, 1, 0, 0.5, 1.0, fake, 0, fake, None) == tm.TM_EINVAL
    assert L.tm_select(fake, fake, fake, 4, 4, 0, 1, 0, 0.5, 1.0, fake, 8, fake, None) == tm.TM_EINVAL
    assert L.tm_refine(None, None, ctypes.byref(sp), 3, fake, 1, None) == tm.TM_EINVAL
    assert L.tm_score_poses(None, None, 0, 3, 0, fake, 1, fake, None) == tm.TM_EINVAL
    assert L.tm_model_level_info(None, 0, None, None, None) == tm.TM_EINVAL
    assert L.tm_pyramid_read(None, 0, None, None, None) == tm.TM_EINVAL
    L.tm_model_free(None)
    L.tm_pyramid_free(None)


def test_continuous_and_batch_entries_validate_first(L):
    """The continuous score, batch and graph entries reject null handles,
    negative counts and bad step-length lists before any device call."""
    from paper_2112_05576_amd import tm

    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: validation fails first
    al = (ctypes.c_double * 3)(0.0, 0.5, 1.0)
    assert L.tm_cont_score(None, None, 0, fake, 1, fake, None) == tm.TM_EINVAL
    assert L.tm_cont_score(fake, fake, 0, fake, -1, fake, None) == tm.TM_EINVAL
    assert L.tm_cont_score(fake, fake, 0, None, 1, fake, None) == tm.TM_EINVAL
    assert L.tm_cont_score_backward(fake, fake, 0, fake, 1, None, None, None) == tm.TM_EINVAL
    assert L.tm_cont_line_search(fake, fake, 0, fake, fake, 1, al, 0, None, None) == tm.TM_EINVAL
    assert b"step lengths" in L.tm_last_error()
    assert L.tm_cont_line_search(fake, fake, 0, fake, fake, 1, al, 17, None, None) == tm.TM_EINVAL
    bad = (ctypes.c_double * 2)(0.0, float("nan"))
    assert L.tm_cont_line_search(fake, fake, 0, fake, fake, 1, bad, 2, None, None) == tm.TM_EINVAL
    assert b"non-finite" in L.tm_last_error()
    assert L.tm_batch_run(None, None) == tm.TM_EINVAL
    assert L.tm_batch_run_graph(None, None) == tm.TM_EINVAL
    assert L.tm_batch_tune(None, None, 3, None, None, None, None, None, None) == tm.TM_EINVAL
    assert L.tm_batch_set_form(None, 4, 4, 0) == tm.TM_EINVAL
    assert L.tm_batch_search_launch(None, None, None) == tm.TM_EINVAL
    assert L.tm_batch_cont_score(None, 0, fake, 1, fake, None) == tm.TM_EINVAL
    assert L.tm_batch_cont_score_backward(None, 0, fake, 1, None, fake, None) == tm.TM_EINVAL
    assert L.tm_batch_cont_line_search(None, 0, fake, fake, 1, al, 3, None, None) == tm.TM_EINVAL
    out = vp()
    pp = tm.PyrParamsC(4, 30.0, tm.TM_FP32)
    sp = tm.SearchParams().c()
    one = (ctypes.c_int32 * 1)(64)
    ptrs = (vp * 1)(fake)
    assert L.tm_batch_create(ptrs, 0, ptrs, one, one, one, 1, ctypes.byref(pp), ctypes.byref(sp), fake, 8, fake, None,
                             ctypes.byref(out)) == tm.TM_EINVAL
    assert L.tm_batch_create(ptrs, 1, ptrs, one, one, one, 1, ctypes.byref(pp), ctypes.byref(sp), fake, 0, fake, None,
                             ctypes.byref(out)) == tm.TM_EINVAL
    assert L.tm_batch_create(ptrs, 1, ptrs, one, one, one, 1, ctypes.byref(pp), ctypes.byref(sp), None, 8, fake,
                             None, ctypes.byref(out)) == tm.TM_EINVAL
    badv = tm.SearchParams(vote=2).c()  # neither window reading
    assert L.tm_batch_create(ptrs, 1, ptrs, one, one, one, 1, ctypes.byref(pp), ctypes.byref(badv), fake, 8, fake,
                             None, ctypes.byref(out)) == tm.TM_EINVAL
    assert b"vote" in L.tm_last_error()
    assert not out.value
    L.tm_batch_free(None)


def test_search_params_validation(L):
    """Search parameters are checked before the handles are used."""
    from paper_2112_05576_amd import tm
    import ctypes as C

    # tm_detect validates the pair first, so use tm_score_map's order: pair, then params.
    # A fake model/pyramid pair cannot be built without a device; check the
    # parameter checker through a null pair, which must still name the pair.
    sp = tm.SearchParams(neighbourhood=2).c()
    assert L.tm_detect(None, None, C.byref(sp), None, 1, None, None) == tm.TM_EINVAL
    assert L.tm_timing_enable(0) == tm.TM_OK
    ms, n = C.c_double(), C.c_int32()
    assert L.tm_timing_read(C.byref(ms), C.byref(n)) == tm.TM_OK and n.value == 0


def test_allocator_registration_is_validated(L):
    from paper_2112_05576_amd import tm

    half = tm.AllocatorC(tm._ALLOC_FN(lambda n, c, s: None), tm._FREE_FN(), None)  # alloc without free
    assert L.tm_set_allocator(ctypes.byref(half)) == tm.TM_EINVAL
    assert b"alloc and free" in L.tm_last_error()
    assert L.tm_set_allocator(None) == tm.TM_OK  # back to hipMalloc / hipFree


def test_capacity_count_maps_to_ecapacity():
    """A count above the caller's capacity is the TM_ECAPACITY case: the
    binding raises it with the truncated result attached."""
    import numpy as np

    from paper_2112_05576_amd import tm

    poses = np.zeros(2, tm.POSE_DTYPE)
    assert tm.check_count(2, 2, poses) is poses
    with pytest.raises(tm.TMError) as e:
        tm.check_count(5, 2, poses)
    assert e.value.status == tm.TM_ECAPACITY and e.value.poses is poses
