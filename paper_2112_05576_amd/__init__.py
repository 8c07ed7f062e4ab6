"""MI355X (gfx950) edge-orientation template matcher: the detector of
Le & Lin, arXiv 2112.05576 (Sec. II), as hand-written HIP kernels behind the
C ABI of include/tm.h.  This package holds the HIP sources (csrc/), the
in-tree build (build.py -> lib/libtm.so) and the ctypes binding (tm.py)."""
from .tm import (  # noqa: F401
    EVAL_DTYPE,
    POSE_DTYPE,
    TM_FP16,
    TM_FP32,
    Batch,
    ContinuousScore,
    cont_line_search,
    cont_score,
    cont_score_backward,
    refine_continuous,
    Model,
    Pyramid,
    SearchParams,
    TMError,
    detect,
    detect_async,
    lib,
    poses_to_numpy,
    refine,
    score_map,
    score_poses,
    select,
    timing_enable,
    timing_read,
    version,
)
