"""Plain FP64 CPU oracle of the detector (arXiv 2112.05576, Sec. II).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users; the HIP library never imports it and it
never imports the HIP library.  The loops live in ``tm_oracle.c`` (compiled
with ``-ffp-contract=off``); this module composes them in the paper's order:
edge extraction, pyramid, then the search from the top image down (Sec. II,
para. 2), scoring with Eq. (1) under the rigid projection of Eq. (2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP for the row loop)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.orc_sobel.argtypes = [_u8p, ctypes.c_int, ctypes.c_int, _i32p, _i32p]
        L.orc_sobel.restype = None
        L.orc_edge_threshold.argtypes = [ctypes.c_double]
        L.orc_edge_threshold.restype = ctypes.c_int64
        L.orc_edge_field.argtypes = [_i32p, _i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _f64p]
        L.orc_edge_field.restype = ctypes.c_int
        L.orc_pyr_down.argtypes = [_u8p, ctypes.c_int, ctypes.c_int, _u8p]
        L.orc_pyr_down.restype = None
        L.orc_model_points.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, _i32p, _f64p, ctypes.c_int]
        L.orc_model_points.restype = ctypes.c_int
        L.orc_level_step.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.orc_level_step.restype = ctypes.c_double
        L.orc_level_count.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_level_count.restype = ctypes.c_int
        L.orc_theta.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_theta.restype = ctypes.c_double
        L.orc_angle_index.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_angle_index.restype = ctypes.c_int
        L.orc_sincos_deg.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        L.orc_sincos_deg.restype = None
        L.orc_rotate.argtypes = [ctypes.c_int, _i32p, _f64p, ctypes.c_double, _i32p, _f64p]
        L.orc_rotate.restype = None
        L.orc_score.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.orc_score.restype = None
        L.orc_top_map.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, _f64p, _f64p, _i32p, ctypes.c_int]
        L.orc_top_map.restype = None
        L.orc_select.argtypes = [_f64p, _f64p, _i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_float,
                                 ctypes.c_int, _i32p, _i32p, _i32p, _f64p, _f64p]
        L.orc_select.restype = ctypes.c_int
        L.orc_refine_level.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i32p, _f64p, _f64p]
        L.orc_refine_level.restype = None
        L.orc_final.argtypes = [ctypes.c_int, _i32p, _i32p, _i32p, _f64p, _f64p, ctypes.c_double,
                                ctypes.c_float, ctypes.c_int]
        L.orc_final.restype = ctypes.c_int
        L.orc_cont_score.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _f64p]
        L.orc_cont_score.restype = None
        L.orc_project.argtypes = [ctypes.c_int, _i32p, _f64p, ctypes.c_double, ctypes.c_double, _i32p, _f64p]
        L.orc_project.restype = None
        L.orc_scale.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_scale.restype = ctypes.c_double
        L.orc_top_map_sim.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _f64p, _f64p, _i32p, ctypes.c_int]
        L.orc_top_map_sim.restype = None
        L.orc_refine_level_sim.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, _i32p, _i32p, _i32p, _f64p, _f64p]
        L.orc_refine_level_sim.restype = None
        L.orc_grad_down.argtypes = [_i32p, _i32p, ctypes.c_int, ctypes.c_int, _i32p, _i32p]
        L.orc_grad_down.restype = None
        _lib = L
    return _lib


def default_threads() -> int:
    """Threads for the exhaustive-search row loop (the host's usable cores)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


# ------------------------------------------------------------- parameters
@dataclass
class PyrParams:
    """Pyramid parameters of Sec. II para. 2: number of levels and the edge
    (gradient magnitude) threshold, on the scale of the integer Sobel."""
    levels: int = 1
    edge_thresh: float = 30.0
    # "grey": pyramid of the grey image, edges per level (O3); "gradient": the
    # pyramid of the full image's Sobel gradients (O17)
    source: str = "grey"


@dataclass
class SearchParams:
    """Search parameters of Sec. II para. 2: step sizes in x, y and theta,
    the angle range, the per-point neighbouring-search size (3 in the paper),
    and the candidate-selection settings of the multi-instance reading."""
    step_x: int = 1
    step_y: int = 1
    theta_min: float = 0.0
    theta_range: float = 360.0
    theta_step_top: float = 1.0
    neighbourhood: int = 3
    min_score: float = 0.5
    nms_min_dist: float = 0.0  # level-0 pixels; <= 0 selects 0.5 x model radius
    max_candidates: int = 32
    max_matches: int = 8
    # "all": every tap of the window votes, off-edge taps 0 (O7); "edge": edge
    # taps only, 0 for a window without one (O16)
    vote: str = "all"
    # similarity pose (O13-O15): scales scale_min + j * scale_step, j < scale_count
    scale_min: float = 1.0
    scale_step: float = 0.0
    scale_count: int = 1

    @property
    def similarity(self) -> bool:
        return self.scale_count > 1 or self.scale_min != 1.0

    @property
    def vote_mode(self) -> int:
        return _vote_mode(self.vote)


def _vote_mode(vote) -> int:
    if vote in ("all", 0):
        return 0
    if vote in ("edge", 1):
        return 1
    raise ValueError(f"vote must be 'all' or 'edge', got {vote!r}")


# ------------------------------------------------------------- O1 .. O4
def sobel(img: np.ndarray):
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    gx = np.empty((H, W), np.int32)
    gy = np.empty((H, W), np.int32)
    lib().orc_sobel(img, W, H, gx, gy)
    return gx, gy


def edge_threshold(tau: float) -> int:
    return int(lib().orc_edge_threshold(float(np.float32(tau))))


def direction_field(gx: np.ndarray, gy: np.ndarray, tau: float) -> np.ndarray:
    """O2 on integer gradients: unit direction field (H, W, 2), zero off the edge set."""
    gx = np.ascontiguousarray(gx, np.int32)
    gy = np.ascontiguousarray(gy, np.int32)
    H, W = gx.shape
    g = np.empty((H, W, 2), np.float64)
    lib().orc_edge_field(gx, gy, W, H, edge_threshold(tau), g)
    return g


def edge_field(img: np.ndarray, tau: float) -> np.ndarray:
    """Unit direction field (H, W, 2), zero off the edge set (O1 + O2)."""
    return direction_field(*sobel(img), tau)


def grad_down(gx: np.ndarray, gy: np.ndarray):
    """O17: one step of the gradient-map pyramid (floored 2x2 means)."""
    gx = np.ascontiguousarray(gx, np.int32)
    gy = np.ascontiguousarray(gy, np.int32)
    H, W = gx.shape
    ox = np.empty((H // 2, W // 2), np.int32)
    oy = np.empty((H // 2, W // 2), np.int32)
    lib().orc_grad_down(gx, gy, W, H, ox, oy)
    return ox, oy


def gradient_pyramid(img: np.ndarray, levels: int):
    """O17: Sobel gradients of the full image, then their pyramid."""
    out = [sobel(img)]
    for _ in range(1, levels):
        out.append(grad_down(*out[-1]))
    return out


def pyr_down(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.empty((H // 2, W // 2), np.uint8)
    lib().orc_pyr_down(img, W, H, out)
    return out


def pyramid(img: np.ndarray, levels: int):
    """Grey-level pyramid; edges are then extracted on every level (O3)."""
    out = [np.ascontiguousarray(img, dtype=np.uint8)]
    for _ in range(1, levels):
        out.append(pyr_down(out[-1]))
    return out


def field_pyramid(img: np.ndarray, levels: int, tau: float, source: str = "grey"):
    """Direction field of every level: edges of each grey level (O3), or of
    each level of the gradient-map pyramid (O17)."""
    if source == "grey":
        return [edge_field(lv, tau) for lv in pyramid(img, levels)]
    if source == "gradient":
        return [direction_field(gx, gy, tau) for gx, gy in gradient_pyramid(img, levels)]
    raise ValueError(f"source must be 'grey' or 'gradient', got {source!r}")


@dataclass
class ModelLevel:
    t: np.ndarray  # (n, 2) int32, offsets from the integer centre
    d: np.ndarray  # (n, 2) float64, unit gradient directions
    width: int
    height: int


@dataclass
class Model:
    levels: list = field(default_factory=list)
    radius2: int = 0  # max |t|^2 at level 0

    @property
    def default_dmin(self) -> float:
        return float(np.float32(0.5 * np.sqrt(float(self.radius2))))


def model_points(g: np.ndarray):
    H, W, _ = g.shape
    cap = H * W
    t = np.empty((cap, 2), np.int32)
    d = np.empty((cap, 2), np.float64)
    n = lib().orc_model_points(np.ascontiguousarray(g), W, H, t, d, cap)
    return t[:n].copy(), d[:n].copy()


def build_model(img: np.ndarray, pp: PyrParams) -> Model:
    """O4: edge points of the model image on each pyramid level."""
    m = Model()
    for g in field_pyramid(img, pp.levels, pp.edge_thresh, pp.source):
        t, d = model_points(g)
        m.levels.append(ModelLevel(t, d, g.shape[1], g.shape[0]))
    t0 = m.levels[0].t.astype(np.int64)
    m.radius2 = int((t0 ** 2).sum(axis=1).max()) if len(t0) else 0
    return m


# ------------------------------------------------------------- O5, O6
def level_step(sp: SearchParams, L: int, l: int) -> float:
    return float(lib().orc_level_step(sp.theta_step_top, L, l))


def level_count(sp: SearchParams, step_l: float) -> int:
    return int(lib().orc_level_count(sp.theta_range, step_l))


def theta(theta_min: float, step_l: float, k: int) -> float:
    return float(lib().orc_theta(theta_min, step_l, k))


def sincos_deg(deg: float):
    c = ctypes.c_double()
    s = ctypes.c_double()
    lib().orc_sincos_deg(float(deg), ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def rotate(t: np.ndarray, d: np.ndarray, theta_deg: float):
    """Eq. (2) applied to the model points: (q, r) = (round(R t), R d)."""
    n = len(t)
    t = np.ascontiguousarray(t, np.int32)
    d = np.ascontiguousarray(d, np.float64)
    q = np.empty((n, 2), np.int32)
    r = np.empty((n, 2), np.float64)
    lib().orc_rotate(n, t, d, float(theta_deg), q, r)
    return q, r


def project(t: np.ndarray, d: np.ndarray, theta_deg: float, sigma: float):
    """O13, the similarity projection: (q, r) = (round(sigma R t), R d)."""
    n = len(t)
    t = np.ascontiguousarray(t, np.int32)
    d = np.ascontiguousarray(d, np.float64)
    q = np.empty((n, 2), np.int32)
    r = np.empty((n, 2), np.float64)
    lib().orc_project(n, t, d, float(theta_deg), float(sigma), q, r)
    return q, r


def scale(sigma_min: float, sigma_step: float, j: int) -> float:
    return float(lib().orc_scale(float(sigma_min), float(sigma_step), int(j)))


# ------------------------------------------------------------- O7, O8
def score(g: np.ndarray, t, d, ux: int, uy: int, theta_deg: float, win: int = 3, sigma: float = 1.0,
          vote="all"):
    """Eq. (1) at one pose (scale sigma: O13; vote "edge": O16): returns (S_w, S_1)."""
    H, W, _ = g.shape
    q, r = rotate(t, d, theta_deg) if sigma == 1.0 else project(t, d, theta_deg, sigma)
    sw = ctypes.c_double()
    s1 = ctypes.c_double()
    lib().orc_score(np.ascontiguousarray(g), W, H, len(t), q, r, int(ux), int(uy), int(win), _vote_mode(vote),
                    ctypes.byref(sw), ctypes.byref(s1))
    return sw.value, s1.value


def top_map(g: np.ndarray, t, d, theta_min: float, step: float, K: int, sx: int = 1, sy: int = 1,
            win: int = 3, nthreads: int | None = None, vote="all"):
    """O8: best (S_w, S_1, k) per translation of the step grid, shape (Gh, Gw)."""
    H, W, _ = g.shape
    Gw, Gh = (W + sx - 1) // sx, (H + sy - 1) // sy
    mw = np.empty((Gh, Gw), np.float64)
    m1 = np.empty((Gh, Gw), np.float64)
    mk = np.empty((Gh, Gw), np.int32)
    lib().orc_top_map(np.ascontiguousarray(g), W, H, len(t), np.ascontiguousarray(t, np.int32),
                      np.ascontiguousarray(d, np.float64), float(theta_min), float(step), int(K),
                      int(sx), int(sy), int(win), _vote_mode(vote), mw, m1, mk,
                      int(nthreads if nthreads else default_threads()))
    return mw, m1, mk


def top_map_sim(g: np.ndarray, t, d, theta_min: float, step: float, K: int, sigma_min: float, sigma_step: float,
                S: int, sx: int = 1, sy: int = 1, win: int = 3, nthreads: int | None = None, vote="all"):
    """O14: best (S_w, S_1, m = j K + k) per translation over angles and scales."""
    H, W, _ = g.shape
    Gw, Gh = (W + sx - 1) // sx, (H + sy - 1) // sy
    mw = np.empty((Gh, Gw), np.float64)
    m1 = np.empty((Gh, Gw), np.float64)
    mk = np.empty((Gh, Gw), np.int32)
    lib().orc_top_map_sim(np.ascontiguousarray(g), W, H, len(t), np.ascontiguousarray(t, np.int32),
                          np.ascontiguousarray(d, np.float64), float(theta_min), float(step), int(K),
                          float(sigma_min), float(sigma_step), int(S), int(sx), int(sy), int(win), _vote_mode(vote),
                          mw, m1, mk,
                          int(nthreads if nthreads else default_threads()))
    return mw, m1, mk


def cont_score(g: np.ndarray, t, d, ux: float, uy: float, theta_deg: float):
    """O12: continuous (bilinear) score and its gradient (d/dux, d/duy, d/dtheta_deg)."""
    H, W, _ = g.shape
    S = ctypes.c_double()
    grad = np.empty(3, np.float64)
    lib().orc_cont_score(np.ascontiguousarray(g), W, H, len(t), np.ascontiguousarray(t, np.int32),
                         np.ascontiguousarray(d, np.float64), float(ux), float(uy), float(theta_deg),
                         ctypes.byref(S), grad)
    return S.value, grad


# ------------------------------------------------------------- O9 .. O11
@dataclass
class Candidates:
    x: np.ndarray
    y: np.ndarray
    k: np.ndarray
    sw: np.ndarray
    s1: np.ndarray

    def __len__(self):
        return len(self.x)

    def rows(self):
        return [(int(self.x[i]), int(self.y[i]), int(self.k[i]), float(self.sw[i]), float(self.s1[i]))
                for i in range(len(self))]


def select(mw, m1, mk, sx: int, sy: int, level: int, min_score: float, dmin: float, max_out: int):
    """O9 on a score map: strict local maxima, key sort, greedy NMS."""
    Gh, Gw = mw.shape
    ox = np.empty(max_out, np.int32)
    oy = np.empty(max_out, np.int32)
    ok = np.empty(max_out, np.int32)
    ow = np.empty(max_out, np.float64)
    o1 = np.empty(max_out, np.float64)
    m = lib().orc_select(np.ascontiguousarray(mw, np.float64), np.ascontiguousarray(m1, np.float64),
                         np.ascontiguousarray(mk, np.int32), Gw, Gh, int(sx), int(sy), int(level),
                         float(min_score), float(np.float32(dmin)), int(max_out), ox, oy, ok, ow, o1)
    return Candidates(ox[:m].copy(), oy[:m].copy(), ok[:m].copy(), ow[:m].copy(), o1[:m].copy())


def refine_level(g, ml: ModelLevel, cand: Candidates, theta_min: float, step_l: float, K: int,
                 full: bool, win: int, vote="all") -> Candidates:
    """O10: one coarse-to-fine step (level l+1 -> l) of every candidate."""
    H, W, _ = g.shape
    c = Candidates(cand.x.astype(np.int32).copy(), cand.y.astype(np.int32).copy(),
                   cand.k.astype(np.int32).copy(), cand.sw.astype(np.float64).copy(),
                   cand.s1.astype(np.float64).copy())
    lib().orc_refine_level(np.ascontiguousarray(g), W, H, len(ml.t), ml.t, ml.d, float(theta_min),
                           float(step_l), int(K), int(bool(full)), int(win), _vote_mode(vote), len(c), c.x, c.y, c.k,
                           c.sw, c.s1)
    return c


def refine_level_sim(g, ml: ModelLevel, cand: Candidates, theta_min: float, step_l: float, K: int, K_above: int,
                     full: bool, win: int, sigma_min: float, sigma_step: float, vote="all") -> Candidates:
    """O15: one coarse-to-fine step at each candidate's scale; k holds m = j K + k."""
    H, W, _ = g.shape
    c = Candidates(cand.x.astype(np.int32).copy(), cand.y.astype(np.int32).copy(),
                   cand.k.astype(np.int32).copy(), cand.sw.astype(np.float64).copy(),
                   cand.s1.astype(np.float64).copy())
    lib().orc_refine_level_sim(np.ascontiguousarray(g), W, H, len(ml.t), ml.t, ml.d, float(theta_min),
                               float(step_l), int(K), int(K_above), int(bool(full)), int(win), _vote_mode(vote),
                               float(sigma_min),
                               float(sigma_step), len(c), c.x, c.y, c.k, c.sw, c.s1)
    return c


def final(cand: Candidates, min_score: float, dmin: float, max_out: int) -> Candidates:
    """O11: key sort, greedy NMS at level 0, score floor, at most max_out."""
    c = Candidates(cand.x.astype(np.int32).copy(), cand.y.astype(np.int32).copy(),
                   cand.k.astype(np.int32).copy(), cand.sw.astype(np.float64).copy(),
                   cand.s1.astype(np.float64).copy())
    m = lib().orc_final(len(c), c.x, c.y, c.k, c.sw, c.s1, float(min_score),
                        float(np.float32(dmin)), int(max_out))
    return Candidates(c.x[:m].copy(), c.y[:m].copy(), c.k[:m].copy(), c.sw[:m].copy(), c.s1[:m].copy())


@dataclass
class Detection:
    x: int
    y: int
    k: int
    theta: float
    sw: float
    s1: float
    j: int = 0          # scale index (similarity pose)
    scale: float = 1.0


@dataclass
class DetectTrace:
    """Every intermediate of one oracle detection, for parity tests."""
    fields: list
    model: Model
    top: tuple          # (mw, m1, mk) at the top level
    candidates: Candidates
    refined: list       # Candidates after each refinement level (top-1 ... 0)
    detections: list


def detect(search: np.ndarray, model_img: np.ndarray, pp_search: PyrParams, pp_model: PyrParams,
           sp: SearchParams, nthreads: int | None = None, model: Model | None = None,
           fields: list | None = None) -> DetectTrace:
    """O1-O11: full detection of one model in one search image."""
    L = pp_search.levels
    if model is None:
        model = build_model(model_img, PyrParams(L, pp_model.edge_thresh, pp_model.source))
    if fields is None:
        fields = field_pyramid(search, L, pp_search.edge_thresh, pp_search.source)
    full = sp.theta_range >= 360.0
    dmin = sp.nms_min_dist if sp.nms_min_dist > 0 else model.default_dmin
    top = L - 1
    step_top = level_step(sp, L, top)
    K_top = level_count(sp, step_top)
    ml = model.levels[top]
    if sp.similarity:
        mw, m1, mk = top_map_sim(fields[top], ml.t, ml.d, sp.theta_min, step_top, K_top, sp.scale_min,
                                 sp.scale_step, sp.scale_count, sp.step_x, sp.step_y, sp.neighbourhood, nthreads,
                                 sp.vote)
    else:
        mw, m1, mk = top_map(fields[top], ml.t, ml.d, sp.theta_min, step_top, K_top, sp.step_x, sp.step_y,
                             sp.neighbourhood, nthreads, sp.vote)
    cand = select(mw, m1, mk, sp.step_x, sp.step_y, top, sp.min_score, dmin, sp.max_candidates)
    refined = []
    cur = cand
    K_above = K_top
    for l in range(L - 2, -1, -1):
        step_l = level_step(sp, L, l)
        K_l = level_count(sp, step_l)
        if sp.similarity:
            cur = refine_level_sim(fields[l], model.levels[l], cur, sp.theta_min, step_l, K_l, K_above, full,
                                   sp.neighbourhood, sp.scale_min, sp.scale_step, sp.vote)
        else:
            cur = refine_level(fields[l], model.levels[l], cur, sp.theta_min, step_l, K_l, full,
                               sp.neighbourhood, sp.vote)
        K_above = K_l
        refined.append(cur)
    fin = final(cur, sp.min_score, dmin, sp.max_matches)
    step0 = level_step(sp, L, 0)
    K0 = level_count(sp, step0)
    dets = []
    for x, y, m, w, s in fin.rows():
        j, k = (m // K0, m % K0) if sp.similarity else (0, m)
        dets.append(Detection(int(x), int(y), int(k), theta(sp.theta_min, step0, int(k)), float(w), float(s),
                              j, scale(sp.scale_min, sp.scale_step, j) if sp.similarity else 1.0))
    return DetectTrace(fields, model, (mw, m1, mk), cand, refined, dets)
