"""Python binding of the C ABI in include/tm.h (argument marshalling only).

Every computation runs in the HIP library ``lib/libtm.so``; torch supplies
device memory and the current stream.  Importing works without the library;
the first call that needs it raises ``TMError`` if it has not been built
(``python -m paper_2112_05576_amd.build``).  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libtm.so")

TM_OK, TM_EINVAL, TM_ENOMEM, TM_EDEVICE, TM_ECAPACITY = 0, -1, -2, -3, -4
TM_FP32, TM_FP16 = 0, 1
TM_PYR_GREY, TM_PYR_GRADIENT = 0, 1
TM_VOTE_ALL, TM_VOTE_EDGE = 0, 1
MAX_LEVELS = 8


class TMError(RuntimeError):
    def __init__(self, status: int, msg: str, poses=None):
        super().__init__(f"tm status {status}: {msg}")
        self.status = status
        self.poses = poses  # TM_ECAPACITY: the truncated result (the best `capacity` by key)


class AllocatorC(ctypes.Structure):
    pass


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
AllocatorC._fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class PyrParamsC(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("edge_thresh", ctypes.c_float), ("precision", ctypes.c_int32),
                ("source", ctypes.c_int32)]


class SearchParamsC(ctypes.Structure):
    _fields_ = [("step_x", ctypes.c_int32), ("step_y", ctypes.c_int32), ("theta_min_deg", ctypes.c_double),
                ("theta_range_deg", ctypes.c_double), ("theta_step_top_deg", ctypes.c_double),
                ("neighbourhood", ctypes.c_int32), ("min_score", ctypes.c_float), ("nms_min_dist", ctypes.c_float),
                ("max_candidates", ctypes.c_int32), ("max_matches", ctypes.c_int32), ("scale_min", ctypes.c_double),
                ("scale_step", ctypes.c_double), ("scale_count", ctypes.c_int32), ("vote", ctypes.c_int32)]


# tm_pose: x, y, k, level (int32), theta_deg, score_w, score_1 (float32), j (scale index)
POSE_WORDS = 8
POSE_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("k", "<i4"), ("level", "<i4"), ("theta", "<f4"),
                       ("sw", "<f4"), ("s1", "<f4"), ("j", "<i4")])
EVAL_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("theta", "<f8")])

_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


def lib():
    """The loaded C library; raises TMError if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TMError(TM_EDEVICE, f"HIP library not built: {LIB_PATH} (run paper_2112_05576_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "tm_build_model": [_vp, _i32, _i32, _i32, ctypes.POINTER(PyrParamsC), _vp, ctypes.POINTER(_vp)],
            "tm_build_pyramid": [_vp, _i32, _i32, _i32, ctypes.POINTER(PyrParamsC), _vp, ctypes.POINTER(_vp)],
            "tm_update_pyramid": [_vp, _vp, _i32, _vp],
            "tm_score_poses": [_vp, _vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp],
            "tm_score_map": [_vp, _vp, _i32, ctypes.POINTER(SearchParamsC), _vp, _vp, _vp, _vp],
            "tm_select": [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, ctypes.c_float, ctypes.c_float, _vp, _i32,
                          _vp, _vp],
            "tm_detect": [_vp, _vp, ctypes.POINTER(SearchParamsC), _vp, _i32, _vp, _vp],
            "tm_detect_static": [_vp, _vp, ctypes.POINTER(SearchParamsC), _vp, _i32, _vp, _vp],
            "tm_refine": [_vp, _vp, ctypes.POINTER(SearchParamsC), _i32, _vp, _i32, _vp],
            "tm_model_level_info": [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
            "tm_model_points": [_vp, _i32, _vp, _vp, _vp],
            "tm_model_table": [_vp, _i32, ctypes.c_double, ctypes.c_double, _i32, _vp, _vp, _vp],
            "tm_pyramid_level": [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), ctypes.POINTER(_i32)],
            "tm_pyramid_read": [_vp, _i32, _vp, _vp, _vp],
            "tm_timing_enable": [_i32],
            "tm_batch_create": [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), ctypes.POINTER(_i32),
                                ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32, ctypes.POINTER(PyrParamsC),
                                ctypes.POINTER(SearchParamsC), _vp, _i32, _vp, _vp, ctypes.POINTER(_vp)],
            "tm_batch_run": [_vp, _vp],
            "tm_batch_run_graph": [_vp, _vp],
            "tm_batch_tune": [_vp, _vp, _i32, _vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                              ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)],
            "tm_batch_search_form": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
            "tm_batch_search_launch": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
            "tm_batch_set_form": [_vp, _i32, _i32, _i32],
            "tm_batch_cont_score": [_vp, _i32, _vp, _i32, _vp, _vp],
            "tm_batch_cont_score_backward": [_vp, _i32, _vp, _i32, _vp, _vp, _vp],
            "tm_batch_cont_line_search": [_vp, _i32, _vp, _vp, _i32, ctypes.POINTER(ctypes.c_double), _i32, _vp, _vp],
            "tm_cont_score": [_vp, _vp, _i32, _vp, _i32, _vp, _vp],
            "tm_cont_score_backward": [_vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp],
            "tm_cont_line_search": [_vp, _vp, _i32, _vp, _vp, _i32, ctypes.POINTER(ctypes.c_double), _i32, _vp,
                                    _vp],
            "tm_batch_pyramid": [_vp, _i32, ctypes.POINTER(_vp)],
            "tm_timing_read": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)],
            "tm_set_allocator": [ctypes.POINTER(AllocatorC)],
            "tm_probe": [_i32, _i32, _vp, ctypes.c_int64, _vp, ctypes.POINTER(ctypes.c_double)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.tm_model_free.argtypes = [_vp]
        L.tm_model_free.restype = None
        L.tm_pyramid_free.argtypes = [_vp]
        L.tm_pyramid_free.restype = None
        L.tm_batch_free.argtypes = [_vp]
        L.tm_batch_free.restype = None
        L.tm_last_error.restype = ctypes.c_char_p
        L.tm_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st: int):
    if st != TM_OK:
        raise TMError(st, lib().tm_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_u8(img) -> torch.Tensor:
    if isinstance(img, np.ndarray):
        img = torch.from_numpy(np.ascontiguousarray(img, dtype=np.uint8))
    if img.dtype != torch.uint8 or img.dim() != 2:
        raise TMError(TM_EINVAL, "image must be a 2-D uint8 array")
    if not img.is_cuda:
        img = img.cuda()
    if img.stride(1) != 1:
        img = img.contiguous()
    return img


@dataclass
class SearchParams:
    """Search settings (see tm_search_params in include/tm.h)."""
    step_x: int = 1
    step_y: int = 1
    theta_min: float = 0.0
    theta_range: float = 360.0
    theta_step_top: float = 1.0
    neighbourhood: int = 3
    min_score: float = 0.5
    nms_min_dist: float = 0.0
    max_candidates: int = 32
    max_matches: int = 8
    scale_min: float = 1.0     # similarity pose: scales scale_min + j * scale_step, j < scale_count
    scale_step: float = 0.0
    scale_count: int = 1
    vote: int = 0              # TM_VOTE_ALL, or TM_VOTE_EDGE: only edge taps of a window vote

    def c(self) -> SearchParamsC:
        return SearchParamsC(self.step_x, self.step_y, self.theta_min, self.theta_range, self.theta_step_top,
                             self.neighbourhood, self.min_score, self.nms_min_dist, self.max_candidates,
                             self.max_matches, self.scale_min, self.scale_step, self.scale_count, self.vote)

    def scale(self, j: int) -> float:
        return self.scale_min + j * self.scale_step


class Model:
    """Edge-point model of a template image on every pyramid level."""

    def __init__(self, img, levels: int, edge_thresh: float, stream=None, source: int = 0):
        img = _dev_u8(img)
        self._h = _vp()
        p = PyrParamsC(levels, edge_thresh, TM_FP32, source)
        H, W = img.shape
        _check(lib().tm_build_model(_vp(img.data_ptr()), W, H, img.stride(0), ctypes.byref(p),
                                    _vp(_stream(stream)), ctypes.byref(self._h)))
        self.levels = levels

    @property
    def handle(self):
        return self._h

    def level_info(self, level: int):
        w, h, n = _i32(), _i32(), _i32()
        _check(lib().tm_model_level_info(self._h, level, ctypes.byref(w), ctypes.byref(h), ctypes.byref(n)))
        return w.value, h.value, n.value

    def points(self, level: int, stream=None):
        n = self.level_info(level)[2]
        t = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        g = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        _check(lib().tm_model_points(self._h, level, _vp(t.data_ptr()), _vp(g.data_ptr()), _vp(_stream(stream))))
        return t, g

    def table(self, level: int, theta_min: float, step: float, K: int, stream=None):
        n = self.level_info(level)[2]
        q = torch.empty((K, n, 2), dtype=torch.int32, device="cuda")
        r = torch.empty((K, n, 2), dtype=torch.float32, device="cuda")
        _check(lib().tm_model_table(self._h, level, theta_min, step, K, _vp(q.data_ptr()), _vp(r.data_ptr()),
                                    _vp(_stream(stream))))
        return q, r

    def free(self):
        if self._h:
            lib().tm_model_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Pyramid:
    """Grey-level pyramid and unit-direction field of a search image."""

    def __init__(self, img, levels: int, edge_thresh: float, precision: int = TM_FP32, stream=None,
                 source: int = 0):
        img = _dev_u8(img)
        self._h = _vp()
        p = PyrParamsC(levels, edge_thresh, precision, source)
        H, W = img.shape
        _check(lib().tm_build_pyramid(_vp(img.data_ptr()), W, H, img.stride(0), ctypes.byref(p),
                                      _vp(_stream(stream)), ctypes.byref(self._h)))
        self.levels = levels
        self.precision = precision
        self.shape = (H, W)

    @property
    def handle(self):
        return self._h

    def update(self, img, stream=None):
        img = _dev_u8(img)
        _check(lib().tm_update_pyramid(self._h, _vp(img.data_ptr()), img.stride(0), _vp(_stream(stream))))

    def level_shape(self, level: int):
        w, h, prec = _i32(), _i32(), _i32()
        a, b = _vp(), _vp()
        _check(lib().tm_pyramid_level(self._h, level, ctypes.byref(w), ctypes.byref(h), ctypes.byref(a),
                                      ctypes.byref(b), ctypes.byref(prec)))
        return h.value, w.value

    def read(self, level: int, stream=None):
        """(uint8 image, direction field as float32 (H, W, 2)) of a level."""
        H, W = self.level_shape(level)
        img = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        dt = torch.float16 if self.precision == TM_FP16 else torch.float32
        fld = torch.empty((H, W, 2), dtype=dt, device="cuda")
        _check(lib().tm_pyramid_read(self._h, level, _vp(img.data_ptr()), _vp(fld.data_ptr()),
                                     _vp(_stream(stream))))
        return img, fld

    def free(self):
        if self._h:
            lib().tm_pyramid_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def poses_to_numpy(t: torch.Tensor, n: int | None = None) -> np.ndarray:
    a = t.detach().cpu().numpy().view(POSE_DTYPE).reshape(-1)
    return a if n is None else a[:n]


def score_poses(model: Model, pyr: Pyramid, level: int, x, y, theta, neighbourhood: int = 3, stream=None,
                vote: int = 0):
    """S_w and S_1 (float32 tensor (n, 2)) of integer translations x, y and angles theta (degrees)."""
    ep = np.zeros(len(x), EVAL_DTYPE)
    ep["x"] = np.asarray(x, np.int32)
    ep["y"] = np.asarray(y, np.int32)
    ep["theta"] = np.asarray(theta, np.float64)
    dev = torch.from_numpy(ep.view(np.uint8)).cuda()
    out = torch.empty((len(ep), 2), dtype=torch.float32, device="cuda")
    _check(lib().tm_score_poses(model.handle, pyr.handle, level, neighbourhood, vote, _vp(dev.data_ptr()), len(ep),
                                _vp(out.data_ptr()), _vp(_stream(stream))))
    return out


def score_map(model: Model, pyr: Pyramid, level: int, sp: SearchParams, stream=None):
    """Best (S_w, S_1, k) per translation of the level's step grid."""
    H, W = pyr.level_shape(level)
    gh, gw = (H + sp.step_y - 1) // sp.step_y, (W + sp.step_x - 1) // sp.step_x
    sw = torch.empty((gh, gw), dtype=torch.float32, device="cuda")
    s1 = torch.empty((gh, gw), dtype=torch.float32, device="cuda")
    k = torch.empty((gh, gw), dtype=torch.int32, device="cuda")
    c = sp.c()
    _check(lib().tm_score_map(model.handle, pyr.handle, level, ctypes.byref(c), _vp(sw.data_ptr()),
                              _vp(s1.data_ptr()), _vp(k.data_ptr()), _vp(_stream(stream))))
    return sw, s1, k


def select(sw: torch.Tensor, s1: torch.Tensor, k: torch.Tensor, sx: int, sy: int, level: int, min_score: float,
           dmin: float, capacity: int, stream=None):
    """Candidate selection on a map; returns (poses int32 tensor (capacity, 8), count tensor)."""
    sw, s1, k = sw.contiguous(), s1.contiguous(), k.contiguous().to(torch.int32)
    gh, gw = sw.shape
    out = torch.empty((capacity, POSE_WORDS), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    _check(lib().tm_select(_vp(sw.data_ptr()), _vp(s1.data_ptr()), _vp(k.data_ptr()), gw, gh, sx, sy, level,
                           min_score, dmin, _vp(out.data_ptr()), capacity, _vp(n.data_ptr()), _vp(_stream(stream))))
    return out, n


def detect_async(model: Model, pyr: Pyramid, sp: SearchParams, out: torch.Tensor, n_out: torch.Tensor,
                 stream=None):
    """Enqueue a detection writing into caller buffers (no synchronisation)."""
    c = sp.c()
    _check(lib().tm_detect(model.handle, pyr.handle, ctypes.byref(c), _vp(out.data_ptr()), out.shape[0],
                           _vp(n_out.data_ptr()), _vp(_stream(stream))))


def check_count(n: int, capacity: int, poses: np.ndarray | None = None) -> np.ndarray | None:
    """TM_ECAPACITY when a call produced more poses than its buffer holds
    (the count the library wrote exceeds the capacity); `poses` (the
    truncated result) rides on the error."""
    if n > capacity:
        raise TMError(TM_ECAPACITY, f"{n} poses found, capacity {capacity}: the best {capacity} by key were kept",
                      poses)
    return poses


def detect_static_async(model: Model, pyr: Pyramid, sp: SearchParams, out: torch.Tensor, n_out: torch.Tensor,
                        stream=None):
    """As detect_async, through tm_detect_static: the detection's scratch
    in the library's static device array, nothing allocated."""
    c = sp.c()
    _check(lib().tm_detect_static(model.handle, pyr.handle, ctypes.byref(c), _vp(out.data_ptr()), out.shape[0],
                                  _vp(n_out.data_ptr()), _vp(_stream(stream))))


def detect(model: Model, pyr: Pyramid, sp: SearchParams, capacity: int | None = None, stream=None) -> np.ndarray:
    """Detections at level 0 as a numpy structured array (POSE_DTYPE);
    TMError(TM_ECAPACITY) if there were more than `capacity`."""
    cap = capacity or sp.max_matches
    out = torch.empty((cap, POSE_WORDS), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    detect_async(model, pyr, sp, out, n, stream)
    m = int(n.item())
    return check_count(m, cap, poses_to_numpy(out, min(m, cap)))


def refine(model: Model, pyr: Pyramid, sp: SearchParams, poses: np.ndarray, from_level: int,
           stream=None) -> np.ndarray:
    """Refine poses (POSE_DTYPE) of level `from_level` down to level 0."""
    a = np.ascontiguousarray(poses, dtype=POSE_DTYPE)
    dev = torch.from_numpy(a.view(np.int32).reshape(-1, POSE_WORDS).copy()).cuda()
    c = sp.c()
    _check(lib().tm_refine(model.handle, pyr.handle, ctypes.byref(c), from_level, _vp(dev.data_ptr()), len(a),
                           _vp(_stream(stream))))
    return poses_to_numpy(dev)


class Batch:
    """Every model against every image in one enqueue (tm_batch_run).  The
    images (2-D uint8 device tensors) stay bound: write new contents into the
    same tensors and run again.  Results: `out` (pairs, capacity, 8) int32 and
    `n_out` (pairs,), pair = image * n_models + model."""

    def __init__(self, models, images, levels: int, edge_thresh: float, sp: SearchParams,
                 precision: int = TM_FP32, capacity: int | None = None, stream=None, source: int = 0):
        self.images = [_dev_u8(im) for im in images]
        self.models = list(models)
        self.capacity = capacity or sp.max_matches
        npairs = len(self.images) * len(self.models)
        self.out = torch.empty((npairs, self.capacity, POSE_WORDS), dtype=torch.int32, device="cuda")
        self.n_out = torch.zeros((npairs,), dtype=torch.int32, device="cuda")
        nm, ni = len(self.models), len(self.images)
        mh = (_vp * nm)(*[m.handle for m in self.models])
        ih = (_vp * ni)(*[im.data_ptr() for im in self.images])
        ws = (_i32 * ni)(*[im.shape[1] for im in self.images])
        hs = (_i32 * ni)(*[im.shape[0] for im in self.images])
        ps = (_i32 * ni)(*[im.stride(0) for im in self.images])
        pp = PyrParamsC(levels, edge_thresh, precision, source)
        c = sp.c()
        self._h = _vp()
        _check(lib().tm_batch_create(mh, nm, ih, ws, hs, ps, ni, ctypes.byref(pp), ctypes.byref(c),
                                     _vp(self.out.data_ptr()), self.capacity, _vp(self.n_out.data_ptr()),
                                     _vp(_stream(stream)), ctypes.byref(self._h)))
        self.n_models = nm

    def run(self, stream=None, graph: bool = False):
        """Enqueue the batch; graph=True launches it as one captured HIP graph."""
        f = lib().tm_batch_run_graph if graph else lib().tm_batch_run
        _check(f(self._h, _vp(_stream(stream))))

    @property
    def handle(self):
        return self._h

    def tune(self, iterations: int = 3, stream=None, partner: "Batch | None" = None, partner_stream=None) -> dict:
        """Autotune the search's schedule (variant, waves per chunk, angles per
        chunk) on the bound images and keep the fastest (results are
        bit-identical whichever runs).  With a partner batch of the same
        shape on its own stream, the chunkings are timed on the pipelined
        step of the two and both keep the choice."""
        v, w, c, us = _i32(), _i32(), _i32(), ctypes.c_float()
        ph = partner.handle if partner is not None else None
        ps = _vp(_stream(partner_stream)) if partner is not None else None
        _check(lib().tm_batch_tune(self._h, ph, iterations, _vp(_stream(stream)), ps, ctypes.byref(v), ctypes.byref(w),
                                   ctypes.byref(c), ctypes.byref(us)))
        return {"variant": v.value, "waves_per_chunk": w.value, "chunk_angles": c.value,
                ("step_us" if partner is not None else "search_us"): us.value}

    def set_form(self, variant: int, waves_per_chunk: int, chunk_angles: int = 0):
        """Use this search schedule (e.g. another batch's tuned one) from now on
        (chunk_angles 0: keep the chunking)."""
        _check(lib().tm_batch_set_form(self._h, int(variant), int(waves_per_chunk), int(chunk_angles)))

    def search_form(self) -> dict:
        """The search schedule in use: variant, waves sharing a chunk, angles per chunk."""
        v, w, c = _i32(), _i32(), _i32()
        _check(lib().tm_batch_search_form(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(c)))
        return {"variant": v.value, "waves_per_chunk": w.value, "chunk_angles": c.value}

    def search_launch(self) -> dict:
        """Launch shape of the search kernel in the current schedule."""
        g, t = _i32(), _i32()
        _check(lib().tm_batch_search_launch(self._h, ctypes.byref(g), ctypes.byref(t)))
        return {"workgroups": g.value, "threads": t.value}

    def cont_score(self, level: int, poses: torch.Tensor, pairs, stream=None) -> torch.Tensor:
        """S_c of (n, 3) poses on pairs[i] (image * n_models + model)."""
        return _score(_ContBatch(self), level, _cont_poses(poses, pairs), stream)

    def cont_score_backward(self, level: int, poses: torch.Tensor, pairs, grad_scores=None, stream=None):
        return _backward(_ContBatch(self), level, _cont_poses(poses, pairs), grad_scores, stream)

    def cont_line_search(self, level: int, poses: torch.Tensor, pairs, dirs: torch.Tensor, alphas, stream=None):
        rec, sc = _line_search(_ContBatch(self), level, _cont_poses(poses, pairs), dirs, alphas, stream)
        return rec[:, :3].clone(), sc

    def refine_continuous(self, poses: torch.Tensor, pairs, steps: int = 8, level: int = 0, step_xy: float = 0.5,
                          step_theta: float = 0.5, decay: float = 0.6):
        """refine_continuous over the batch's pairs (see the module function)."""
        return _ascend(_ContBatch(self), _cont_poses(poses, pairs), steps, level, step_xy, step_theta, decay)

    def results(self):
        """Per pair, the detections as a numpy structured array (waits for the
        device); TMError(TM_ECAPACITY), with the truncated lists, if a pair had
        more matches than the capacity."""
        n = self.n_out.cpu().numpy()
        o = self.out.cpu().numpy()
        res = [o[p].view(POSE_DTYPE).reshape(-1)[:min(int(n[p]), self.capacity)] for p in range(len(n))]
        over = [p for p in range(len(n)) if n[p] > self.capacity]
        if over:
            raise TMError(TM_ECAPACITY, f"pairs {over[:8]} found more than {self.capacity} matches: the best "
                                        f"{self.capacity} by key were kept", res)
        return res

    def free(self):
        if self._h:
            lib().tm_batch_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------- continuous score
def _cont_poses(poses: torch.Tensor, pairs=None) -> torch.Tensor:
    """(n, 3) (x, y, theta_deg) [+ (n,) pair indices] -> device tm_cont_pose
    records, as an (n, 4) float32 tensor whose last column holds the int32
    pair bits."""
    p = poses.detach().to(device="cuda", dtype=torch.float32).reshape(-1, 3)
    rec = torch.zeros((p.shape[0], 4), dtype=torch.float32, device="cuda")
    rec[:, :3] = p
    if pairs is not None:
        pr = torch.as_tensor(pairs, dtype=torch.int32).to("cuda").reshape(-1)
        if pr.shape[0] != p.shape[0]:
            raise TMError(TM_EINVAL, "one pair index per pose")
        rec.view(torch.int32)[:, 3] = pr
    return rec.contiguous()


def _alphas(alphas):
    return (ctypes.c_double * len(alphas))(*[float(v) for v in alphas]), len(alphas)


class _ContSingle:
    """Continuous-score calls on one (model, pyramid) pair."""

    def __init__(self, model: Model, pyr: Pyramid):
        self.model, self.pyr = model, pyr

    def score(self, level, rec, out, st):
        _check(lib().tm_cont_score(self.model.handle, self.pyr.handle, level, _vp(rec.data_ptr()), rec.shape[0],
                                   _vp(out.data_ptr()), _vp(st)))

    def backward(self, level, rec, gin, gout, st):
        _check(lib().tm_cont_score_backward(self.model.handle, self.pyr.handle, level, _vp(rec.data_ptr()),
                                            rec.shape[0], gin, _vp(gout.data_ptr()), _vp(st)))

    def line_search(self, level, rec, dirs, alphas, sc, st):
        a, na = _alphas(alphas)
        _check(lib().tm_cont_line_search(self.model.handle, self.pyr.handle, level, _vp(rec.data_ptr()),
                                         _vp(dirs.data_ptr()), rec.shape[0], a, na, _vp(sc.data_ptr()), _vp(st)))


class _ContBatch:
    """Continuous-score calls over the pairs of a batch."""

    def __init__(self, batch):
        self.batch = batch

    def score(self, level, rec, out, st):
        _check(lib().tm_batch_cont_score(self.batch.handle, level, _vp(rec.data_ptr()), rec.shape[0],
                                         _vp(out.data_ptr()), _vp(st)))

    def backward(self, level, rec, gin, gout, st):
        _check(lib().tm_batch_cont_score_backward(self.batch.handle, level, _vp(rec.data_ptr()), rec.shape[0], gin,
                                                  _vp(gout.data_ptr()), _vp(st)))

    def line_search(self, level, rec, dirs, alphas, sc, st):
        a, na = _alphas(alphas)
        _check(lib().tm_batch_cont_line_search(self.batch.handle, level, _vp(rec.data_ptr()), _vp(dirs.data_ptr()),
                                               rec.shape[0], a, na, _vp(sc.data_ptr()), _vp(st)))


def _score(t, level, rec, stream=None):
    out = torch.empty(rec.shape[0], dtype=torch.float32, device="cuda")
    t.score(level, rec, out, _stream(stream))
    return out


def _backward(t, level, rec, grad_scores=None, stream=None):
    out = torch.empty((rec.shape[0], 3), dtype=torch.float32, device="cuda")
    g = None if grad_scores is None else grad_scores.detach().to(device="cuda", dtype=torch.float32).contiguous()
    t.backward(level, rec, _vp(g.data_ptr()) if g is not None else None, out, _stream(stream))
    return out


def _line_search(t, level, rec, dirs, alphas, stream=None):
    rec = rec.clone()
    d = dirs.detach().to(device="cuda", dtype=torch.float32).reshape(-1, 3).contiguous()
    sc = torch.empty(rec.shape[0], dtype=torch.float32, device="cuda")
    t.line_search(level, rec, d, alphas, sc, _stream(stream))
    return rec, sc


def _ascend(t, rec, steps, level, step_xy, step_theta, decay):
    alphas = [0.0, 0.125, 0.25, 0.5, 1.0, 2.0]
    sxy, sth = step_xy, step_theta
    sc = None
    for _ in range(max(1, steps)):
        g = _backward(t, level, rec)
        d = torch.cat([sxy * g[:, :2] / g[:, :2].norm(dim=1, keepdim=True).clamp_min(1e-20),
                       (sth * torch.sign(g[:, 2]))[:, None]], dim=1)
        rec, sc = _line_search(t, level, rec, d, alphas)
        sxy *= decay
        sth *= decay
    return rec[:, :3].clone(), sc


def cont_score(model: Model, pyr: Pyramid, level: int, poses: torch.Tensor, stream=None) -> torch.Tensor:
    """Continuous score of (n, 3) poses (x, y, theta_deg) at `level`."""
    return _score(_ContSingle(model, pyr), level, _cont_poses(poses), stream)


def cont_score_backward(model: Model, pyr: Pyramid, level: int, poses: torch.Tensor,
                        grad_scores: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """grad_scores[i] * dS/d(x, y, theta_deg) of each pose, (n, 3)."""
    return _backward(_ContSingle(model, pyr), level, _cont_poses(poses), grad_scores, stream)


def cont_line_search(model: Model, pyr: Pyramid, level: int, poses: torch.Tensor, dirs: torch.Tensor, alphas,
                     stream=None):
    """Move each pose to the best of pose + alpha_j dir (scores in FP64); returns (poses, scores)."""
    rec, sc = _line_search(_ContSingle(model, pyr), level, _cont_poses(poses), dirs, alphas, stream)
    return rec[:, :3].clone(), sc


class ContinuousScore(torch.autograd.Function):
    """S_c of (n, 3) poses with the hand-written backward kernel.  Call as
    ContinuousScore.apply(poses, model, pyramid, level), or with a Batch in
    place of the model and the (n,) pair indices in place of the pyramid."""

    @staticmethod
    def forward(ctx, poses, model_or_batch, pyr_or_pairs, level):
        if isinstance(model_or_batch, Batch):
            t, rec = _ContBatch(model_or_batch), _cont_poses(poses, pyr_or_pairs)
        else:
            t, rec = _ContSingle(model_or_batch, pyr_or_pairs), _cont_poses(poses)
        ctx.t, ctx.rec, ctx.level = t, rec, level
        return _score(t, level, rec)

    @staticmethod
    def backward(ctx, grad):
        return _backward(ctx.t, ctx.level, ctx.rec, grad), None, None, None


def refine_continuous(model: Model, pyr: Pyramid, poses: torch.Tensor, steps: int = 8, level: int = 0,
                      step_xy: float = 0.5, step_theta: float = 0.5, decay: float = 0.6):
    """Sub-pixel / sub-degree refinement of (n, 3) poses (x, y, theta_deg) by
    gradient ascent on S_c.  Each step takes the gradient (backward kernel),
    scales its translation part to length step_xy and its angle part to
    +-step_theta degrees, and moves each pose to the best of the step lengths
    {0, 1/8, 1/4, 1/2, 1, 2} along it, scored in FP64; so no pose's score goes
    down.  Step lengths shrink by `decay` per step.  Returns (poses, scores),
    the scores those of the FP64 line search (FP32-rounded)."""
    return _ascend(_ContSingle(model, pyr), _cont_poses(poses), steps, level, step_xy, step_theta, decay)


_allocator_keep = None  # the registered callbacks stay referenced while the library may call them


def _torch_alloc(nbytes, ctx, stream):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:  # out of memory: the library returns TM_ENOMEM
        return None


def _torch_free(ptr, ctx, stream):
    torch.cuda.caching_allocator_delete(int(ptr))


def use_torch_allocator(on: bool = True):
    """Handles created from now on take their device memory from torch's
    caching allocator (on=False: back to hipMalloc / hipFree).  Handles keep
    the allocator they were created with."""
    global _allocator_keep
    if on:
        a = AllocatorC(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)
        _check(lib().tm_set_allocator(ctypes.byref(a)))
        # the old callbacks stay alive too: handles made with them free through them
        _allocator_keep = (a, _allocator_keep)
    else:
        _check(lib().tm_set_allocator(None))


PROBE_VALU_MIX, PROBE_VALU_ADD, PROBE_LDS, PROBE_HBM, PROBE_DOT2, PROBE_MAX_DPP, PROBE_MAX3 = 0, 1, 2, 3, 4, 5, 6


def probe_rate(kind: int, iterations: int = 2000, hbm_bytes: int = 1 << 30, repeats: int = 5) -> float:
    """Rate of a ceiling probe (tm_probe): work per second of the best of
    `repeats` launches, timed with events on the current stream (VALU:
    wave-level instructions/s; LDS and HBM: bytes/s)."""
    nbytes = hbm_bytes if kind == PROBE_HBM else 4096
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    work = ctypes.c_double()
    st = torch.cuda.current_stream()
    _check(lib().tm_probe(kind, iterations, _vp(buf.data_ptr()), nbytes, _vp(st.cuda_stream), ctypes.byref(work)))
    best = float("inf")
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        _check(lib().tm_probe(kind, iterations, _vp(buf.data_ptr()), nbytes, _vp(st.cuda_stream),
                              ctypes.byref(work)))
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    return work.value / best


def timing_enable(on: bool = True):
    """Record HIP events around every exhaustive-search kernel launch."""
    _check(lib().tm_timing_enable(1 if on else 0))


def timing_read():
    """(total ms, launches) of the search kernels recorded since the last read."""
    ms, n = ctypes.c_double(), _i32()
    _check(lib().tm_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def version() -> str:
    return lib().tm_version().decode()
