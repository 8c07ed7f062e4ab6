"""Seeded scene generators for the five workload configurations.

Conventions shared with the detector's pose (and nothing else):
  * a model image of W x H pixels has its reference point at the integer pixel
    (W // 2, H // 2); shape coordinates t are relative to that pixel;
  * an instance at pose (ux, uy, theta) maps model point t to search position
    R(theta) t + u, theta in degrees, image axes x right and y down.
Rendering samples every pixel at 4 x 4 sub-positions and maps each back to the
model frame with the inverse pose, so the instance is drawn analytically
rather than by resampling the model image.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20211200

_SUB = (np.arange(4, dtype=np.float64) + 0.5) / 4.0 - 0.5  # 4x4 supersampling offsets


# ---------------------------------------------------------------- shapes
@dataclass
class Rect:
    cx: float
    cy: float
    hw: float
    hh: float

    def contains(self, x, y):
        return (np.abs(x - self.cx) <= self.hw) & (np.abs(y - self.cy) <= self.hh)


@dataclass
class Ellipse:
    cx: float
    cy: float
    a: float
    b: float

    def contains(self, x, y):
        return ((x - self.cx) / self.a) ** 2 + ((y - self.cy) / self.b) ** 2 <= 1.0


@dataclass
class Polygon:
    xs: np.ndarray
    ys: np.ndarray

    def contains(self, x, y):
        inside = np.zeros(np.shape(x), dtype=bool)
        n = len(self.xs)
        for i in range(n):
            x0, y0 = self.xs[i], self.ys[i]
            x1, y1 = self.xs[(i + 1) % n], self.ys[(i + 1) % n]
            cond = (y0 > y) != (y1 > y)
            with np.errstate(divide="ignore", invalid="ignore"):
                xc = x0 + (y - y0) * (x1 - x0) / (y1 - y0)
            inside ^= cond & (x < xc)
        return inside


@dataclass
class Shape:
    """A union of filled parts minus a union of holes, in model coordinates."""
    parts: list
    holes: list = field(default_factory=list)
    radius: float = 0.0  # bounding radius around the reference point

    def contains(self, x, y):
        m = np.zeros(np.shape(x), dtype=bool)
        for p in self.parts:
            m |= p.contains(x, y)
        for h in self.holes:
            m &= ~h.contains(x, y)
        return m


def make_model_shape(kind: str, size: int, rng: np.random.Generator, n_holes=(1, 3), hole_frac=(0.08, 0.16)) -> Shape:
    """'blocks': 2-3 rectangles or ellipses (small models);
    'polygon': a star-shaped polygon of 5-9 vertices with n_holes[0]..n_holes[1]
    elliptic holes of radius hole_frac * size (fewer if they do not fit)."""
    half = size / 2.0
    if kind == "blocks":
        parts = []
        for _ in range(int(rng.integers(2, 4))):
            cx, cy = rng.uniform(-0.3, 0.3, 2) * size
            a, b = rng.uniform(0.12, 0.25, 2) * size
            a = min(a, half - 3 - abs(cx))
            b = min(b, half - 3 - abs(cy))
            if rng.random() < 0.5:
                parts.append(Rect(cx, cy, a, b))
            else:
                parts.append(Ellipse(cx, cy, a, b))
        return Shape(parts, [], radius=half * np.sqrt(2.0))
    if kind == "polygon":
        nv = int(rng.integers(5, 10))
        # vertices angularly spread so the polygon stays simple
        ang = np.linspace(0, 2 * np.pi, nv, endpoint=False) + rng.uniform(-0.25, 0.25, nv) * (2 * np.pi / nv)
        rmax = half - 6.0
        rad = rng.uniform(0.6, 1.0, nv) * rmax
        poly = Polygon(rad * np.cos(ang), rad * np.sin(ang))
        holes = []
        rin = rad.min() * np.cos(np.pi / nv)  # inscribed radius bound
        for _ in range(int(rng.integers(n_holes[0], n_holes[1] + 1))):
            for _try in range(50):
                hr = rng.uniform(*hole_frac) * size
                hb = hr * rng.uniform(0.6, 1.0)
                cr = rng.uniform(0.0, max(rin - hr - 4.0, 0.0))
                ca = rng.uniform(0, 2 * np.pi)
                h = Ellipse(cr * np.cos(ca), cr * np.sin(ca), hr, hb)
                if all(np.hypot(h.cx - o.cx, h.cy - o.cy) > h.a + o.a + 3 for o in holes):
                    holes.append(h)
                    break
        return Shape([poly], holes, radius=float(rad.max()) + 1.0)
    raise ValueError(kind)


def _coverage(shape: Shape, X: np.ndarray, Y: np.ndarray, ux: float, uy: float, theta_deg: float,
              scale: float = 1.0):
    """Fraction of each pixel (X, Y) covered by the shape posed at (u, theta)
    and scaled by `scale` about its reference point."""
    c, s = np.cos(np.deg2rad(theta_deg)), np.sin(np.deg2rad(theta_deg))
    acc = np.zeros(X.shape, np.float64)
    for oy in _SUB:
        for ox in _SUB:
            px = X + ox - ux
            py = Y + oy - uy
            tx = (c * px + s * py) / scale  # R(theta)^T (p - u) / scale
            ty = (-s * px + c * py) / scale
            acc += shape.contains(tx, ty)
    return acc / 16.0


def render_model(shape: Shape, size: int, fg: float = 200.0, bg: float = 40.0) -> np.ndarray:
    """The model image: the shape at the identity pose about pixel (size//2, size//2)."""
    Y, X = np.mgrid[0:size, 0:size].astype(np.float64)
    cov = _coverage(shape, X, Y, size // 2, size // 2, 0.0)
    return np.clip(np.rint(bg + (fg - bg) * cov), 0, 255).astype(np.uint8)


@dataclass
class Instance:
    x: float
    y: float
    theta: float
    scale: float = 1.0


@dataclass
class Scene:
    image: np.ndarray          # (H, W) uint8 search image
    model: np.ndarray          # (S, S) uint8 model image
    instances: list            # ground-truth poses
    shape: Shape
    config: dict


def _place(rng, W, H, radius, count, taken):
    out = []
    for _ in range(count):
        for _try in range(500):
            x = rng.uniform(radius + 2, W - radius - 2)
            y = rng.uniform(radius + 2, H - radius - 2)
            if all(np.hypot(x - a, y - b) > radius + r + 2 for a, b, r in taken):
                taken.append((x, y, radius))
                out.append((x, y))
                break
    return out


def _paint_instance(img, shape, ux, uy, theta, fg, scale=1.0):
    H, W = img.shape
    r = shape.radius * scale + 2
    x0, x1 = max(0, int(np.floor(ux - r))), min(W, int(np.ceil(ux + r)) + 1)
    y0, y1 = max(0, int(np.floor(uy - r))), min(H, int(np.ceil(uy + r)) + 1)
    Y, X = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    cov = _coverage(shape, X, Y, ux, uy, theta, scale)
    sub = img[y0:y1, x0:x1]
    img[y0:y1, x0:x1] = sub + (fg - sub) * cov


def _clutter(img, rng, count):
    H, W = img.shape
    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    for _ in range(count):
        grey = rng.uniform(0, 255)
        thick = rng.uniform(1, 3)
        if rng.random() < 0.5:
            x0, x1 = rng.uniform(0, W, 2)
            y0, y1 = rng.uniform(0, H, 2)
            bx0, bx1 = int(max(0, min(x0, x1) - 3)), int(min(W, max(x0, x1) + 4))
            by0, by1 = int(max(0, min(y0, y1) - 3)), int(min(H, max(y0, y1) + 4))
            xs, ys = X[by0:by1, bx0:bx1], Y[by0:by1, bx0:bx1]
            dx, dy = x1 - x0, y1 - y0
            L2 = dx * dx + dy * dy + 1e-12
            tt = np.clip(((xs - x0) * dx + (ys - y0) * dy) / L2, 0, 1)
            dist = np.hypot(xs - (x0 + tt * dx), ys - (y0 + tt * dy))
        else:
            cx, cy = rng.uniform(0, W), rng.uniform(0, H)
            a, b = rng.uniform(5, 60, 2)
            bx0, bx1 = int(max(0, cx - a - 4)), int(min(W, cx + a + 5))
            by0, by1 = int(max(0, cy - b - 4)), int(min(H, cy + b + 5))
            if bx1 <= bx0 or by1 <= by0:
                continue
            xs, ys = X[by0:by1, bx0:bx1], Y[by0:by1, bx0:bx1]
            rr = np.hypot((xs - cx) / a, (ys - cy) / b)
            dist = np.abs(rr - 1.0) * min(a, b)
        w = np.clip(thick / 2 + 0.5 - dist, 0, 1)
        sub = img[by0:by1, bx0:bx1]
        img[by0:by1, bx0:bx1] = sub + (grey - sub) * w


def render_scene(rng: np.random.Generator, W: int, H: int, shape: Shape, model_size: int,
                 n_inst: int, noise: float, occl_max: float = 0.0, gain=(1.0, 1.0),
                 offset=(0.0, 0.0), clutter: int = 0, fg: float = 200.0, bg: float = 40.0,
                 cfg: dict | None = None, theta_max: float = 360.0, scales=None) -> Scene:
    """Render n_inst posed instances (angles U[0, theta_max); with `scales`
    (lo, hi), each instance also scaled by U[lo, hi]), then apply the
    distortions in order: occluders, global gain and offset, clutter, Gaussian
    noise, clip and round."""
    img = np.full((H, W), bg, np.float64)
    taken = []
    spots = _place(rng, W, H, shape.radius * (scales[1] if scales else 1.0), n_inst, taken)
    inst = []
    for (x, y) in spots:
        th = float(rng.uniform(0.0, theta_max))
        sc = float(rng.uniform(*scales)) if scales else 1.0
        _paint_instance(img, shape, x, y, th, fg, sc)
        inst.append(Instance(float(x), float(y), th, sc))
    if occl_max > 0:
        for it in inst:
            frac = rng.uniform(0.0, occl_max)
            area = frac * model_size * model_size
            aspect = rng.uniform(0.5, 2.0)
            rw, rh = np.sqrt(area * aspect), np.sqrt(area / aspect)
            cx = it.x + rng.uniform(-0.5, 0.5) * model_size
            cy = it.y + rng.uniform(-0.5, 0.5) * model_size
            x0, x1 = int(max(0, np.rint(cx - rw / 2))), int(min(W, np.rint(cx + rw / 2)))
            y0, y1 = int(max(0, np.rint(cy - rh / 2))), int(min(H, np.rint(cy + rh / 2)))
            if x1 > x0 and y1 > y0:
                img[y0:y1, x0:x1] = rng.uniform(0, 255)
    a = rng.uniform(*gain)
    b = rng.uniform(*offset)
    img = a * img + b
    if clutter:
        _clutter(img, rng, clutter)
    if noise > 0:
        img = img + rng.normal(0.0, noise, img.shape)
    out = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    model = render_model(shape, model_size, fg, bg)
    return Scene(out, model, inst, shape, dict(cfg or {}))


# ------------------------------------------------------------- configs
# Sizes and search settings of the five workloads.  tau_m / tau_s are the
# model / search edge thresholds (L2 magnitude of the integer Sobel).
CONFIGS = {
    1: dict(name="C1 128x128 single instance", W=128, H=128, model_size=32, shape="blocks", n_inst=1,
            noise=5.0, occl=0.0, gain=(1.0, 1.0), offset=(0.0, 0.0), clutter=0, levels=1, tau_m=30.0,
            tau_s=30.0, theta_step_top=5.0, theta_range=360.0),
    2: dict(name="C2 640x480 industrial", W=640, H=480, model_size=128, shape="polygon", n_inst=3,
            noise=8.0, occl=0.30, gain=(0.5, 2.0), offset=(-40.0, 40.0), clutter=50, levels=4,
            tau_m=30.0, tau_s=80.0, theta_step_top=1.0, theta_range=360.0),
    3: dict(name="C3 2048x2048 large frame", W=2048, H=2048, model_size=256, shape="polygon", n_inst=5,
            noise=8.0, occl=0.40, gain=(0.5, 2.0), offset=(-40.0, 40.0), clutter=50, levels=5,
            tau_m=30.0, tau_s=80.0, theta_step_top=8.0, theta_range=360.0),
    # The paper's own experiment (Sec. III): 812x617 frames, search over every
    # 3rd pixel in x and y and 90 degrees in 3 degree steps, one level, one best
    # pose.  Its Basler samples are not available; this stands in for them with
    # one instance of a 96x96 polygon model at an angle inside the range and
    # the C2 distortions.
    6: dict(name="paper-shaped 812x617", W=812, H=617, model_size=96, shape="polygon", n_inst=1,
            noise=8.0, occl=0.30, gain=(0.5, 2.0), offset=(-40.0, 40.0), clutter=50, levels=1,
            tau_m=30.0, tau_s=80.0, theta_step_top=3.0, theta_range=90.0, step_xy=3, theta_max_inst=90.0,
            max_matches=1),
    # Similarity pose (x, y, theta, scale): C2 scenes whose instances are also
    # scaled by U[0.8, 1.2]; searched over scales 0.8 .. 1.2 in steps of 0.1,
    # 3 levels (a 32-pixel model at the top) and 4 degree top steps.
    7: dict(name="similarity 640x480", W=640, H=480, model_size=128, shape="polygon", n_inst=3,
            noise=8.0, occl=0.30, gain=(0.5, 2.0), offset=(-40.0, 40.0), clutter=50, levels=3,
            tau_m=30.0, tau_s=80.0, theta_step_top=4.0, theta_range=360.0, scales=(0.8, 1.2),
            scale_min=0.8, scale_step=0.1, scale_count=5),
}


# C4: eight models of increasing size (level-0 point counts at tau_m = 30 about
# 210, 305, 500, 750, 1100, 1700, 2500 and 3900), polygon with holes
# (size, hole count range, hole radius range as a fraction of the size).
C4_MODELS = [(40, (0, 0), (0.1, 0.1)), (52, (0, 0), (0.1, 0.1)), (64, (1, 1), (0.08, 0.14)),
             (90, (1, 1), (0.08, 0.14)), (128, (2, 3), (0.08, 0.14)), (160, (3, 5), (0.07, 0.12)),
             (208, (6, 8), (0.06, 0.10)), (256, (14, 18), (0.05, 0.08))]
C4_SIZES = [(640, 480), (1280, 1024), (2448, 2048)]
C4 = dict(name="C4 64 images x 8 models", n_images=64, levels=4, tau_m=30.0, tau_s=80.0, theta_step_top=1.0,
          theta_range=360.0, noise=8.0, occl=0.30, gain=(0.5, 2.0), offset=(-40.0, 40.0), clutter=50,
          inst=(1, 6))


@dataclass
class BatchScene:
    image: np.ndarray
    instances: list            # Instance poses
    models: list               # model index of each instance


def c4_model(k: int):
    """(shape, model image) of C4 model k (0..7)."""
    size, nh, hf = C4_MODELS[k]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + 4, spawn_key=(10**6 + k,))))
    shape = make_model_shape("polygon", size, rng, n_holes=nh, hole_frac=hf)
    return shape, render_model(shape, size)


def c4_image(index: int, shapes=None) -> BatchScene:
    """Image `index` of C4: its size drawn from C4_SIZES, 1-6 instances of
    models drawn uniformly (placed without overlap; fewer if they do not fit),
    then the C2 distortions (occluders, gain and offset, clutter, noise)."""
    cfg = C4
    if shapes is None:
        shapes = [c4_model(k)[0] for k in range(len(C4_MODELS))]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + 4, spawn_key=(index,))))
    W, H = C4_SIZES[int(rng.integers(0, len(C4_SIZES)))]
    n_inst = int(rng.integers(cfg["inst"][0], cfg["inst"][1] + 1))
    img = np.full((H, W), 40.0, np.float64)
    taken, inst, mids = [], [], []
    for _ in range(n_inst):
        k = int(rng.integers(0, len(shapes)))
        spot = _place(rng, W, H, shapes[k].radius, 1, taken)
        if not spot:
            continue
        x, y = spot[0]
        th = float(rng.uniform(0.0, 360.0))
        _paint_instance(img, shapes[k], x, y, th, 200.0)
        inst.append(Instance(float(x), float(y), th))
        mids.append(k)
    for it, k in zip(inst, mids):
        size = C4_MODELS[k][0]
        frac = rng.uniform(0.0, cfg["occl"])
        area = frac * size * size
        aspect = rng.uniform(0.5, 2.0)
        rw, rh = np.sqrt(area * aspect), np.sqrt(area / aspect)
        cx = it.x + rng.uniform(-0.5, 0.5) * size
        cy = it.y + rng.uniform(-0.5, 0.5) * size
        x0, x1 = int(max(0, np.rint(cx - rw / 2))), int(min(W, np.rint(cx + rw / 2)))
        y0, y1 = int(max(0, np.rint(cy - rh / 2))), int(min(H, np.rint(cy + rh / 2)))
        if x1 > x0 and y1 > y0:
            img[y0:y1, x0:x1] = rng.uniform(0, 255)
    img = rng.uniform(*cfg["gain"]) * img + rng.uniform(*cfg["offset"])
    _clutter(img, rng, cfg["clutter"])
    img = img + rng.normal(0.0, cfg["noise"], img.shape)
    return BatchScene(np.clip(np.rint(img), 0, 255).astype(np.uint8), inst, mids)


def c5_poses(scenes, n: int = 4096, seed: int = 5):
    """C5 start poses: ground-truth instances of the C4 scenes, cycled to n,
    each moved by U[-1.5, 1.5] px in x and y and U[-2, 2] degrees.  Returns
    (image index, model index, start (x, y, theta), truth (x, y, theta))."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + 5, spawn_key=(seed,))))
    gt = [(i, k, it) for i, sc in enumerate(scenes) for it, k in zip(sc.instances, sc.models)]
    img_i = np.empty(n, np.int32)
    mod_i = np.empty(n, np.int32)
    start = np.empty((n, 3), np.float64)
    truth = np.empty((n, 3), np.float64)
    for j in range(n):
        i, k, it = gt[j % len(gt)]
        img_i[j], mod_i[j] = i, k
        truth[j] = (it.x, it.y, it.theta)
        start[j] = (it.x + rng.uniform(-1.5, 1.5), it.y + rng.uniform(-1.5, 1.5), it.theta + rng.uniform(-2, 2))
    return img_i, mod_i, start, truth


def scene_for_config(ci: int, index: int = 0, **override) -> Scene:
    """Scene `index` of configuration `ci` (seed BASE_SEED + ci, image index
    as a spawn key, so every image is reproducible on its own)."""
    cfg = dict(CONFIGS[ci])
    cfg.update(override)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + ci, spawn_key=(index,))))
    shape_rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED + ci, spawn_key=(10**6,))))
    shape = make_model_shape(cfg["shape"], cfg["model_size"], shape_rng)
    return render_scene(rng, cfg["W"], cfg["H"], shape, cfg["model_size"], cfg["n_inst"], cfg["noise"],
                        cfg["occl"], cfg["gain"], cfg["offset"], cfg["clutter"], cfg=cfg,
                        theta_max=cfg.get("theta_max_inst", 360.0), scales=cfg.get("scales"))


def render_posed(shape: Shape, W: int, H: int, x: float, y: float, theta: float, scale: float = 1.0,
                 fg: float = 200.0, bg: float = 40.0) -> np.ndarray:
    """A clean W x H image with one instance of `shape` at pose (x, y, theta)
    and scale, drawn analytically (no distortions)."""
    img = np.full((H, W), bg, np.float64)
    _paint_instance(img, shape, x, y, theta, fg, scale)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def paste_rot90(model: np.ndarray, W: int, H: int, ux: int, uy: int, quarter: int, bg: int = 40) -> np.ndarray:
    """A constant-`bg` image with every model pixel moved exactly: model pixel
    with offset t from (S//2, S//2) lands at u + R(quarter*90 deg) t.  Pure
    integer index mapping, no resampling."""
    S_h, S_w = model.shape
    out = np.full((H, W), bg, np.uint8)
    ty, tx = np.mgrid[0:S_h, 0:S_w]
    tx = tx - S_w // 2
    ty = ty - S_h // 2
    c, s = [(1, 0), (0, 1), (-1, 0), (0, -1)][quarter % 4]
    px = ux + c * tx - s * ty
    py = uy + s * tx + c * ty
    ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
    out[py[ok], px[ok]] = model[ok]
    return out
