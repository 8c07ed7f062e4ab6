"""Independent NumPy brute force of the score definition, for tiny inputs.

Written from the definitions, not from the oracle's C: Sobel through
scipy.ndimage.correlate, edge directions by array arithmetic, the rotation
with numpy's cos/sin of radians, and each pose evaluated by gathering all
n x w x w taps from a zero-padded field.  Used to pin the oracle (Eq. (1) with
the neighbouring search, Eq. (2), exhaustive search of Sec. II para. 3).
"""
import numpy as np
from scipy import ndimage

SOBEL_X = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], dtype=np.int64)
SOBEL_Y = SOBEL_X.T.copy()


def sobel(img):
    a = img.astype(np.int64)
    gx = ndimage.correlate(a, SOBEL_X, mode="constant")
    gy = ndimage.correlate(a, SOBEL_Y, mode="constant")
    gx[0, :] = gx[-1, :] = 0
    gx[:, 0] = gx[:, -1] = 0
    gy[0, :] = gy[-1, :] = 0
    gy[:, 0] = gy[:, -1] = 0
    return gx, gy


def field(img, tau):
    gx, gy = sobel(img)
    m2 = gx * gx + gy * gy
    edge = m2 > np.floor(np.float64(np.float32(tau)) ** 2)
    m = np.sqrt(np.where(edge, m2, 1).astype(np.float64))
    g = np.stack([np.where(edge, gx / m, 0.0), np.where(edge, gy / m, 0.0)], axis=-1)
    return g


def model(img, tau):
    g = field(img, tau)
    ys, xs = np.nonzero(np.any(g != 0, axis=-1))  # row-major order
    H, W = img.shape
    t = np.stack([xs - W // 2, ys - H // 2], axis=1)
    d = g[ys, xs]
    return t, d


def rotate(t, d, theta_deg, sigma=1.0):
    th = np.deg2rad(theta_deg)
    c, s = np.cos(th), np.sin(th)
    R = np.array([[c, -s], [s, c]])
    v = t.astype(np.float64) @ R.T
    q = np.floor(sigma * v + 0.5 + 1e-9).astype(np.int64)
    r = d @ R.T
    return q, r


def grad_pyramid(img, levels):
    """Sobel gradients of the full image, then 2x2 block sums floored after
    adding 2 (numpy floor division), level by level."""
    gx, gy = sobel(img)
    out = [(gx, gy)]
    for _ in range(1, levels):
        H, W = gx.shape
        h2, w2 = H // 2, W // 2
        gx = np.floor_divide(gx[:2 * h2, :2 * w2].reshape(h2, 2, w2, 2).sum(axis=(1, 3)) + 2, 4)
        gy = np.floor_divide(gy[:2 * h2, :2 * w2].reshape(h2, 2, w2, 2).sum(axis=(1, 3)) + 2, 4)
        out.append((gx, gy))
    return out


def score_volume(g, t, d, thetas, win=3, sigma=1.0, vote="all"):
    """S_w and S_1 for every (k, y, x) at scale sigma: arrays of shape (K, H, W).
    vote "edge": only taps on the edge set (a nonzero field) enter the window
    maximum, and a window without one votes 0."""
    H, W, _ = g.shape
    h = (win - 1) // 2
    P = 2 * (int(np.ceil(sigma * np.abs(t).max())) + 2 + h) + 2
    gp = np.zeros((H + 2 * P, W + 2 * P, 2))
    gp[P:P + H, P:P + W] = g
    edge = np.any(gp != 0, axis=-1)
    K = len(thetas)
    Sw = np.zeros((K, H, W))
    S1 = np.zeros((K, H, W))
    ys, xs = np.mgrid[0:H, 0:W]
    n = len(t)
    for k, th in enumerate(thetas):
        q, r = rotate(t, d, th, sigma)
        best = np.full((n, H, W), -np.inf)
        centre = None
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                X = xs[None] + q[:, 0, None, None] + dx + P
                Y = ys[None] + q[:, 1, None, None] + dy + P
                v = gp[Y, X, 0] * r[:, 0, None, None] + gp[Y, X, 1] * r[:, 1, None, None]
                if dx == 0 and dy == 0:
                    centre = v
                if vote == "edge":
                    v = np.where(edge[Y, X], v, -np.inf)
                best = np.maximum(best, v)
        if vote == "edge":
            best = np.where(np.isneginf(best), 0.0, best)
        Sw[k] = best.sum(axis=0) / n
        S1[k] = centre.sum(axis=0) / n
    return Sw, S1
