"""Pins of the oracle's two alternative readings, each switchable:

  * the gradient-map pyramid (O17): Sobel gradients of the full image, then a
    pyramid of the gradient maps by floored 2x2 means, edges per level;
  * the edge-taps-only vote (O16): a point's window maximum runs over the
    edge pixels of its window only, and a window without one votes 0.

They are pinned by a characterisation of the floored mean that does not
compute it (the residual bound), a NumPy reshape-sum, the closed form on an
intensity ramp, exact transposition equivariance, hand-worked fields whose
scores follow by inspection, an independent NumPy brute force, and the exact
order relation between the two votes."""
import numpy as np
import pytest

import bruteforce as BF
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _rng(i):
    return np.random.default_rng(20211200 + 3000 + i)


# ------------------------------------------------------------------ O17
def test_grad_down_residual_bound_and_values(oracle_mod):
    """floor((s + 2) / 4) is the unique G with s - 4 G in [-2, 1]."""
    rng = _rng(1)
    for (H, W) in [(9, 7), (32, 48), (33, 71)]:
        gx = rng.integers(-1020, 1021, (H, W)).astype(np.int32)
        gy = rng.integers(-1020, 1021, (H, W)).astype(np.int32)
        ox, oy = oracle_mod.grad_down(gx, gy)
        h2, w2 = H // 2, W // 2
        assert ox.shape == (h2, w2)
        for g, o in ((gx, ox), (gy, oy)):
            s = g[:2 * h2, :2 * w2].astype(np.int64).reshape(h2, 2, w2, 2).sum(axis=(1, 3))
            res = s - 4 * o.astype(np.int64)
            assert res.min() >= -2 and res.max() <= 1
    # block sums -7 .. 7 written out: -7 -> -2, -6 .. -3 -> -1, -2 .. 1 -> 0, 2 .. 5 -> 1, 6, 7 -> 2
    sums = np.arange(-7, 8)
    gx = np.zeros((2, 2 * len(sums)), np.int32)
    gx[0, 0::2] = sums
    ox, _ = oracle_mod.grad_down(gx, gx)
    assert ox[0].tolist() == [-2, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2]


def test_gradient_pyramid_matches_reshape_floor_divide(oracle_mod):
    img = _rng(2).integers(0, 256, (75, 101), dtype=np.uint8)
    ours = oracle_mod.gradient_pyramid(img, 4)
    ref = BF.grad_pyramid(img, 4)
    assert [g[0].shape for g in ours] == [(75, 101), (37, 50), (18, 25), (9, 12)]
    for (ax, ay), (bx, by) in zip(ours, ref):
        assert np.array_equal(ax, bx) and np.array_equal(ay, by)


def _footprint_inside(mask0, l):
    """Level-l pixels whose 2^l x 2^l block of level 0 lies inside mask0."""
    b = 1 << l
    H, W = mask0.shape[0] >> l, mask0.shape[1] >> l
    return mask0[:H * b, :W * b].reshape(H, b, W, b).all(axis=(1, 3))


def test_gradient_pyramid_ramp_keeps_level0_units(oracle_mod):
    """I = 2x + y + 10: the Sobel pair is (16, 8) on the interior, and every
    level of the gradient-map pyramid keeps (16, 8) where its block lies in
    the interior (the grey pyramid's ramp instead steepens by 2 per level);
    the unit directions of both readings agree there."""
    H, W = 48, 64
    ys, xs = np.mgrid[0:H, 0:W]
    img = (2 * xs + ys + 10).astype(np.uint8)
    interior = np.zeros((H, W), bool)
    interior[1:-1, 1:-1] = True
    pyr = oracle_mod.gradient_pyramid(img, 4)
    grey_imgs = oracle_mod.pyramid(img, 4)
    grey = oracle_mod.field_pyramid(img, 4, 5.0, "grey")
    grad = oracle_mod.field_pyramid(img, 4, 5.0, "gradient")
    u = np.array([2.0, 1.0]) / np.sqrt(5.0)
    for l, (gx, gy) in enumerate(pyr):
        inner = _footprint_inside(interior, l)
        assert inner.sum() > 10
        assert (gx[inner] == 16).all() and (gy[inner] == 8).all(), l
        assert np.allclose(grad[l][inner], u, atol=1e-15), l
        # the grey level is an exact ramp of slopes (2, 1) * 2^l
        gl = grey_imgs[l].astype(np.int64)
        assert (np.diff(gl, axis=1) == 2 << l).all() and (np.diff(gl, axis=0) == 1 << l).all(), l
        assert np.allclose(grey[l][1:-1, 1:-1], u, atol=1e-15), l


def test_gradient_pyramid_transpose_equivariant(oracle_mod):
    """Transposing the image swaps gx and gy at every level, bit for bit (no
    sign change, so the floored mean commutes with it exactly)."""
    img = _rng(3).integers(0, 256, (45, 70), dtype=np.uint8)
    a = oracle_mod.gradient_pyramid(img, 4)
    b = oracle_mod.gradient_pyramid(np.ascontiguousarray(img.T), 4)
    for (ax, ay), (bx, by) in zip(a, b):
        assert np.array_equal(ax.T, by) and np.array_equal(ay.T, bx)
    fa = oracle_mod.field_pyramid(img, 4, 40.0, "gradient")
    fb = oracle_mod.field_pyramid(np.ascontiguousarray(img.T), 4, 40.0, "gradient")
    for ga, gb in zip(fa, fb):
        assert np.array_equal(ga.transpose(1, 0, 2)[..., ::-1], gb)


def test_gradient_model_levels_follow_the_gradient_pyramid(oracle_mod):
    img = np.full((64, 64), 40, np.uint8)
    img[20:44, 14:50] = 210
    pp = oracle_mod.PyrParams(3, 30.0, "gradient")
    M = oracle_mod.build_model(img, pp)
    for l, (gx, gy) in enumerate(oracle_mod.gradient_pyramid(img, 3)):
        g = oracle_mod.direction_field(gx, gy, 30.0)
        t, d = oracle_mod.model_points(g)
        assert np.array_equal(M.levels[l].t, t) and np.array_equal(M.levels[l].d, d)
        assert (M.levels[l].width, M.levels[l].height) == (64 >> l, 64 >> l)
    # level 0 is the grey reading's level 0
    G = oracle_mod.build_model(img, oracle_mod.PyrParams(3, 30.0))
    assert np.array_equal(G.levels[0].t, M.levels[0].t) and np.array_equal(G.levels[0].d, M.levels[0].d)


# ------------------------------------------------------------------ O16
def _field(W, H, edges):
    g = np.zeros((H, W, 2))
    for (x, y), v in edges.items():
        g[y, x] = np.array(v, float) / np.hypot(*v)
    return g


def test_edge_vote_worked_examples(oracle_mod):
    one_t = np.array([[0, 0]], np.int32)
    one_d = np.array([[1.0, 0.0]])
    # one anti-parallel edge beside an off-edge centre: all taps 0, edge taps -1
    g = _field(7, 7, {(4, 3): (-1, 0)})
    assert oracle_mod.score(g, one_t, one_d, 3, 3, 0.0, vote="all") == (0.0, 0.0)
    assert oracle_mod.score(g, one_t, one_d, 3, 3, 0.0, vote="edge") == (-1.0, 0.0)
    # a window without edge pixels votes 0 in both readings
    assert oracle_mod.score(g, one_t, one_d, 1, 1, 0.0, vote="edge") == (0.0, 0.0)
    # the window reaching outside the image: outside taps are skipped, not 0
    g = _field(5, 5, {(0, 1): (0, 1)})
    assert oracle_mod.score(g, one_t, one_d, 0, 0, 0.0, vote="all") == (0.0, 0.0)
    assert oracle_mod.score(g, one_t, one_d, 0, 0, 0.0, vote="edge") == (0.0, 0.0)  # r.g = 0 exactly
    # a positive edge tap wins in both; all-edge windows agree
    g = _field(5, 5, {(1, 1): (3, 4), (2, 2): (-1, 0)})
    for v in ("all", "edge"):
        sw, s1 = oracle_mod.score(g, one_t, one_d, 2, 2, 0.0, vote=v)
        assert sw == 0.6 and s1 == -1.0
    full = {(x, y): (-1, 1 + x + 2 * y) for x in range(5) for y in range(5)}
    g = _field(5, 5, full)
    a = oracle_mod.score(g, one_t, one_d, 2, 2, 0.0, vote="all")
    b = oracle_mod.score(g, one_t, one_d, 2, 2, 0.0, vote="edge")
    assert a == b and a[0] < 0
    # two points: one with an anti-parallel edge only, one with an empty window
    two_t = np.array([[0, 0], [10, 0]], np.int32)
    two_d = np.array([[1.0, 0.0], [0.0, 1.0]])
    g = _field(20, 7, {(4, 3): (-1, 0)})
    assert oracle_mod.score(g, two_t, two_d, 3, 3, 0.0, vote="edge") == (-0.5, 0.0)
    assert oracle_mod.score(g, two_t, two_d, 3, 3, 0.0, vote="all") == (0.0, 0.0)


def test_edge_vote_bruteforce_volume(oracle_mod):
    for trial in range(2):
        rng = _rng(20 + trial)
        mimg = np.full((8, 8), 40, np.uint8)
        mimg[2:6, 1:5] = 200
        mimg[1, 5:7] = 120
        simg = rng.integers(0, 256, (18, 21), dtype=np.uint8)
        simg[5:13, 8:16] = np.rot90(mimg, trial + 1)
        M = oracle_mod.build_model(mimg, oracle_mod.PyrParams(1, 30.0))
        ml = M.levels[0]
        g = oracle_mod.edge_field(simg, 150.0)  # sparse edges: many windows partly or wholly off the edge set
        thetas = [oracle_mod.theta(0.0, 30.0, k) for k in range(12)]
        for win in (3, 5):
            Sw, S1 = BF.score_volume(g, ml.t, ml.d, thetas, win=win, vote="edge")
            for k in range(0, 12, 3):
                for (x, y) in [(0, 0), (4, 7), (11, 9), (20, 17), (9, 2)]:
                    a = oracle_mod.score(g, ml.t, ml.d, x, y, thetas[k], win=win, vote="edge")
                    assert abs(a[0] - Sw[k, y, x]) <= 1e-12 and abs(a[1] - S1[k, y, x]) <= 1e-12
            mw, m1, mk = oracle_mod.top_map(g, ml.t, ml.d, 0.0, 30.0, 12, win=win, nthreads=2, vote="edge")
            assert np.allclose(mw, Sw.max(axis=0), atol=1e-12)
            ys, xs = np.mgrid[0:18, 0:21]
            assert np.allclose(Sw[mk, ys, xs], mw, atol=1e-12)


def test_edge_vote_order_relation_and_window_one(oracle_mod):
    """Per point the edge-taps vote never exceeds the all-taps vote (a positive
    maximum comes from an edge tap; otherwise the all-taps vote is >= every
    edge tap), and FP64 addition is monotone, so S_w(edge) <= S_w(all) exactly;
    S_1 is the same; with a 1-pixel window the readings coincide."""
    cfg = synth.CONFIGS[2]
    sc = synth.scene_for_config(2, 0)
    M = oracle_mod.build_model(sc.model, oracle_mod.PyrParams(1, cfg["tau_m"]))
    ml = M.levels[0]
    g = oracle_mod.edge_field(sc.image, cfg["tau_s"])
    rng = _rng(30)
    differ = 0
    for _ in range(300):
        x, y = int(rng.integers(0, g.shape[1])), int(rng.integers(0, g.shape[0]))
        th = float(rng.integers(0, 360))
        a = oracle_mod.score(g, ml.t, ml.d, x, y, th, vote="all")
        b = oracle_mod.score(g, ml.t, ml.d, x, y, th, vote="edge")
        assert b[0] <= a[0] and b[1] == a[1]
        differ += b[0] < a[0]
        assert oracle_mod.score(g, ml.t, ml.d, x, y, th, win=1, vote="edge") == \
            oracle_mod.score(g, ml.t, ml.d, x, y, th, win=1, vote="all")
    assert differ > 100
    for inst in sc.instances[:2]:
        a = oracle_mod.score(g, ml.t, ml.d, int(round(inst.x)), int(round(inst.y)), round(inst.theta), vote="all")
        b = oracle_mod.score(g, ml.t, ml.d, int(round(inst.x)), int(round(inst.y)), round(inst.theta), vote="edge")
        assert b[0] <= a[0] and a[0] - b[0] < 0.2


@pytest.mark.parametrize("source,vote", [("gradient", "all"), ("grey", "edge"), ("gradient", "edge")])
def test_detect_with_readings_finds_the_instances(oracle_mod, source, vote):
    cfg = synth.CONFIGS[2]
    sc = synth.scene_for_config(2, 1)
    L = cfg["levels"]
    tr = oracle_mod.detect(sc.image, sc.model, oracle_mod.PyrParams(L, cfg["tau_s"], source),
                           oracle_mod.PyrParams(L, cfg["tau_m"], source),
                           oracle_mod.SearchParams(theta_step_top=cfg["theta_step_top"], vote=vote))
    assert len(tr.detections) >= 1
    d = tr.detections[0]
    near = [i for i in sc.instances if abs(i.x - d.x) <= 2 and abs(i.y - d.y) <= 2]
    assert near, (d, sc.instances)
