"""Pins of the FP64 oracle against facts fixed outside it: library special
cases (scipy Sobel, NumPy reshape-sum), closed forms of Eq. (1), invariances
of Eq. (1)-(2), high-precision rotation (mpmath), and an independent NumPy
brute force on tiny inputs.  None of these retypes the oracle's own code."""
import numpy as np
import pytest

import bruteforce as BF
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _rng(i):
    return np.random.default_rng(20211200 + 1000 + i)


# ---------------------------------------------------------------- O1 .. O3
def test_sobel_matches_scipy_correlate(oracle_mod):
    img = _rng(1).integers(0, 256, (37, 53), dtype=np.uint8)
    gx, gy = oracle_mod.sobel(img)
    bx, by = BF.sobel(img)
    assert np.array_equal(gx, bx) and np.array_equal(gy, by)
    # the one-pixel frame is zero
    for g in (gx, gy):
        assert not g[0].any() and not g[-1].any() and not g[:, 0].any() and not g[:, -1].any()


def test_sobel_sign_on_ramp(oracle_mod):
    # intensity increasing with x gives gx > 0, gy == 0 (x right, y down)
    img = np.tile(np.arange(0, 200, 10, dtype=np.uint8), (8, 1))
    gx, gy = oracle_mod.sobel(img)
    assert (gx[1:-1, 1:-1] == 80).all() and (gy == 0).all()
    gx, gy = oracle_mod.sobel(img.T.copy())
    assert (gy[1:-1, 1:-1] == 80).all() and (gx == 0).all()


def test_edge_threshold_strict_and_unit(oracle_mod):
    # a vertical step of height h gives |gx| in {h, 3h, 4h}: threshold at exactly 4h*4h excludes
    img = np.zeros((9, 9), np.uint8)
    img[:, 5:] = 25
    gx, gy = oracle_mod.sobel(img)
    assert gx.max() == 100
    g_at = oracle_mod.edge_field(img, 100.0)  # floor(100^2) = 10000 == m2: not an edge (strict >)
    assert not g_at.any()
    g_below = oracle_mod.edge_field(img, 99.99)
    e = np.any(g_below != 0, axis=-1)
    assert e.sum() == 2 * 7  # two columns of full-step pixels, interior rows
    assert np.allclose(g_below[e], [1.0, 0.0], atol=0, rtol=0)
    img2 = _rng(2).integers(0, 256, (30, 31), dtype=np.uint8)
    g = oracle_mod.edge_field(img2, 30.0)
    e = np.any(g != 0, axis=-1)
    assert np.allclose(np.hypot(g[e, 0], g[e, 1]), 1.0, atol=1e-15)
    assert np.array_equal(g, BF.field(img2, 30.0))


def test_pyramid_matches_reshape_sum(oracle_mod):
    for (H, W) in [(64, 48), (33, 71), (7, 5)]:
        img = _rng(3).integers(0, 256, (H, W), dtype=np.uint8)
        d = oracle_mod.pyr_down(img)
        h2, w2 = H // 2, W // 2
        s = img[:2 * h2, :2 * w2].astype(np.int64).reshape(h2, 2, w2, 2).sum(axis=(1, 3))
        assert np.array_equal(d, ((s + 2) >> 2).astype(np.uint8))
    levels = oracle_mod.pyramid(np.zeros((480, 640), np.uint8), 4)
    assert [lv.shape for lv in levels] == [(480, 640), (240, 320), (120, 160), (60, 80)]


def test_model_points_row_major_centre(oracle_mod):
    img = np.full((16, 20), 40, np.uint8)
    img[5:11, 6:13] = 200
    t, d = oracle_mod.model_points(oracle_mod.edge_field(img, 30.0))
    bt, bd = BF.model(img, 30.0)
    assert np.array_equal(t, bt) and np.array_equal(d, bd)
    # the reference pixel (W//2, H//2) = (10, 8) maps to t = 0
    ys, xs = t[:, 1] + 8, t[:, 0] + 10
    assert (np.diff(ys * 100 + xs) > 0).all()  # strictly row-major


# ---------------------------------------------------------------- O5, O6
def test_angle_grid(oracle_mod):
    sp = oracle_mod.SearchParams(theta_step_top=1.0, theta_range=360.0)
    assert [oracle_mod.level_step(sp, 4, l) for l in range(4)] == [0.125, 0.25, 0.5, 1.0]
    assert oracle_mod.level_count(sp, 1.0) == 360 and oracle_mod.level_count(sp, 0.125) == 2880
    sp90 = oracle_mod.SearchParams(theta_step_top=3.0, theta_range=90.0)
    assert oracle_mod.level_count(sp90, 3.0) == 31  # 0, 3, ..., 90 inclusive
    assert oracle_mod.level_count(sp90, 1.5) == 61
    sp7 = oracle_mod.SearchParams(theta_step_top=7.0, theta_range=360.0)
    assert oracle_mod.level_count(sp7, 7.0) == 52
    L = oracle_mod.lib()
    assert [L.orc_angle_index(k, 360, 1) for k in (-1, 0, 359, 360, 721)] == [359, 0, 359, 0, 1]
    assert [L.orc_angle_index(k, 31, 0) for k in (-1, 0, 30, 31)] == [0, 0, 30, 30]
    assert oracle_mod.theta(10.0, 0.125, 7) == 10.875


def test_sincos_deg_exact_quadrants_and_accuracy(oracle_mod):
    import mpmath as mp
    mp.mp.dps = 50
    for k in range(-8, 9):
        c, s = oracle_mod.sincos_deg(90.0 * k)
        exp = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][k % 4]
        assert (c, s) == exp
    for deg in np.concatenate([np.arange(-720, 721, 0.125), _rng(4).uniform(-1000, 1000, 500)]):
        c, s = oracle_mod.sincos_deg(float(deg))
        rad = mp.mpf(float(deg)) * mp.pi / 180
        assert abs(mp.mpf(c) - mp.cos(rad)) <= 4e-16 and abs(mp.mpf(s) - mp.sin(rad)) <= 4e-16


def _tables_vs_mpmath(oracle_mod, t, thetas):
    """Every q of every angle equals the 50-digit rounding; returns the
    smallest distance of R t + 1/2 + 1e-9 to an integer (the snap margin)."""
    import mpmath as mp
    mp.mp.dps = 50
    tx = [mp.mpf(int(v)) for v in t[:, 0]]
    ty = [mp.mpf(int(v)) for v in t[:, 1]]
    margin = mp.mpf(1)
    snap = mp.mpf("0.5") + mp.mpf("1e-9")
    for th in thetas:
        q, _ = oracle_mod.rotate(t, np.zeros_like(t, dtype=np.float64), th)
        rad = mp.mpf(th) * mp.pi / 180
        c, s = mp.cos(rad), mp.sin(rad)
        for i in range(len(t)):
            vx = c * tx[i] - s * ty[i] + snap
            vy = s * tx[i] + c * ty[i] + snap
            fx, fy = int(mp.floor(vx)), int(mp.floor(vy))
            assert (q[i, 0], q[i, 1]) == (fx, fy), (th, i)
            margin = min(margin, vx - fx, fx + 1 - vx, vy - fy, fy + 1 - vy)
    return float(margin)


@pytest.mark.parametrize("ci", [1, 2, 3])
def test_rotated_tables_vs_mpmath(oracle_mod, ci):
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    m = oracle_mod.build_model(sc.model, oracle_mod.PyrParams(cfg["levels"], cfg["tau_m"]))
    sp = oracle_mod.SearchParams(theta_step_top=cfg["theta_step_top"], theta_range=cfg["theta_range"])
    L = cfg["levels"]
    top = L - 1
    st = oracle_mod.level_step(sp, L, top)
    K = oracle_mod.level_count(sp, st)
    thetas = [oracle_mod.theta(0.0, st, k) for k in range(K)]
    margin = _tables_vs_mpmath(oracle_mod, m.levels[top].t, thetas)
    assert margin > 1e-12
    if L > 1:  # a sample of the level-0 angles used by refinement
        s0 = oracle_mod.level_step(sp, L, 0)
        K0 = oracle_mod.level_count(sp, s0)
        ks = _rng(5).choice(K0, 24, replace=False)
        margin = _tables_vs_mpmath(oracle_mod, m.levels[0].t, [oracle_mod.theta(0.0, s0, int(k)) for k in ks])
        assert margin > 1e-12


def test_rotation_half_snaps_up(oracle_mod):
    # 3 sin 30 = 1.5 exactly; FP64 gives 1.4999999999999998 and the snap still rounds up
    q, r = oracle_mod.rotate(np.array([[3, 0], [0, 3], [-3, 0]], np.int32), np.array([[1.0, 0.0]] * 3), 30.0)
    assert q[0].tolist() == [3, 2] and q[1].tolist() == [-1, 3] and q[2].tolist() == [-3, -1]
    assert np.allclose(r[0], [np.cos(np.pi / 6), 0.5], atol=1e-15)


# ---------------------------------------------------------------- O7 pins
def _model32(seed=0):
    rng = np.random.default_rng(20211200 + 500 + seed)
    shape = synth.make_model_shape("blocks", 32, rng)
    return synth.render_model(shape, 32)


@pytest.mark.parametrize("quarter", [0, 1, 2, 3])
def test_T1_pasted_model_scores_one_and_is_found(oracle_mod, quarter):
    """Eq. (1) reaches its maximum 1 at the true pose, and the exhaustive
    search (Sec. II para. 3) returns that pose."""
    model = _model32(quarter)
    ux, uy = 41, 37
    img = synth.paste_rot90(model, 96, 80, ux, uy, quarter)
    M = oracle_mod.build_model(model, oracle_mod.PyrParams(1, 30.0))
    g = oracle_mod.edge_field(img, 30.0)
    ml = M.levels[0]
    sw, s1 = oracle_mod.score(g, ml.t, ml.d, ux, uy, 90.0 * quarter)
    assert abs(sw - 1.0) <= 1e-12 and abs(s1 - 1.0) <= 1e-12
    sp = oracle_mod.SearchParams(theta_step_top=5.0, min_score=0.5, max_matches=1)
    tr = oracle_mod.detect(img, model, oracle_mod.PyrParams(1, 30.0), oracle_mod.PyrParams(1, 30.0), sp)
    d = tr.detections[0]
    assert (d.x, d.y, d.k) == (ux, uy, 18 * quarter)
    # the plateau of S_w == 1 around the match is broken by S_1
    mw, m1, mk = tr.top
    assert np.sum(mw >= mw[uy, ux]) >= 2 and m1[uy, ux] == m1[mw >= mw[uy, ux]].max()


@pytest.mark.parametrize("levels,ux,uy,quarter", [(2, 47, 40, 1), (2, 49, 42, 1), (3, 63, 48, 1), (3, 67, 52, 1),
                                                  (3, 64, 48, 0), (3, 63, 47, 2), (3, 64, 47, 3)])
def test_T1_coarse_to_fine_finds_exact_pose(oracle_mod, levels, ux, uy, quarter):
    """Search starts at the top image and refines down (Sec. II para. 2).
    A level-l cell of the model covers offsets t in [2^l a - 16, 2^l a - 16 +
    2^l - 1] on each axis.  A turn that keeps an axis starts the cell at
    u - 16 + 2^l a, a multiple of 2^l when u = 0 (mod 2^l); a turn that
    negates it starts the cell at u + 17 - 2^l (a + 1), a multiple when
    u = -1 (mod 2^l).  Then every level of the search image is an exact paste
    of the model's level and the top level scores exactly 1 at the turn."""
    model = _model32(7)
    img = synth.paste_rot90(model, 128, 112, ux, uy, quarter)
    sp = oracle_mod.SearchParams(theta_step_top=10.0, min_score=0.5, max_matches=1)
    tr = oracle_mod.detect(img, model, oracle_mod.PyrParams(levels, 30.0), oracle_mod.PyrParams(levels, 30.0), sp)
    d = tr.detections[0]
    assert (d.x, d.y, d.theta) == (ux, uy, 90.0 * quarter)
    assert abs(d.sw - 1.0) <= 1e-12 and abs(d.s1 - 1.0) <= 1e-12


def test_T2_gain_offset_invariance_bitwise(oracle_mod):
    model = _model32(1)
    base = synth.paste_rot90(model, 64, 64, 30, 33, 0).astype(np.int64)
    base = (base // 2 + _rng(6).integers(0, 8, base.shape)).astype(np.uint8)  # values <= 127
    img2 = (2 * base.astype(np.int64) + 3).astype(np.uint8)
    M = oracle_mod.build_model(model, oracle_mod.PyrParams(1, 30.0))
    ml = M.levels[0]
    g1 = oracle_mod.edge_field(base, 30.0)
    g2 = oracle_mod.edge_field(img2, 60.0)
    assert np.array_equal(g1, g2)
    for (ux, uy, th) in [(30, 33, 0.0), (20, 25, 35.0), (31, 32, 185.0)]:
        assert oracle_mod.score(g1, ml.t, ml.d, ux, uy, th) == oracle_mod.score(g2, ml.t, ml.d, ux, uy, th)


def _has_exact_half(oracle_mod, t, th):
    c, s = oracle_mod.sincos_deg(th)
    v = np.concatenate([c * t[:, 0] - s * t[:, 1], s * t[:, 0] + c * t[:, 1]])
    return np.any(np.abs(np.abs(v - np.floor(v)) - 0.5) < 1e-6)


def test_T3_rot90_exact(oracle_mod):
    """Rotating the search image by -90 degrees (np.rot90) maps the score at
    (u, theta) to (rho(u), theta - 90) bit for bit."""
    model = _model32(2)
    scene = synth.render_scene(_rng(7), 72, 60, synth.make_model_shape("blocks", 32, _rng(8)), 32, 1, 5.0)
    img = scene.image
    H, W = img.shape
    rot = np.ascontiguousarray(np.rot90(img))
    M = oracle_mod.build_model(model, oracle_mod.PyrParams(1, 30.0))
    ml = M.levels[0]
    g = oracle_mod.edge_field(img, 30.0)
    gr = oracle_mod.edge_field(rot, 30.0)
    checked = 0
    for th in np.arange(0.0, 360.0, 5.0):
        if _has_exact_half(oracle_mod, ml.t, th):
            continue
        for (ux, uy) in [(20, 17), (40, 30), (3, 55), (71, 0)]:
            a = oracle_mod.score(g, ml.t, ml.d, ux, uy, th)
            b = oracle_mod.score(gr, ml.t, ml.d, uy, W - 1 - ux, th - 90.0)
            assert a == b, (th, ux, uy)
            checked += 1
    assert checked > 200


def test_T4_bruteforce_volume_and_argmax(oracle_mod):
    for trial in range(3):
        rng = _rng(10 + trial)
        mimg = np.full((8, 8), 40, np.uint8)
        mimg[2:6, 1:5] = 200
        mimg[1, 5:7] = 120
        simg = rng.integers(0, 256, (20, 22), dtype=np.uint8)
        simg[6:14, 9:17] = np.rot90(mimg, trial)
        tm_, ts_ = 30.0, 60.0
        M = oracle_mod.build_model(mimg, oracle_mod.PyrParams(1, tm_))
        ml = M.levels[0]
        bt, bd = BF.model(mimg, tm_)
        assert np.array_equal(ml.t, bt) and np.allclose(ml.d, bd, atol=0)
        g = oracle_mod.edge_field(simg, ts_)
        thetas = [oracle_mod.theta(0.0, 15.0, k) for k in range(24)]
        Sw, S1 = BF.score_volume(g, bt, bd, thetas)
        for k in range(0, 24, 5):
            for (x, y) in [(0, 0), (5, 7), (12, 10), (21, 19), (10, 3)]:
                a = oracle_mod.score(g, ml.t, ml.d, x, y, thetas[k])
                assert abs(a[0] - Sw[k, y, x]) <= 1e-12 and abs(a[1] - S1[k, y, x]) <= 1e-12
        mw, m1, mk = oracle_mod.top_map(g, ml.t, ml.d, 0.0, 15.0, 24, nthreads=2)
        assert np.allclose(mw, Sw.max(axis=0), atol=1e-12)
        # the chosen angle attains the volume's best (S_w, then S_1) at each translation
        ys, xs = np.mgrid[0:20, 0:22]
        assert np.allclose(Sw[mk, ys, xs], mw, atol=1e-12) and np.allclose(S1[mk, ys, xs], m1, atol=1e-12)
        best1 = np.where(np.abs(Sw - mw[None]) <= 1e-12, S1, -np.inf).max(axis=0)
        assert np.allclose(m1, best1, atol=1e-12)


def test_T5_blank_and_polarity(oracle_mod):
    model = _model32(3)
    M = oracle_mod.build_model(model, oracle_mod.PyrParams(1, 30.0))
    ml = M.levels[0]
    blank = np.full((64, 64), 77, np.uint8)
    g0 = oracle_mod.edge_field(blank, 30.0)
    for th in (0.0, 33.0, 270.0):
        assert oracle_mod.score(g0, ml.t, ml.d, 30, 30, th) == (0.0, 0.0)
    img = synth.paste_rot90(model, 64, 64, 30, 31, 0)
    inv = (255 - img).astype(np.uint8)
    sw, s1 = oracle_mod.score(oracle_mod.edge_field(inv, 30.0), ml.t, ml.d, 30, 31, 0.0)
    assert abs(s1 + 1.0) <= 1e-12 and sw <= 1e-12


def test_T6_occlusion_is_linear(oracle_mod):
    """Occluded points contribute nothing while n stays the model's count (Sec. II para. 6)."""
    model = _model32(4)
    img = synth.paste_rot90(model, 64, 64, 32, 30, 0)
    M = oracle_mod.build_model(model, oracle_mod.PyrParams(1, 30.0))
    ml = M.levels[0]
    n = len(ml.t)
    g = oracle_mod.edge_field(img, 30.0)
    for kk in (1, 7, n // 3, n):
        idx = _rng(20 + kk).choice(n, kk, replace=False)
        g2 = g.copy()
        g2[30 + ml.t[idx, 1], 32 + ml.t[idx, 0]] = 0.0
        _, s1 = oracle_mod.score(g2, ml.t, ml.d, 32, 30, 0.0)
        assert abs(s1 - (1.0 - kk / n)) <= 1e-12


def test_T7_window_bounds_centre(oracle_mod):
    rng = _rng(30)
    img = rng.integers(0, 256, (40, 44), dtype=np.uint8)
    M = oracle_mod.build_model(_model32(5), oracle_mod.PyrParams(1, 30.0))
    ml = M.levels[0]
    g = oracle_mod.edge_field(img, 50.0)
    for _ in range(40):
        x, y, th = int(rng.integers(-5, 50)), int(rng.integers(-5, 45)), float(rng.uniform(0, 360))
        sw, s1 = oracle_mod.score(g, ml.t, ml.d, x, y, th, 3)
        assert sw >= s1
        a = oracle_mod.score(g, ml.t, ml.d, x, y, th, 1)
        assert a[0] == a[1] == s1
        w5 = oracle_mod.score(g, ml.t, ml.d, x, y, th, 5)
        assert w5[0] >= sw and w5[1] == s1


def test_T8_translation_equivariance(oracle_mod):
    rng = _rng(40)
    big = np.full((90, 90), 40, np.uint8)
    big[20:70, 20:70] = rng.integers(0, 256, (50, 50))
    a, b = 7, 4
    shifted = np.full_like(big, 40)
    shifted[a:, b:] = big[:-a, :-b]  # content moves by (+b, +a) in (x, y)
    M = oracle_mod.build_model(_model32(6), oracle_mod.PyrParams(1, 30.0))
    ml = M.levels[0]
    g1 = oracle_mod.edge_field(big, 40.0)
    g2 = oracle_mod.edge_field(shifted, 40.0)
    for (x, y, th) in [(40, 40, 0.0), (45, 38, 123.0), (50, 50, 271.5)]:
        assert oracle_mod.score(g1, ml.t, ml.d, x, y, th) == oracle_mod.score(g2, ml.t, ml.d, x + b, y + a, th)


# ---------------------------------------------------------------- O12
def test_continuous_score_equals_centre_score_on_the_grid(oracle_mod):
    """At integer translations and quarter turns every projected point is a
    pixel, so bilinear interpolation returns the pixel and S_c equals S_1."""
    rng = _rng(60)
    img = rng.integers(0, 256, (60, 64), dtype=np.uint8)
    ml = oracle_mod.build_model(_model32(8), oracle_mod.PyrParams(1, 30.0)).levels[0]
    g = oracle_mod.edge_field(img, 40.0)
    for (x, y, th) in [(20, 30, 0.0), (31, 17, 90.0), (40, 41, 180.0), (3, 58, 270.0), (-5, 10, -90.0)]:
        sc, _ = oracle_mod.cont_score(g, ml.t, ml.d, x, y, th)
        assert sc == oracle_mod.score(g, ml.t, ml.d, x, y, th)[1]


def test_continuous_score_constant_field_closed_form(oracle_mod):
    """On a constant unit field f the interpolated direction is f wherever all
    four neighbours are inside, so S_c = mean(R(theta) d_i) . f, and its
    gradient in translation is zero."""
    ml = oracle_mod.build_model(_model32(9), oracle_mod.PyrParams(1, 30.0)).levels[0]
    f = np.array([0.6, 0.8])
    g = np.broadcast_to(f, (90, 90, 2)).copy()
    for (x, y, th) in [(45.3, 44.7, 12.5), (40.9, 50.2, 200.0)]:
        sc, grad = oracle_mod.cont_score(g, ml.t, ml.d, x, y, th)
        c, s = np.cos(np.deg2rad(th)), np.sin(np.deg2rad(th))
        r = ml.d @ np.array([[c, -s], [s, c]]).T
        assert abs(sc - (r @ f).mean()) <= 1e-14
        assert abs(grad[0]) <= 1e-14 and abs(grad[1]) <= 1e-14
        # d/dtheta of mean(R d) . f in degrees
        dr = ml.d @ np.array([[-s, -c], [c, -s]]).T
        assert abs(grad[2] - np.pi / 180 * (dr @ f).mean()) <= 1e-14


def test_continuous_gradient_matches_central_differences(oracle_mod):
    """Away from pixel-cell boundaries the score is smooth: central
    differences (h = 1e-3 px / degree) agree with the analytic gradient."""
    model = _model32(10)
    img = synth.paste_rot90(model, 90, 90, 45, 44, 0)
    img = np.clip(img.astype(np.int64) + _rng(61).integers(-3, 4, img.shape), 0, 255).astype(np.uint8)
    ml = oracle_mod.build_model(model, oracle_mod.PyrParams(1, 30.0)).levels[0]
    g = oracle_mod.edge_field(img, 30.0)
    rng = _rng(62)
    h = 1e-3
    checked = 0
    for _ in range(400):
        x, y, th = 45 + rng.uniform(-1.5, 1.5), 44 + rng.uniform(-1.5, 1.5), rng.uniform(-3, 3)
        c, s = np.cos(np.deg2rad(th)), np.sin(np.deg2rad(th))
        p = ml.t @ np.array([[c, -s], [s, c]]).T + [x, y]
        f = p - np.floor(p)
        if np.min(np.minimum(f, 1 - f)) < 4 * h:
            continue  # a point would cross a cell boundary inside the stencil
        _, grad = oracle_mod.cont_score(g, ml.t, ml.d, x, y, th)
        fd = []
        for e in np.eye(3):
            sp_, _ = oracle_mod.cont_score(g, ml.t, ml.d, x + h * e[0], y + h * e[1], th + h * e[2])
            sm_, _ = oracle_mod.cont_score(g, ml.t, ml.d, x - h * e[0], y - h * e[1], th - h * e[2])
            fd.append((sp_ - sm_) / (2 * h))
        assert np.allclose(grad, fd, atol=1e-8, rtol=1e-6), (grad, fd)
        checked += 1
        if checked >= 5:
            break
    assert checked >= 3


# ---------------------------------------------------------------- O10
def test_refine_picks_best_of_27_by_bruteforce(oracle_mod):
    rng = _rng(50)
    img = rng.integers(0, 256, (30, 34), dtype=np.uint8)
    mimg = np.full((8, 8), 40, np.uint8)
    mimg[2:6, 2:7] = 210
    bt, bd = BF.model(mimg, 30.0)
    M = oracle_mod.build_model(mimg, oracle_mod.PyrParams(1, 30.0))
    g = BF.field(img, 50.0)
    K, step = 48, 7.5
    cands = oracle_mod.Candidates(np.array([0, 8, 16], np.int32), np.array([0, 7, 14], np.int32),
                                  np.array([0, 11, 23], np.int32), np.zeros(3), np.zeros(3))
    out = oracle_mod.refine_level(g, M.levels[0], cands, 0.0, step, K, True, 3)
    thetas = [oracle_mod.theta(0.0, step, k) for k in range(K)]
    Sw, S1 = BF.score_volume(g, bt, bd, thetas)
    for c in range(3):
        best = None
        for dk in (-1, 0, 1):
            k = (2 * int(cands.k[c]) + dk) % K
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    x, y = 2 * int(cands.x[c]) + a, 2 * int(cands.y[c]) + b
                    if not (0 <= x < 34 and 0 <= y < 30):
                        continue
                    key = (-Sw[k, y, x], -S1[k, y, x], x, y, k)
                    best = key if best is None or key < best else best
        assert (int(out.x[c]), int(out.y[c]), int(out.k[c])) == best[2:]
        assert abs(out.sw[c] + best[0]) <= 1e-12 and abs(out.s1[c] + best[1]) <= 1e-12
