"""Pins of the similarity-pose extension of the oracle (O13-O15): the
projection p = sigma R(theta) t + u, the exhaustive search over angles and
scales, and refinement at the chosen scale.

* at scale 1 every step is the rigid one, bit for bit;
* the rounded offsets equal a 50-digit evaluation of sigma R t for every
  point, angle and scale of a workload, with a safe margin from the rounding
  boundaries;
* an independent NumPy brute force (tests/bruteforce.py) gives the same score
  volume and best (angle, scale) per translation on tiny inputs;
* an instance drawn by the generator at a known angle and scale is found at
  that scale (the generator scales through its own inverse map), so larger
  sigma means a larger instance, as in Eq. (2) with a scale factor.
"""
import numpy as np
import pytest

import bruteforce as BF
import synth


def _rng(k):
    return np.random.default_rng(20211200 + 700 + k)


def test_unit_scale_is_the_rigid_search(oracle_mod):
    O = oracle_mod
    sc = synth.scene_for_config(1)
    ml = O.build_model(sc.model, O.PyrParams(1, 30.0)).levels[0]
    g = O.edge_field(sc.image, 30.0)
    a = O.top_map(g, ml.t, ml.d, 0.0, 5.0, 72, nthreads=4)
    b = O.top_map_sim(g, ml.t, ml.d, 0.0, 5.0, 72, 1.0, 0.25, 1, nthreads=4)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    q1, r1 = O.rotate(ml.t, ml.d, 37.5)
    q2, r2 = O.project(ml.t, ml.d, 37.5, 1.0)
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    # refinement: one scale, index m = k, is O10
    sc2 = synth.scene_for_config(2)
    om = O.build_model(sc2.model, O.PyrParams(2, 30.0))
    fields = O.field_pyramid(sc2.image, 2, 80.0)
    rng = _rng(1)
    cand = O.Candidates(rng.integers(0, 320, 8).astype(np.int32), rng.integers(0, 240, 8).astype(np.int32),
                        rng.integers(0, 180, 8).astype(np.int32), np.zeros(8), np.zeros(8))
    r_a = O.refine_level(fields[0], om.levels[0], cand, 0.0, 1.0, 360, True, 3)
    r_b = O.refine_level_sim(fields[0], om.levels[0], cand, 0.0, 1.0, 360, 180, True, 3, 1.0, 0.0)
    assert all(np.array_equal(getattr(r_a, f), getattr(r_b, f)) for f in ("x", "y", "k", "sw", "s1"))


def test_scaled_offsets_vs_mpmath(oracle_mod):
    """Every q of the similarity workload's top level (all 90 angles, all 5
    scales) equals the 50-digit rounding of sigma R t + 1/2 + 1e-9, sigma being
    the FP64 scale the search uses."""
    import mpmath as mp

    mp.mp.dps = 50
    O = oracle_mod
    sc = synth.scene_for_config(7)
    cfg = sc.config
    L = cfg["levels"]
    ml = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"])).levels[L - 1]
    tx = [mp.mpf(int(v)) for v in ml.t[:, 0]]
    ty = [mp.mpf(int(v)) for v in ml.t[:, 1]]
    snap = mp.mpf("0.5") + mp.mpf("1e-9")
    margin = mp.mpf(1)
    thetas = [O.theta(0.0, cfg["theta_step_top"], k) for k in range(0, 90, 3)]
    for j in range(cfg["scale_count"]):
        sig = O.scale(cfg["scale_min"], cfg["scale_step"], j)
        ms = mp.mpf(sig)
        for th in thetas:
            q, _ = O.project(ml.t, np.zeros((len(ml.t), 2)), th, sig)
            rad = mp.mpf(th) * mp.pi / 180
            c, s = mp.cos(rad), mp.sin(rad)
            for i in range(len(tx)):
                vx = ms * (c * tx[i] - s * ty[i]) + snap
                vy = ms * (s * tx[i] + c * ty[i]) + snap
                fx, fy = int(mp.floor(vx)), int(mp.floor(vy))
                assert (q[i, 0], q[i, 1]) == (fx, fy), (sig, th, i)
                margin = min(margin, vx - fx, fx + 1 - vx, vy - fy, fy + 1 - vy)
    assert margin > 1e-12


def test_scaled_volume_matches_brute_force(oracle_mod):
    O = oracle_mod
    for trial in range(2):
        rng = _rng(10 + trial)
        mimg = np.full((10, 10), 40, np.uint8)
        mimg[2:7, 2:6] = 200
        mimg[7, 6:9] = 130
        simg = rng.integers(0, 256, (22, 24), dtype=np.uint8)
        simg[6:16, 8:18] = np.rot90(mimg, trial)
        M = O.build_model(mimg, O.PyrParams(1, 30.0))
        ml = M.levels[0]
        bt, bd = BF.model(mimg, 30.0)
        g = O.edge_field(simg, 60.0)
        thetas = [O.theta(0.0, 20.0, k) for k in range(18)]
        sigmas = [O.scale(0.75, 0.25, j) for j in range(3)]
        vols = [BF.score_volume(g, bt, bd, thetas, sigma=sg) for sg in sigmas]
        Sw = np.concatenate([v[0] for v in vols])  # index m = j K + k
        S1 = np.concatenate([v[1] for v in vols])
        for m in range(0, 54, 7):
            j, k = divmod(m, 18)
            for (x, y) in [(0, 0), (5, 7), (12, 10), (23, 21), (10, 3)]:
                a = O.score(g, ml.t, ml.d, x, y, thetas[k], sigma=sigmas[j])
                assert abs(a[0] - Sw[m, y, x]) <= 1e-12 and abs(a[1] - S1[m, y, x]) <= 1e-12
        mw, m1, mk = O.top_map_sim(g, ml.t, ml.d, 0.0, 20.0, 18, 0.75, 0.25, 3, nthreads=2)
        assert np.allclose(mw, Sw.max(axis=0), atol=1e-12)
        ys, xs = np.mgrid[0:22, 0:24]
        assert np.allclose(Sw[mk, ys, xs], mw, atol=1e-12) and np.allclose(S1[mk, ys, xs], m1, atol=1e-12)
        best1 = np.where(np.abs(Sw - mw[None]) <= 1e-12, S1, -np.inf).max(axis=0)
        assert np.allclose(m1, best1, atol=1e-12)
        # the chosen index is one of the keys' best (ties within rounding:
        # either member); where the best is unique it is that one
        tie = (np.abs(Sw - mw[None]) <= 1e-12) & (np.abs(S1 - m1[None]) <= 1e-12)
        assert np.all(tie[mk, ys, xs])
        one = tie.sum(axis=0) == 1
        assert np.array_equal(mk[one], np.argmax(tie, axis=0)[one])


@pytest.mark.parametrize("sigma,theta", [(1.2, 40.0), (0.9, 250.0)])
def test_scaled_instance_is_found_at_its_scale(oracle_mod, sigma, theta):
    O = oracle_mod
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(20211200 + 7, spawn_key=(10**6,))))
    shape = synth.make_model_shape("polygon", 128, rng)
    model = synth.render_model(shape, 128)
    img = synth.render_posed(shape, 320, 240, 160.0, 120.0, theta, sigma)
    sp = O.SearchParams(theta_step_top=2.0, scale_min=0.8, scale_step=0.1, scale_count=5, max_matches=1)
    tr = O.detect(img, model, O.PyrParams(3, 30.0), O.PyrParams(3, 30.0), sp)
    d = tr.detections[0]
    assert abs(d.scale - sigma) <= 1e-9, d
    assert abs(d.x - 160) <= 1 and abs(d.y - 120) <= 1, d
    assert abs((d.theta - theta + 180) % 360 - 180) <= 1.0, d
    assert d.sw > 0.9


@pytest.mark.parametrize("j", [0, 2])
def test_refine_sim_picks_best_of_27_by_bruteforce(oracle_mod, j):
    """O15 at a scale other than 1: each candidate (x, y, m = j K' + k) of the
    level above moves to the best by the key of the 27 poses (2x + a, 2y + b,
    2k + c) at its own scale sigma_j, the scores taken from the independent
    NumPy brute force (tests/bruteforce.py) at that scale."""
    O = oracle_mod
    rng = _rng(60 + j)
    img = rng.integers(0, 256, (30, 34), dtype=np.uint8)
    mimg = np.full((9, 9), 40, np.uint8)
    mimg[2:6, 2:7] = 210
    mimg[6, 3:8] = 120
    bt, bd = BF.model(mimg, 30.0)
    M = O.build_model(mimg, O.PyrParams(1, 30.0))
    g = BF.field(img, 50.0)
    K, step = 48, 7.5            # this level's grid; the level above has K / 2 angles
    K_above = K // 2
    sigma_min, sigma_step = 0.8, 0.25
    sigma = O.scale(sigma_min, sigma_step, j)
    assert sigma != 1.0
    cx = np.array([0, 8, 16], np.int32)
    cy = np.array([0, 7, 14], np.int32)
    ck = np.array([0, 11, 23], np.int32)
    cands = O.Candidates(cx, cy, (j * K_above + ck).astype(np.int32), np.zeros(3), np.zeros(3))
    out = O.refine_level_sim(g, M.levels[0], cands, 0.0, step, K, K_above, True, 3, sigma_min, sigma_step)
    thetas = [O.theta(0.0, step, k) for k in range(K)]
    Sw, S1 = BF.score_volume(g, bt, bd, thetas, sigma=sigma)
    for c in range(3):
        best = None
        for dk in (-1, 0, 1):
            k = (2 * int(ck[c]) + dk) % K
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    x, y = 2 * int(cx[c]) + a, 2 * int(cy[c]) + b
                    if not (0 <= x < 34 and 0 <= y < 30):
                        continue
                    key = (-Sw[k, y, x], -S1[k, y, x], x, y, k)
                    best = key if best is None or key < best else best
        assert (int(out.x[c]), int(out.y[c])) == best[2:4]
        assert int(out.k[c]) == j * K + best[4]  # the key's last component: m = j K + k
        assert abs(out.sw[c] + best[0]) <= 1e-12 and abs(out.s1[c] + best[1]) <= 1e-12
