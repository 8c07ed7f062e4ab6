"""Continuous (bilinear) score and its gradient: HIP kernels through the C
ABI against the FP64 oracle on the same seeded poses.

Bars: S_c within 1e-5 (FP32 field, FP32 sums); gradient within 5e-5 + 1e-5
|ref| per component; FP16 fields within 2 * 2^-11 + 2e-5 (one FP16 rounding
of each interpolated component); the FP64 line search picks a step whose
oracle score is within 1e-6 of the best step's (the field itself is FP32)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL16 = 2 * 2.0 ** -11 + 2e-5


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05576_amd as P

    P.lib()
    return P


def _P():
    import paper_2112_05576_amd as P

    return P


def _setup(level, precision=0, index=0):
    P = _P()
    sc = synth.scene_for_config(2, index)
    cfg = sc.config
    L = cfg["levels"]
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=precision)
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, L, cfg["tau_s"])[level]
    return sc, gm, pyr, om.levels[level], g


def _poses(sc, level, g, n, seed):
    """FP32 poses: near the instances, anywhere in the image, and outside."""
    rng = np.random.default_rng(seed)
    H, W, _ = g.shape
    s = 2.0 ** -level
    out = []
    for i in range(n):
        if i % 3 == 0 and sc.instances:
            it = sc.instances[(i // 3) % len(sc.instances)]
            out.append((it.x * s + rng.uniform(-1.5, 1.5), it.y * s + rng.uniform(-1.5, 1.5),
                        it.theta + rng.uniform(-3, 3)))
        elif i % 3 == 1:
            out.append((rng.uniform(0, W), rng.uniform(0, H), rng.uniform(-360, 720)))
        else:
            out.append((rng.uniform(-60, W + 60), rng.uniform(-60, H + 60), rng.uniform(0, 360)))
    return np.array(out, np.float32)


def _off_cell_edges(ml, x, y, th, eps=1e-7):
    """True when no projected point lies within eps of a pixel-cell edge, so
    that FP64 rounding differences cannot select another cell's derivative."""
    c, s = np.cos(np.deg2rad(th)), np.sin(np.deg2rad(th))
    p = ml.t @ np.array([[c, -s], [s, c]]).T + [x, y]
    f = p - np.floor(p)
    return np.min(np.minimum(f, 1 - f)) > eps


def _oracle(g, ml, poses):
    S = np.empty(len(poses))
    G = np.empty((len(poses), 3))
    for i, (x, y, th) in enumerate(poses.astype(np.float64)):
        S[i], G[i] = O.cont_score(g, ml.t, ml.d, x, y, th)
    return S, G


@pytest.mark.parametrize("level", [0, 1, 3])
def test_cont_score_and_gradient(level):
    P = _P()
    case(f"cont_score C2 level={level}")
    sc, gm, pyr, ml, g = _setup(level)
    poses = _poses(sc, level, g, 240, 100 + level)
    S, G = _oracle(g, ml, poses)
    t = torch.from_numpy(poses).cuda()
    got = P.cont_score(gm, pyr, level, t).cpu().numpy().astype(np.float64)
    err = np.abs(got - S).max()
    print(f"score: max |err| = {err:.3g}, max S_c {S.max():.4f}")
    assert err <= TOL
    gg = P.cont_score_backward(gm, pyr, level, t).cpu().numpy().astype(np.float64)
    keep = np.array([_off_cell_edges(ml, *p) for p in poses.astype(np.float64)])
    assert keep.sum() >= 200
    gerr = np.abs(gg - G)[keep]
    print(f"gradient: max |err| = {gerr.max():.3g}, max |grad| {np.abs(G).max():.3g}")
    assert np.all(gerr <= 5e-5 + 1e-5 * np.abs(G[keep]))


def test_cont_score_fp16():
    P = _P()
    case("cont_score FP16 C2 level 1")
    sc, gm, pyr, ml, g = _setup(1, precision=P.TM_FP16)
    poses = _poses(sc, 1, g, 150, 120)
    S, G = _oracle(g, ml, poses)
    got = P.cont_score(gm, pyr, 1, torch.from_numpy(poses).cuda()).cpu().numpy().astype(np.float64)
    assert np.abs(got - S).max() <= TOL16


def test_cont_autograd_weights_the_gradient():
    P = _P()
    case("ContinuousScore autograd")
    sc, gm, pyr, ml, g = _setup(0)
    poses = _poses(sc, 0, g, 60, 130)
    S, G = _oracle(g, ml, poses)
    keep = np.array([_off_cell_edges(ml, *p) for p in poses.astype(np.float64)])
    w = np.random.default_rng(131).uniform(-2, 2, len(poses)).astype(np.float32)
    p = torch.from_numpy(poses).cuda().requires_grad_(True)
    s = P.ContinuousScore.apply(p, gm, pyr, 0)
    (s * torch.from_numpy(w).cuda()).sum().backward()
    got = p.grad.cpu().numpy().astype(np.float64)
    ref = w[:, None].astype(np.float64) * G
    assert np.all(np.abs(got - ref)[keep] <= 2 * (5e-5 + 1e-5 * np.abs(ref[keep])))


def test_cont_line_search_picks_best_step():
    P = _P()
    case("cont_line_search C2 level 0")
    sc, gm, pyr, ml, g = _setup(0)
    poses = _poses(sc, 0, g, 90, 140)
    rng = np.random.default_rng(141)
    dirs = rng.normal(size=(len(poses), 3)).astype(np.float32)
    alphas = [0.0, 0.1, -0.1, 0.5, 1.0, 2.5, -1.0]
    newp, sc_ = P.cont_line_search(gm, pyr, 0, torch.from_numpy(poses).cuda(), torch.from_numpy(dirs).cuda(),
                                   alphas)
    newp = newp.cpu().numpy()
    sc_ = sc_.cpu().numpy().astype(np.float64)
    for i in range(len(poses)):
        cands = [(poses[i].astype(np.float64) + a * dirs[i].astype(np.float64)).astype(np.float32) for a in alphas]
        ref = [O.cont_score(g, ml.t, ml.d, *c.astype(np.float64))[0] for c in cands]
        hit = [j for j, c in enumerate(cands) if np.array_equal(c, newp[i])]
        assert hit, (i, newp[i], cands)
        assert max(ref[j] for j in hit) >= max(ref) - 1e-6
        assert abs(sc_[i] - max(ref[j] for j in hit)) <= 1e-6


def test_refine_continuous_never_lowers_the_score():
    P = _P()
    case("refine_continuous C2 image 0")
    sc, gm, pyr, ml, g = _setup(0)
    dets = P.detect(gm, pyr, P.SearchParams(theta_step_top=1.0))
    assert len(dets) >= 1
    start = np.array([(d["x"], d["y"], d["theta"]) for d in dets], np.float32)
    S0, _ = _oracle(g, ml, start)
    newp, s = P.refine_continuous(gm, pyr, torch.from_numpy(start).cuda())
    newp = newp.cpu().numpy()
    s = s.cpu().numpy().astype(np.float64)
    S1, _ = _oracle(g, ml, newp)
    print(f"S_c {np.round(S0, 4)} -> {np.round(S1, 4)}")
    assert np.all(S1 >= S0 - 1e-6)
    assert np.abs(s - S1).max() <= 1e-6
    # nothing moves further than the sum of its step bounds
    assert np.abs(newp[:, :2] - start[:, :2]).max() <= 2 * 0.5 / (1 - 0.6) + 1e-3
