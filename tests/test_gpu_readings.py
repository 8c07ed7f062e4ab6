"""The two switchable readings on the GPU, against the oracle on the same
seeded inputs: the gradient-map pyramid (TM_PYR_GRADIENT: Sobel pair of the
full image, then floored 2x2 means of the gradient maps) and the
edge-taps-only window (TM_VOTE_EDGE: only edge pixels of a window vote, a
window without one votes 0).

Bars as for the default readings: bit-exact edge masks, model points and
integer gradients; directions within FP32 rounding; scores within 1e-5
(FP32) or the FP16 bound 2 * 2^-11 + 2e-5; chosen poses equal to the
oracle's or an oracle tie within the bar; the batch, the graph replay and the
staged refinement bit-identical to the single-image gathers."""
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


@pytest.mark.parametrize("H,W,L,tau", [(480, 640, 4, 80.0), (211, 333, 3, 45.5), (24, 40, 4, 20.0)])
def test_gradient_pyramid_fields(H, W, L, tau):
    P = _P()
    case(f"gradient pyramid {W}x{H} L={L} tau={tau}")
    rng = np.random.default_rng(8100 + H)
    sh = synth.make_model_shape("polygon", 96, rng)
    img = synth.render_scene(rng, W, H, sh, 96, 1 if min(H, W) > 110 else 0, 6.0, 0.2, (0.7, 1.4), (-20, 20),
                             clutter=20).image
    ref = O.field_pyramid(img, L, tau, "gradient")
    for prec in (P.TM_FP32, P.TM_FP16):
        pyr = P.Pyramid(img, L, tau, precision=prec, source=P.TM_PYR_GRADIENT)
        for l in range(L):
            _, gf = pyr.read(l)
            gf = gf.cpu().numpy().astype(np.float64)
            of = ref[l]
            assert np.array_equal(np.any(gf != 0, -1), np.any(of != 0, -1)), (prec, l)
            if prec == P.TM_FP32:
                assert np.array_equal(gf, of.astype(np.float32).astype(np.float64)), l
            else:
                assert np.array_equal(gf, of.astype(np.float32).astype(np.float16).astype(np.float64)), l
    # the levels differ from the grey reading's above level 0
    grey = O.field_pyramid(img, L, tau, "grey")
    assert np.array_equal(grey[0], ref[0]) and (L == 1 or not np.array_equal(grey[1], ref[1]))


@pytest.mark.parametrize("ci", [1, 2])
def test_gradient_model_points(ci):
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    case(f"gradient model C{ci} L={L}")
    gm = P.Model(sc.model, L, cfg["tau_m"], source=P.TM_PYR_GRADIENT)
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"], "gradient"))
    gp = O.gradient_pyramid(sc.model, L)
    for l in range(L):
        t, g = gm.points(l)
        t = t.cpu().numpy()
        g = g.cpu().numpy()
        ml = om.levels[l]
        assert np.array_equal(t, ml.t), l
        ys, xs = ml.t[:, 1] + ml.height // 2, ml.t[:, 0] + ml.width // 2
        assert np.array_equal(g[:, 0], gp[l][0][ys, xs]) and np.array_equal(g[:, 1], gp[l][1][ys, xs]), l


@pytest.mark.parametrize("ci,level,win,prec", [(1, 0, 3, 0), (1, 0, 5, 0), (2, 2, 3, 0), (2, 0, 3, 1), (2, 1, 1, 0)])
def test_score_poses_edge_vote(ci, level, win, prec):
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    case(f"score_poses edge vote C{ci} level={level} win={win} prec={prec}")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=prec)
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, L, cfg["tau_s"])[level]
    H, W, _ = g.shape
    rng = np.random.default_rng(31 + level)
    n = 300
    xs = rng.integers(-12, W + 12, n)
    ys = rng.integers(-12, H + 12, n)
    th = rng.uniform(-400.0, 400.0, n)
    got = P.score_poses(gm, pyr, level, xs, ys, th, win, vote=P.TM_VOTE_EDGE).cpu().numpy().astype(np.float64)
    ml = om.levels[level]
    ref = np.array([O.score(g, ml.t, ml.d, int(xs[i]), int(ys[i]), float(th[i]), win, vote="edge")
                    for i in range(n)])
    allv = np.array([O.score(g, ml.t, ml.d, int(xs[i]), int(ys[i]), float(th[i]), win) for i in range(n)])
    err = np.abs(got - ref).max()
    print(f"max |err| = {err:.3g}; poses where the readings differ: {(ref[:, 0] < allv[:, 0]).sum()}")
    assert err <= (TOL16 if prec else TOL)
    assert win == 1 or (ref[:, 0] < allv[:, 0] - 1e-3).sum() > 20  # the reading is exercised


def _check_map(got, ref, g, ml, step, tol):
    """S_w is the maximum over angles, so it stays within the bar even where
    another angle wins; S_1 belongs to the winning angle: compared where the
    angles agree, and against the oracle at the GPU's angle where they do not
    (which must then be an oracle tie within two bars)."""
    sw, s1, k = [t.cpu().numpy() for t in got]
    mw, m1, mk = ref
    same = k == mk
    ew, e1 = np.abs(sw - mw).max(), np.abs(s1 - m1)[same].max()
    diff = np.argwhere(~same)
    print(f"map {sw.shape}: max |dS_w| {ew:.3g}; max |dS_1| (same angle) {e1:.3g}; "
          f"angle differs at {len(diff)} of {k.size}")
    assert ew <= tol and e1 <= tol
    for (j, i) in diff:
        a = O.score(g, ml.t, ml.d, int(i), int(j), O.theta(0.0, step, int(k[j, i])), vote="edge")
        assert abs(a[0] - mw[j, i]) <= 2 * tol, (i, j, k[j, i], mk[j, i])
        assert abs(a[0] - sw[j, i]) <= tol and abs(a[1] - s1[j, i]) <= tol, (i, j)


@pytest.mark.parametrize("ci,prec", [(1, 0), (2, 0), (2, 1)])
def test_score_map_edge_vote(ci, prec):
    """The fast search kernel (window 3, unit steps) under the edge reading."""
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    top = L - 1
    step = cfg["theta_step_top"] if ci != 1 else 5.0
    case(f"score_map edge vote C{ci} prec={prec}")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=prec)
    got = P.score_map(gm, pyr, top, P.SearchParams(theta_step_top=step, vote=P.TM_VOTE_EDGE))
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, L, cfg["tau_s"])[top]
    ml = om.levels[top]
    K = int(np.ceil(360.0 / step))
    ref = O.top_map(g, ml.t, ml.d, 0.0, step, K, vote="edge")
    _check_map(got, ref, g, ml, step, TOL16 if prec else TOL)


def test_score_map_edge_vote_generic_path():
    """Steps > 1 and a 5-pixel window go through the generic kernel."""
    P = _P()
    case("score_map edge vote generic")
    rng = np.random.default_rng(8200)
    shape = synth.make_model_shape("blocks", 24, rng)
    model = synth.render_model(shape, 24)
    sc = synth.render_scene(rng, 67, 61, shape, 24, 1, 5.0, clutter=6)
    gm = P.Model(model, 1, 30.0)
    pyr = P.Pyramid(sc.image, 1, 60.0)
    for sx, sy, win in ((2, 3, 3), (1, 1, 5)):
        sp = P.SearchParams(step_x=sx, step_y=sy, neighbourhood=win, theta_step_top=7.5, vote=P.TM_VOTE_EDGE)
        sw, s1, k = [t.cpu().numpy() for t in P.score_map(gm, pyr, 0, sp)]
        om = O.build_model(model, O.PyrParams(1, 30.0))
        g = O.edge_field(sc.image, 60.0)
        mw, m1, mk = O.top_map(g, om.levels[0].t, om.levels[0].d, 0.0, 7.5, 48, sx, sy, win, vote="edge")
        assert np.abs(sw - mw).max() <= TOL and np.abs(s1 - m1).max() <= TOL, (sx, sy, win)


def _match(got, tr, osp, L, tol):
    ref = tr.detections
    assert len(got) == len(ref), (len(got), len(ref))
    ties = 0
    for g, r in zip(got, ref):
        if (int(g["x"]), int(g["y"]), int(g["k"])) == (r.x, r.y, r.k):
            assert abs(g["sw"] - r.sw) <= tol and abs(g["s1"] - r.s1) <= tol
            continue
        ml = tr.model.levels[0]
        a = O.score(tr.fields[0], ml.t, ml.d, int(g["x"]), int(g["y"]),
                    O.theta(0.0, O.level_step(osp, L, 0), int(g["k"])), vote=osp.vote)
        assert abs(a[0] - r.sw) <= 2 * tol and abs(a[1] - r.s1) <= 2 * tol, (g, r)
        ties += 1
    return ties


@pytest.mark.parametrize("source,vote,prec,index", [("gradient", "all", 0, 0), ("grey", "edge", 0, 1),
                                                    ("gradient", "edge", 0, 1), ("gradient", "edge", 1, 0)])
def test_detect_with_readings(source, vote, prec, index):
    P = _P()
    sc = synth.scene_for_config(2, index)
    cfg = sc.config
    L = cfg["levels"]
    case(f"detect C2 image {index} source={source} vote={vote} prec={prec}")
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"], vote=vote)
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"], source), O.PyrParams(L, cfg["tau_m"], source), osp)
    src = P.TM_PYR_GRADIENT if source == "gradient" else P.TM_PYR_GREY
    gm = P.Model(sc.model, L, cfg["tau_m"], source=src)
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=prec, source=src)
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"], vote=P.TM_VOTE_EDGE if vote == "edge" else 0)
    got = P.detect(gm, pyr, sp)
    if prec == 0:
        ties = _match(got, tr, osp, L, TOL)
        print(f"{len(got)} detections, {ties} ties")
    else:  # FP16: the top match, or a tie within the FP16 bound
        assert len(got) >= 1 and len(tr.detections) >= 1
        g, r = got[0], tr.detections[0]
        ml = tr.model.levels[0]
        a = O.score(tr.fields[0], ml.t, ml.d, int(g["x"]), int(g["y"]), float(g["theta"]), vote=vote)
        assert abs(a[0] - r.sw) <= 2 * TOL16 and abs(float(g["sw"]) - a[0]) <= TOL16, (g, r, a)
    near = [i for i in sc.instances if abs(i.x - got[0]["x"]) <= 2 and abs(i.y - got[0]["y"]) <= 2]
    assert near


def _poses_equal(a, b):
    return len(a) == len(b) and all(
        (int(x["x"]), int(x["y"]), int(x["k"]), float(x["sw"]), float(x["s1"])) ==
        (int(y["x"]), int(y["y"]), int(y["k"]), float(y["sw"]), float(y["s1"])) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_graph_with_readings_equals_single(precision):
    """Gradient pyramids and the edge vote through the batch (staged
    refinement: 18 pairs x 32 candidates) and its graph replays, against
    single-image calls (gathered refinement): identical poses and scores."""
    P = _P()
    case(f"batch graph gradient+edge precision={precision}")
    cfg = synth.CONFIGS[2]
    scenes = [synth.scene_for_config(2, i) for i in range(8)]
    big = synth.scene_for_config(2, 7, W=1280, H=1024, n_inst=4)
    rng = np.random.default_rng(4243)
    m2 = synth.render_model(synth.make_model_shape("polygon", 96, rng), 96)
    src = P.TM_PYR_GRADIENT
    models = [P.Model(scenes[0].model, 4, cfg["tau_m"], source=src), P.Model(m2, 4, cfg["tau_m"], source=src)]
    images = [torch.from_numpy(s.image).cuda() for s in scenes] + [torch.from_numpy(big.image).cuda()]
    sp = P.SearchParams(theta_step_top=1.0, vote=P.TM_VOTE_EDGE)
    b = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=precision, source=src)
    b.run()
    eager = b.results()
    for i, im in enumerate(images):
        pyr = P.Pyramid(im, 4, cfg["tau_s"], precision=precision, source=src)
        for j, m in enumerate(models):
            ref = P.detect(m, pyr, sp)
            assert _poses_equal(eager[i * 2 + j], ref), (i, j)
    for rep in range(3):
        b.run(graph=True)
        torch.cuda.synchronize()
        assert all(_poses_equal(x, y) for x, y in zip(b.results(), eager)), rep
    print(f"{sum(len(r) for r in eager)} detections over {len(eager)} pairs")


@pytest.mark.parametrize("prec", [0, 1])
def test_edge_vote_search_forms_bit_identical(prec, monkeypatch):
    """The edge-taps search in every launch shape it has (orientation, waves
    per chunk, angles per wave) gives the same bits; in FP16 its products
    carry the per-pixel addend through v_dot2_f32_f16, whose result is read
    only after the hazard wait, which a mismatch between shapes would show."""
    P = _P()
    sc = synth.scene_for_config(2, 3)
    cfg = sc.config
    case(f"edge-vote search forms prec={prec}")
    gm = P.Model(sc.model, 4, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, 4, cfg["tau_s"], precision=prec)
    sp = P.SearchParams(theta_step_top=1.0, vote=P.TM_VOTE_EDGE)
    ref = [t.clone() for t in P.score_map(gm, pyr, 3, sp)]
    for tr, wa, apw in [(0, 4, 1), (1, 16, 1), (0, 2, 3), (1, 8, 2), (1, 1, 1)]:
        monkeypatch.setenv("TM_DENSE_TR", str(tr))
        monkeypatch.setenv("TM_DENSE_WA", str(wa))
        monkeypatch.setenv("TM_DENSE_APW", str(apw))
        got = P.score_map(gm, pyr, 3, sp)
        assert all(torch.equal(x, y) for x, y in zip(ref, got)), (tr, wa, apw)
