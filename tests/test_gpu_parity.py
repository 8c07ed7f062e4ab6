"""GPU (HIP library, through the C ABI) against the FP64 oracle on the same
seeded inputs.

Bars: bit-exact uint8 pyramid levels, edge masks, model points and rotated
position offsets; directions within FP32 rounding; scores within 1e-5
absolute (FP32 path); the chosen angle / pose equal to the oracle's or, where
several are correct, one whose oracle key lies within 1e-5 of the oracle's
best (a tie at FP32 resolution)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05576_amd as P

    P.lib()  # raises if the HIP library is missing
    return P


def _P():
    import paper_2112_05576_amd as P

    return P


def _scene_img(H, W, seed):
    rng = np.random.default_rng(seed)
    sh = synth.make_model_shape("polygon", 96, rng)
    sc = synth.render_scene(rng, W, H, sh, 96, 1 if min(H, W) > 110 else 0, 6.0, 0.2, (0.7, 1.4), (-20, 20),
                            clutter=20)
    return sc.image


# ------------------------------------------------------------ pyramid, edges
@pytest.mark.parametrize("H,W,L,tau,pad", [(128, 128, 1, 30.0, 0), (480, 640, 4, 80.0, 0), (211, 333, 3, 45.5, 13),
                                           (2048, 2048, 5, 80.0, 0), (24, 40, 4, 20.0, 5)])
def test_pyramid_and_edges(H, W, L, tau, pad):
    P = _P()
    case(f"pyramid {W}x{H} L={L} tau={tau} pad={pad}")
    img = _scene_img(H, W, 7000 + H + W)
    big = np.zeros((H, W + pad), np.uint8)
    big[:, :W] = img
    dev = torch.from_numpy(big).cuda()[:, :W]
    pyr = P.Pyramid(dev, L, tau)
    ref_levels = O.pyramid(img, L)
    for l in range(L):
        gi, gf = pyr.read(l)
        gi = gi.cpu().numpy()
        gf = gf.cpu().numpy().astype(np.float64)
        assert np.array_equal(gi, ref_levels[l]), f"level {l} pixels"
        of = O.edge_field(ref_levels[l], tau)
        assert np.array_equal(np.any(gf != 0, -1), np.any(of != 0, -1)), f"level {l} edge mask"
        # the FP32 directions are the FP32 rounding of the oracle's FP64 ones, bit for bit
        assert np.array_equal(gf.astype(np.float32), of.astype(np.float32)), f"level {l} directions"


def test_pyramid_update_reuses_storage():
    P = _P()
    case("pyramid update")
    a = _scene_img(96, 128, 1)
    b = _scene_img(96, 128, 2)
    pyr = P.Pyramid(a, 3, 40.0)
    pyr.update(torch.from_numpy(b).cuda())
    for l, lv in enumerate(O.pyramid(b, 3)):
        assert np.array_equal(pyr.read(l)[0].cpu().numpy(), lv)


# ------------------------------------------------------------ model, tables
@pytest.mark.parametrize("ci", [1, 2, 3])
def test_model_points_and_tables(ci):
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    case(f"model C{ci} L={L}")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    for l in range(L):
        t, g = gm.points(l)
        t = t.cpu().numpy()
        g = g.cpu().numpy().astype(np.float64)
        assert np.array_equal(t, om.levels[l].t), f"level {l} t"
        d = g / np.hypot(g[:, 0], g[:, 1])[:, None]
        assert np.abs(d - om.levels[l].d).max() <= 1e-15
    sp = O.SearchParams(theta_step_top=cfg["theta_step_top"], theta_range=cfg["theta_range"])
    for l in sorted({L - 1, 0}):
        st = O.level_step(sp, L, l)
        K = O.level_count(sp, st)
        q, r = gm.table(l, 0.0, st, K)
        q = q.cpu().numpy()
        r = r.cpu().numpy().astype(np.float64)
        ks = range(K) if l == L - 1 else np.random.default_rng(3).choice(K, 40, replace=False)
        ml = om.levels[l]
        for k in ks:
            oq, orr = O.rotate(ml.t, ml.d, O.theta(0.0, st, int(k)))
            assert np.array_equal(q[k], oq), f"level {l} angle {k} q"
            assert np.abs(r[k] - orr).max() <= 6e-8


# ------------------------------------------------------------ scores
@pytest.mark.parametrize("ci,level,win", [(1, 0, 3), (1, 0, 1), (1, 0, 5), (2, 2, 3), (2, 0, 3), (3, 4, 3)])
def test_score_poses(ci, level, win):
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    case(f"score_poses C{ci} level={level} win={win}")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, L, cfg["tau_s"])[level]
    H, W, _ = g.shape
    rng = np.random.default_rng(11 + level)
    n = 300
    xs = rng.integers(-12, W + 12, n)
    ys = rng.integers(-12, H + 12, n)
    th = rng.uniform(-400.0, 400.0, n)
    th[:8] = [0.0, 90.0, 180.0, 270.0, 30.0, 45.0, 60.0, -90.0]
    for i, it in enumerate(sc.instances[:3]):  # poses on the instances score high
        s = 2.0 ** -level
        xs[8 + i], ys[8 + i], th[8 + i] = int(round(it.x * s)), int(round(it.y * s)), it.theta
    got = P.score_poses(gm, pyr, level, xs, ys, th, win).cpu().numpy().astype(np.float64)
    ml = om.levels[level]
    ref = np.array([O.score(g, ml.t, ml.d, int(xs[i]), int(ys[i]), float(th[i]), win) for i in range(n)])
    err = np.abs(got - ref).max()
    print(f"max |err| = {err:.3g}, max score {ref[:, 0].max():.3f}")
    assert err <= TOL


def _check_map(gm_map, om_map, g, ml, theta_min, step, sx, sy, win):
    """S_w, S_1 within TOL everywhere; the angle equal or an oracle tie."""
    sw, s1, k = [t.cpu().numpy() for t in gm_map]
    mw, m1, mk = om_map
    assert sw.shape == mw.shape
    ew, e1 = np.abs(sw - mw).max(), np.abs(s1 - m1).max()
    print(f"map {sw.shape}: max |dS_w| {ew:.3g} |dS_1| {e1:.3g}")
    assert ew <= TOL and e1 <= TOL
    diff = np.argwhere(k != mk)
    for (j, i) in diff:
        a = O.score(g, ml.t, ml.d, int(i * sx), int(j * sy), O.theta(theta_min, step, int(k[j, i])), win)
        assert abs(a[0] - mw[j, i]) <= TOL and abs(a[1] - m1[j, i]) <= TOL, (i, j, k[j, i], mk[j, i])
    print(f"angle differs at {len(diff)} of {k.size} translations (all ties)")


@pytest.mark.parametrize("ci,step_top", [(1, 5.0), (2, 1.0), (3, 8.0)])
def test_score_map_top_level(ci, step_top):
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    top = L - 1
    case(f"score_map C{ci} top level {top}")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
    sp = P.SearchParams(theta_step_top=step_top)
    got = P.score_map(gm, pyr, top, sp)
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, L, cfg["tau_s"])[top]
    ml = om.levels[top]
    K = int(np.ceil(360.0 / step_top))
    ref = O.top_map(g, ml.t, ml.d, 0.0, step_top, K)
    _check_map(got, ref, g, ml, 0.0, step_top, 1, 1, 3)


@pytest.mark.parametrize("H,W,sx,sy,win,rng_deg", [(61, 67, 1, 1, 3, 360.0), (64, 60, 2, 3, 3, 360.0),
                                                   (50, 53, 1, 1, 5, 90.0), (45, 47, 3, 3, 1, 360.0),
                                                   (40, 201, 1, 1, 3, 360.0)])
def test_score_map_shapes_and_paths(H, W, sx, sy, win, rng_deg):
    """Ragged tile tails, the generic path (steps > 1, other windows), a
    partial angle range."""
    P = _P()
    case(f"score_map {W}x{H} step=({sx},{sy}) win={win} range={rng_deg}")
    rng = np.random.default_rng(900 + H)
    shape = synth.make_model_shape("blocks", 24, rng)
    model = synth.render_model(shape, 24)
    sc = synth.render_scene(rng, W, H, shape, 24, 1, 5.0, clutter=6)
    gm = P.Model(model, 1, 30.0)
    pyr = P.Pyramid(sc.image, 1, 30.0)
    step = 7.5
    sp = P.SearchParams(step_x=sx, step_y=sy, neighbourhood=win, theta_step_top=step, theta_min=-20.0,
                        theta_range=rng_deg)
    got = P.score_map(gm, pyr, 0, sp)
    om = O.build_model(model, O.PyrParams(1, 30.0))
    g = O.edge_field(sc.image, 30.0)
    ml = om.levels[0]
    osp = O.SearchParams(theta_step_top=step, theta_range=rng_deg)
    K = O.level_count(osp, step)
    ref = O.top_map(g, ml.t, ml.d, -20.0, step, K, sx, sy, win)
    _check_map(got, ref, g, ml, -20.0, step, sx, sy, win)
    # FP16 fields through the same path: S_w within the FP16 bound everywhere
    # (a maximum over angles); S_1 where the angle agrees, else the oracle at
    # the GPU's angle, which must tie the oracle's best within two bounds
    tol16 = 2 * 2.0 ** -11 + 2e-5
    pyr16 = P.Pyramid(sc.image, 1, 30.0, precision=P.TM_FP16)
    sw, s1, k = [t.cpu().numpy() for t in P.score_map(gm, pyr16, 0, sp)]
    mw, m1, mk = ref
    same = k == mk
    assert np.abs(sw - mw).max() <= tol16 and np.abs(s1 - m1)[same].max() <= tol16
    for (j, i) in np.argwhere(~same):
        a = O.score(g, ml.t, ml.d, int(i * sx), int(j * sy), O.theta(-20.0, step, int(k[j, i])), win)
        assert abs(a[0] - mw[j, i]) <= 2 * tol16 and abs(a[1] - s1[j, i]) <= tol16, (i, j)


# ------------------------------------------------------------ selection
def test_select_golden_cases():
    import json
    import os

    P = _P()
    cases = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "select_cases.json")))
    for c in cases["select"]:
        case(f"select {c['name']}")
        sw = torch.tensor(c["mw"], dtype=torch.float32).cuda()
        s1 = torch.tensor(c["m1"], dtype=torch.float32).cuda()
        k = torch.tensor(c["mk"], dtype=torch.int32).cuda()
        out, n = P.select(sw, s1, k, c["sx"], c["sy"], c["level"], c["min_score"], c["dmin"], c["max_out"])
        got = P.poses_to_numpy(out, int(n.item()))
        assert len(got) == len(c["expect"]), c["name"]
        for g, e in zip(got, c["expect"]):
            assert (g["x"], g["y"], g["k"]) == tuple(e[:3]), c["name"]
            assert g["sw"] == np.float32(e[3]) and g["s1"] == np.float32(e[4])


@pytest.mark.parametrize("seed,dmin,cap", [(0, 12.0, 32), (1, 0.0, 1024), (2, 40.0, 5)])
def test_select_on_oracle_maps(seed, dmin, cap):
    """The same FP32 map into both selections: identical candidate lists."""
    P = _P()
    case(f"select on C2 map seed={seed} dmin={dmin} cap={cap}")
    sc = synth.scene_for_config(2, seed)
    cfg = sc.config
    om = O.build_model(sc.model, O.PyrParams(4, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, 4, cfg["tau_s"])[3]
    ml = om.levels[3]
    mw, m1, mk = O.top_map(g, ml.t, ml.d, 0.0, 4.0, 90)
    mw32, m132 = mw.astype(np.float32), m1.astype(np.float32)
    ref = O.select(mw32.astype(np.float64), m132.astype(np.float64), mk, 1, 1, 3, 0.3, dmin, cap)
    out, n = P.select(torch.from_numpy(mw32).cuda(), torch.from_numpy(m132).cuda(),
                      torch.from_numpy(mk).cuda(), 1, 1, 3, 0.3, dmin, cap)
    got = P.poses_to_numpy(out, int(n.item()))
    print(f"{len(ref)} candidates")
    assert len(got) == len(ref) and len(ref) > 0
    assert np.array_equal(got["x"], ref.x) and np.array_equal(got["y"], ref.y) and np.array_equal(got["k"], ref.k)
    assert np.array_equal(got["sw"], ref.sw.astype(np.float32))


def test_select_large_candidate_count():
    """More local maxima than the in-LDS sort holds: the global-memory path."""
    P = _P()
    case("select with > 2048 local maxima")
    rng = np.random.default_rng(5)
    gh, gw = 160, 200
    mw = rng.random((gh, gw)).astype(np.float32)
    m1 = rng.random((gh, gw)).astype(np.float32)
    mk = rng.integers(0, 50, (gh, gw)).astype(np.int32)
    ref = O.select(mw.astype(np.float64), m1.astype(np.float64), mk, 2, 2, 1, 0.0, 3.0, 1024)
    out, n = P.select(torch.from_numpy(mw).cuda(), torch.from_numpy(m1).cuda(), torch.from_numpy(mk).cuda(), 2, 2,
                      1, 0.0, 3.0, 1024)
    got = P.poses_to_numpy(out, int(n.item()))
    assert len(got) == len(ref)
    assert np.array_equal(got["x"], ref.x) and np.array_equal(got["y"], ref.y) and np.array_equal(got["k"], ref.k)


@pytest.mark.parametrize("name,gh,gw,sx,levels_q,level,dmin,cap", [
    ("several hundred maxima from staged maps (bucket sort in LDS)", 60, 80, 1, 0, 1, 3.0, 1024),
    ("equal scores everywhere (tie rules of the staged scan)", 60, 80, 1, 8, 0, 2.0, 1024),
    ("coordinates beyond 2^15 (64-bit distance test)", 50, 70, 600, 0, 0, 700.0, 1024),
    ("coordinates beyond 2^15, few accepted", 50, 70, 600, 4, 2, 1000.0, 7),
])
def test_select_paths(name, gh, gw, sx, levels_q, level, dmin, cap):
    """Random maps through each path of the selection, against the oracle's
    list: the scan from maps staged in LDS (bordered grid of at most 5120 cells), the bucket sort
    (129..1024 maxima), many equal S_w and S_1 (levels_q > 0 quantises both),
    and the suppression's distance test in 64 bits (x = i sx beyond 2^15)."""
    P = _P()
    case(f"select: {name}")
    rng = np.random.default_rng(gh * 1000 + gw + sx + levels_q)
    mw = rng.random((gh, gw))
    m1 = rng.random((gh, gw))
    if levels_q:
        mw = np.floor(mw * levels_q) / levels_q
        m1 = np.floor(m1 * 2) / 2
    mw, m1 = mw.astype(np.float32), m1.astype(np.float32)
    mk = rng.integers(0, 90, (gh, gw)).astype(np.int32)
    ref = O.select(mw.astype(np.float64), m1.astype(np.float64), mk, sx, sx, level, 0.0, dmin, cap)
    out, n = P.select(torch.from_numpy(mw).cuda(), torch.from_numpy(m1).cuda(), torch.from_numpy(mk).cuda(), sx, sx,
                      level, 0.0, dmin, cap)
    got = P.poses_to_numpy(out, int(n.item()))
    print(f"{len(ref)} candidates")
    assert len(got) == len(ref) and len(ref) > 0
    assert np.array_equal(got["x"], ref.x) and np.array_equal(got["y"], ref.y) and np.array_equal(got["k"], ref.k)
    assert np.array_equal(got["sw"], ref.sw.astype(np.float32)) and np.array_equal(got["s1"], ref.s1.astype(np.float32))


# ------------------------------------------------------------ refine, detect
def _oracle_key(fields, om, sp, L, x, y, k, level=0):
    st = O.level_step(sp, L, level)
    ml = om.levels[level]
    return O.score(fields[level], ml.t, ml.d, int(x), int(y), O.theta(sp.theta_min, st, int(k)), sp.neighbourhood)


def _match_detections(got, ref, fields, om, osp, L):
    assert len(got) == len(ref), (len(got), len(ref))
    ties = 0
    for g, r in zip(got, ref):
        if (int(g["x"]), int(g["y"]), int(g["k"])) == (r.x, r.y, r.k):
            assert abs(g["sw"] - r.sw) <= TOL and abs(g["s1"] - r.s1) <= TOL
            continue
        a = _oracle_key(fields, om, osp, L, g["x"], g["y"], g["k"])
        assert abs(a[0] - r.sw) <= TOL and abs(a[1] - r.s1) <= TOL, (g, r)
        ties += 1
    return ties


@pytest.mark.parametrize("ci,index", [(1, 0), (1, 1), (2, 0), (2, 1), (3, 0)])
def test_detect_matches_oracle(ci, index):
    P = _P()
    sc = synth.scene_for_config(ci, index)
    cfg = sc.config
    L = cfg["levels"]
    case(f"detect C{ci} image {index}")
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"], theta_range=360.0)
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp)
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
    got = P.detect(gm, pyr, P.SearchParams(theta_step_top=cfg["theta_step_top"]))
    ties = _match_detections(got, tr.detections, tr.fields, tr.model, osp, L)
    print(f"{len(got)} detections, {ties} ties; truth {[(round(i.x), round(i.y), round(i.theta)) for i in sc.instances]}")


@pytest.mark.parametrize("quarter", [0, 1, 2, 3])
def test_detect_pasted_model_exact(quarter):
    P = _P()
    case(f"detect pasted model quarter={quarter}")
    rng = np.random.default_rng(20211200 + 500 + quarter)
    model = synth.render_model(synth.make_model_shape("blocks", 32, rng), 32)
    # the quarter-turned model's cells align with the 4x4 cells of level 2
    ux, uy = [(64, 48), (63, 48), (63, 47), (64, 47)][quarter]
    img = synth.paste_rot90(model, 128, 112, ux, uy, quarter)
    gm = P.Model(model, 3, 30.0)
    pyr = P.Pyramid(img, 3, 30.0)
    got = P.detect(gm, pyr, P.SearchParams(theta_step_top=10.0, max_matches=1))
    assert len(got) == 1
    d = got[0]
    assert (d["x"], d["y"], d["theta"]) == (ux, uy, 90.0 * quarter)
    assert abs(d["sw"] - 1) <= TOL and abs(d["s1"] - 1) <= TOL


def test_refine_matches_oracle():
    P = _P()
    case("refine C2 oracle candidates")
    sc = synth.scene_for_config(2, 2)
    cfg = sc.config
    L = 4
    osp = O.SearchParams(theta_step_top=1.0)
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp)
    cand = tr.candidates
    poses = np.zeros(len(cand), P.POSE_DTYPE)
    poses["x"], poses["y"], poses["k"], poses["level"] = cand.x, cand.y, cand.k, L - 1
    poses["sw"], poses["s1"] = cand.sw, cand.s1
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"])
    got = P.refine(gm, pyr, P.SearchParams(theta_step_top=1.0), poses, L - 1)
    ref = tr.refined[-1]
    ties = 0
    for i in range(len(cand)):
        g = got[i]
        if (g["x"], g["y"], g["k"]) == (ref.x[i], ref.y[i], ref.k[i]):
            assert abs(g["sw"] - ref.sw[i]) <= TOL and abs(g["s1"] - ref.s1[i]) <= TOL
            continue
        a = _oracle_key(tr.fields, tr.model, osp, L, g["x"], g["y"], g["k"])
        assert abs(a[0] - ref.sw[i]) <= TOL and abs(a[1] - ref.s1[i]) <= TOL, (i, g, ref.rows()[i])
        ties += 1
    print(f"{len(cand)} candidates refined, {ties} ties")


@pytest.mark.parametrize("index", [2, 25])
def test_refine_fp16_step_matches_oracle(index):
    """One refinement step on an FP16 pyramid from the oracle's level-1
    poses: the refinement reads the pyramid's FP32 twin, so each pick is the
    oracle's, or a tie within 1e-5 under the oracle's key."""
    P = _P()
    case(f"FP16 refinement step C2 image {index}")
    sc = synth.scene_for_config(2, index)
    cfg = sc.config
    L = 4
    osp = O.SearchParams(theta_step_top=1.0)
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp)
    src, ref = tr.refined[-2], tr.refined[-1]  # level 1, level 0
    poses = np.zeros(len(src.x), P.POSE_DTYPE)
    poses["x"], poses["y"], poses["k"], poses["level"] = src.x, src.y, src.k, 1
    poses["sw"], poses["s1"] = src.sw, src.s1
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP16)
    got = P.refine(gm, pyr, P.SearchParams(theta_step_top=1.0), poses, 1)
    other = 0
    for i in range(len(src.x)):
        g = got[i]
        if (int(g["x"]), int(g["y"]), int(g["k"])) == (ref.x[i], ref.y[i], ref.k[i]):
            assert abs(g["sw"] - ref.sw[i]) <= TOL and abs(g["s1"] - ref.s1[i]) <= TOL
            continue
        a = _oracle_key(tr.fields, tr.model, osp, L, g["x"], g["y"], g["k"])
        assert abs(a[0] - ref.sw[i]) <= TOL and abs(a[1] - ref.s1[i]) <= TOL, (i, g, ref.rows()[i])
        other += 1
    print(f"{len(src.x)} poses, {other} picks differ from the oracle's as ties within 1e-5")


def test_detect_is_deterministic():
    P = _P()
    case("determinism")
    sc = synth.scene_for_config(2, 3)
    cfg = sc.config
    gm = P.Model(sc.model, 4, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, 4, cfg["tau_s"])
    sp = P.SearchParams()
    a = P.detect(gm, pyr, sp)
    m1 = [t.clone() for t in P.score_map(gm, pyr, 3, sp)]
    for _ in range(3):
        assert np.array_equal(P.detect(gm, pyr, sp), a)
        m2 = P.score_map(gm, pyr, 3, sp)
        assert all(torch.equal(x, y) for x, y in zip(m1, m2))


# ------------------------------------------------------------ FP16 directions
# Each component of a unit vector rounded to half has relative error <= 2^-11,
# so |r_h . g_h - r . g| <= 2 * 2^-11 (+ FP32 rounding of the sums); the max of
# a window and the mean over points keep that bound.
TOL16 = 2 * 2.0 ** -11 + 2e-5


@pytest.mark.parametrize("ci", [2, 3])
def test_score_map_fp16(ci):
    P = _P()
    sc = synth.scene_for_config(ci)
    cfg = sc.config
    L = cfg["levels"]
    top = L - 1
    case(f"score_map FP16 C{ci}")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP16)
    st = cfg["theta_step_top"]
    sw, s1, k = [t.cpu().numpy() for t in P.score_map(gm, pyr, top, P.SearchParams(theta_step_top=st))]
    om = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
    g = O.field_pyramid(sc.image, L, cfg["tau_s"])[top]
    ml = om.levels[top]
    mw, m1, mk = O.top_map(g, ml.t, ml.d, 0.0, st, int(np.ceil(360.0 / st)))
    # S_w is the maximum over angles, so it stays within the bound even where
    # another angle wins; S_1 belongs to the winning angle and is compared
    # where the angles agree, and against the oracle at the GPU's angle where
    # they do not (which must then be an oracle tie within two bounds).
    same = k == mk
    ew, e1 = np.abs(sw - mw).max(), np.abs(s1 - m1)[same].max()
    diff = np.argwhere(~same)
    print(f"FP16 map: max |dS_w| {ew:.3g} mean {np.abs(sw - mw).mean():.3g} p99 "
          f"{np.quantile(np.abs(sw - mw), 0.99):.3g}; max |dS_1| (same angle) {e1:.3g}; "
          f"angle differs at {len(diff)} of {k.size}")
    assert ew <= TOL16 and e1 <= TOL16
    for (j, i) in diff:
        a = O.score(g, ml.t, ml.d, int(i), int(j), O.theta(0.0, st, int(k[j, i])))
        assert abs(a[0] - mw[j, i]) <= 2 * TOL16, (i, j)
        assert abs(a[0] - sw[j, i]) <= TOL16 and abs(a[1] - s1[j, i]) <= TOL16, (i, j)


def test_score_poses_fp16():
    P = _P()
    sc = synth.scene_for_config(2)
    cfg = sc.config
    case("score_poses FP16 C2 level 1")
    gm = P.Model(sc.model, 4, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, 4, cfg["tau_s"], precision=P.TM_FP16)
    g = O.field_pyramid(sc.image, 4, cfg["tau_s"])[1]
    ml = O.build_model(sc.model, O.PyrParams(4, cfg["tau_m"])).levels[1]
    rng = np.random.default_rng(77)
    xs, ys, th = rng.integers(0, 320, 200), rng.integers(0, 240, 200), rng.uniform(0, 360, 200)
    got = P.score_poses(gm, pyr, 1, xs, ys, th).cpu().numpy().astype(np.float64)
    ref = np.array([O.score(g, ml.t, ml.d, int(xs[i]), int(ys[i]), float(th[i])) for i in range(200)])
    assert np.abs(got - ref).max() <= TOL16


@pytest.mark.parametrize("ci,index", [(2, 0), (2, 1), (3, 0)])
def test_detect_fp16_matches_oracle(ci, index):
    """FP16 detections: every match the oracle's (the same pose, or a tie
    within 1e-5 under the oracle's key), scores within 1e-5: the FP16 search
    is certified and the refinement reads the FP32 twin."""
    P = _P()
    sc = synth.scene_for_config(ci, index)
    cfg = sc.config
    L, st = cfg["levels"], cfg["theta_step_top"]
    case(f"detect FP16 C{ci} image {index}")
    osp = O.SearchParams(theta_step_top=st)
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp)
    gm = P.Model(sc.model, L, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP16)
    got = P.detect(gm, pyr, P.SearchParams(theta_step_top=st))
    ref = tr.detections
    print(f"FP16 {[(int(d['x']), int(d['y']), int(d['k']), round(float(d['sw']), 4)) for d in got]}")
    print(f"FP64 {[(d.x, d.y, d.k, round(d.sw, 4)) for d in ref]}")
    assert len(got) == len(ref) and len(ref) >= 1
    for g0, r0 in zip(got, ref):
        if (int(g0["x"]), int(g0["y"]), int(g0["k"])) != (r0.x, r0.y, r0.k):
            a = _oracle_key(tr.fields, tr.model, osp, L, g0["x"], g0["y"], g0["k"])
            assert abs(a[0] - r0.sw) <= TOL and abs(a[1] - r0.s1) <= TOL, (g0, r0)
        assert abs(float(g0["sw"]) - r0.sw) <= TOL and abs(float(g0["s1"]) - r0.s1) <= TOL


@pytest.mark.parametrize("precision", [0, 1])
def test_search_kernel_shape_independence(precision, monkeypatch):
    """Every launch shape and every kernel variant gives bit-identical maps
    (the per-lane sums run in point order whatever the tiling)."""
    P = _P()
    sc = synth.scene_for_config(2, 4)
    cfg = sc.config
    case(f"launch shapes precision={precision}")
    gm = P.Model(sc.model, 4, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, 4, cfg["tau_s"], precision=precision)
    sp = P.SearchParams(theta_step_top=1.0)
    ref = [t.clone() for t in P.score_map(gm, pyr, 3, sp)]
    for wy, wa, apw, asm, tr in [(1, 4, 1, 1, 0), (2, 4, 1, 0, 1), (1, 8, 2, 2, 0), (1, 16, 1, 3, 1),
                                 (4, 1, 3, 5, 0), (1, 4, 1, 4, 0), (1, 16, 1, 4, 1), (2, 2, 1, 5, 1)]:
        monkeypatch.setenv("TM_DENSE_WY", str(wy))
        monkeypatch.setenv("TM_DENSE_WA", str(wa))
        monkeypatch.setenv("TM_DENSE_APW", str(apw))
        monkeypatch.setenv("TM_DENSE_ASM", str(asm))
        monkeypatch.setenv("TM_DENSE_TR", str(tr))
        got = P.score_map(gm, pyr, 3, sp)
        assert all(torch.equal(x, y) for x, y in zip(ref, got)), (wy, wa, apw, asm, tr)


@pytest.mark.parametrize("H,W", [(61, 67), (40, 201), (201, 40), (41, 95)])
def test_search_orientation_independence(H, W, monkeypatch):
    """Lanes along x or along y (the tile transposed): bit-identical maps on
    ragged shapes, both equal to the oracle's within the bar."""
    P = _P()
    case(f"orientations {W}x{H}")
    rng = np.random.default_rng(950 + H + W)
    shape = synth.make_model_shape("blocks", 24, rng)
    model = synth.render_model(shape, 24)
    sc = synth.render_scene(rng, W, H, shape, 24, 1, 5.0, clutter=6)
    gm = P.Model(model, 1, 30.0)
    sp = P.SearchParams(theta_step_top=7.5)
    maps = []
    for prec in (0, 1):
        pyr = P.Pyramid(sc.image, 1, 30.0, precision=prec)
        per = []
        for tr in (0, 1):
            monkeypatch.setenv("TM_DENSE_TR", str(tr))
            per.append([t.clone() for t in P.score_map(gm, pyr, 0, sp)])
        assert all(torch.equal(x, y) for x, y in zip(*per)), prec
        maps.append(per[0])
    om = O.build_model(model, O.PyrParams(1, 30.0))
    g = O.edge_field(sc.image, 30.0)
    ref = O.top_map(g, om.levels[0].t, om.levels[0].d, 0.0, 7.5, 48)
    _check_map(maps[0], ref, g, om.levels[0], 0.0, 7.5, 1, 1, 3)


# ------------------------------------------------------------ batches
def _poses_equal(a, b):
    return len(a) == len(b) and all(
        (int(x["x"]), int(x["y"]), int(x["k"]), float(x["sw"]), float(x["s1"])) ==
        (int(y["x"]), int(y["y"]), int(y["k"]), float(y["sw"]), float(y["s1"])) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_detections(precision):
    """One launch per stage over all (image, model) pairs gives exactly the
    detections of the single-image calls (mixed sizes, two models).  With 18
    pairs x 32 candidates the batch refines from LDS-staged field blocks and
    the single calls by gathers: the partial sums must still be identical."""
    P = _P()
    case(f"batch vs single precision={precision}")
    cfg = synth.CONFIGS[2]
    scenes = [synth.scene_for_config(2, i) for i in range(8)]
    big = synth.scene_for_config(2, 7, W=1280, H=1024, n_inst=4)
    rng = np.random.default_rng(4242)
    m2 = synth.render_model(synth.make_model_shape("polygon", 96, rng), 96)
    models = [P.Model(scenes[0].model, 4, cfg["tau_m"]), P.Model(m2, 4, cfg["tau_m"])]
    images = [torch.from_numpy(s.image).cuda() for s in scenes] + [torch.from_numpy(big.image).cuda()]
    sp = P.SearchParams(theta_step_top=1.0)
    b = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=precision)
    b.run()
    got = b.results()
    for i, im in enumerate(images):
        pyr = P.Pyramid(im, 4, cfg["tau_s"], precision=precision)
        for j, m in enumerate(models):
            ref = P.detect(m, pyr, sp)
            assert _poses_equal(got[i * 2 + j], ref), (i, j, got[i * 2 + j], ref)
    # run again on new contents of the same buffers
    images[0].copy_(torch.from_numpy(scenes[1].image).cuda())
    b.run()
    again = b.results()
    assert _poses_equal(again[0], got[2]) and _poses_equal(again[1], got[3])


def test_batch_pyramids_match_oracle():
    P = _P()
    case("batch pyramids")
    imgs = [_scene_img(96, 128, 11), _scene_img(211, 333, 12)]
    dev = [torch.from_numpy(i).cuda() for i in imgs]
    rng = np.random.default_rng(4243)
    m = P.Model(synth.render_model(synth.make_model_shape("blocks", 32, rng), 32), 2, 30.0)
    b = P.Batch([m], dev, 2, 45.5, P.SearchParams(theta_step_top=10.0))
    b.run()
    torch.cuda.synchronize()
    import ctypes
    for i, im in enumerate(imgs):
        h = ctypes.c_void_p()
        assert P.lib().tm_batch_pyramid(b._h, i, ctypes.byref(h)) == 0
        pyr = P.Pyramid.__new__(P.Pyramid)
        pyr._h, pyr.levels, pyr.precision = h, 2, 0
        try:
            for l, lv in enumerate(O.pyramid(im, 2)):
                gi, gf = pyr.read(l)
                assert np.array_equal(gi.cpu().numpy(), lv)
                of = O.edge_field(lv, 45.5)
                assert np.abs(gf.cpu().numpy().astype(np.float64) - of).max() <= 6e-8
        finally:
            pyr._h = ctypes.c_void_p()  # owned by the batch


def test_batch_graph_replays_match_eager(monkeypatch):
    """The captured graph gives the eager batch's detections on every replay,
    with eager work and new image contents between replays; the search's
    work list (XCD-binned, longest first) changes nothing either."""
    P = _P()
    case("batch graph replays")
    cfg = synth.CONFIGS[2]
    scenes = [synth.scene_for_config(2, i) for i in range(4)]
    rng = np.random.default_rng(4244)
    m2 = synth.render_model(synth.make_model_shape("polygon", 80, rng), 80)
    models = [P.Model(scenes[0].model, 4, cfg["tau_m"]), P.Model(m2, 4, cfg["tau_m"])]
    sp = P.SearchParams(theta_step_top=2.0)
    images = [torch.from_numpy(s.image).cuda() for s in scenes[:3]]
    b = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=1)
    b.run()
    eager = b.results()
    monkeypatch.setenv("TM_DENSE_WORKLIST", "0")
    b0 = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=1)
    b0.run()
    plain = b0.results()
    assert all(_poses_equal(a, c) for a, c in zip(eager, plain))
    for r in range(3):
        b.out.zero_()
        b.n_out.zero_()
        torch.cuda.synchronize()
        b.run(graph=True)
        torch.cuda.synchronize()
        got = b.results()
        assert all(_poses_equal(a, c) for a, c in zip(got, eager)), r
    images[0].copy_(torch.from_numpy(scenes[3].image).cuda())
    b0.run()
    ref = b0.results()
    b.run(graph=True)
    got = b.results()
    assert all(_poses_equal(a, c) for a, c in zip(got, ref))


@pytest.mark.parametrize("index", [0, 1, 2])
def test_paper_shaped_search_matches_oracle(index):
    """The paper's own search (812x617, every 3rd pixel, 90 degrees in 3 degree
    steps, one level, one best pose) on the generic search path."""
    P = _P()
    sc = synth.scene_for_config(6, index)
    cfg = sc.config
    case(f"paper-shaped frame {index}")
    kw = dict(step_x=3, step_y=3, theta_min=0.0, theta_range=90.0, theta_step_top=3.0, max_matches=1)
    osp = O.SearchParams(**kw)
    tr = O.detect(sc.image, sc.model, O.PyrParams(1, cfg["tau_s"]), O.PyrParams(1, cfg["tau_m"]), osp)
    gm = P.Model(sc.model, 1, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, 1, cfg["tau_s"])
    got = P.detect(gm, pyr, P.SearchParams(**kw))
    ref = tr.detections
    print(f"GPU {[(int(d['x']), int(d['y']), int(d['k']), float(d['sw'])) for d in got]}")
    print(f"FP64 {[(d.x, d.y, d.k, d.sw) for d in ref]}, truth {sc.instances}")
    assert len(got) == len(ref) == 1
    _match_detections(got, ref, tr.fields, tr.model, osp, 1)


def test_batch_tune_keeps_results():
    """The autotuner only picks among bit-identical schedules of the search
    (variant, waves per chunk, angles per chunk): the tuned batch returns
    exactly the detections of the untuned one, eager and as a graph, alone
    and tuned on the pipelined step with a partner; every chunking the batch
    holds gives the same detections."""
    P = _P()
    case("batch autotune")
    cfg = synth.CONFIGS[2]
    scenes = [synth.scene_for_config(2, i) for i in range(6)]
    models = [P.Model(scenes[0].model, 4, cfg["tau_m"])]
    images = [torch.from_numpy(s.image).cuda() for s in scenes]
    sp = P.SearchParams(theta_step_top=1.0)
    for precision in (0, 1):
        b = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=precision)
        b.run()
        ref = b.results()
        planned = b.search_form()
        b.run(graph=True)  # a graph of the untuned form, to be discarded by tune()
        torch.cuda.synchronize()
        choice = b.tune(iterations=1)
        print(f"precision {precision}: {choice}")
        assert 0 <= choice["variant"] <= 5 and choice["waves_per_chunk"] in (2, 4, 8, 16)
        assert choice["search_us"] > 0 and 4 <= choice["chunk_angles"] <= 360
        b.run()
        assert all(_poses_equal(a, c) for a, c in zip(b.results(), ref))
        b.run(graph=True)
        assert all(_poses_equal(a, c) for a, c in zip(b.results(), ref))
        # every chunking the batch holds, in the planned form: the same detections
        for chunk in (8, 16, 40, 120, 360):
            try:
                b.set_form(planned["variant"], planned["waves_per_chunk"], chunk)
            except P.TMError:  # more chunks than the batch holds
                assert 360 // chunk > 12
                continue
            assert b.search_form()["chunk_angles"] == chunk
            # the launch shape follows the schedule: a wave per 64 threads sharing a chunk, and at least
            # one workgroup per (tile, chunk) of every pair (the work list may pad its XCD bins)
            shape = b.search_launch()
            assert shape["threads"] == 64 * planned["waves_per_chunk"]
            assert shape["workgroups"] >= -(-360 // chunk) * len(images)
            b.run(graph=True)
            assert all(_poses_equal(a, c) for a, c in zip(b.results(), ref)), chunk
        # tuned on the pipelined step with a partner of the same shape: both keep the choice
        b2 = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=precision)
        s2 = torch.cuda.Stream()
        pc = b.tune(iterations=1, partner=b2, partner_stream=s2)
        assert pc["step_us"] > 0 and b2.search_form() == b.search_form()
        b.run(graph=True)
        b2.run(s2, graph=True)
        torch.cuda.synchronize()
        assert all(_poses_equal(a, c) for a, c in zip(b.results(), ref))
        assert all(_poses_equal(a, c) for a, c in zip(b2.results(), ref))
        # another batch of the same shape takes the tuned schedule as it is, and
        # a form that does not apply is refused
        b3 = P.Batch(models, images, 4, cfg["tau_s"], sp, precision=precision)
        b3.set_form(choice["variant"], choice["waves_per_chunk"], choice["chunk_angles"])
        assert b3.search_form() == {"variant": choice["variant"], "waves_per_chunk": choice["waves_per_chunk"],
                                    "chunk_angles": choice["chunk_angles"]}
        b3.run(graph=True)
        assert all(_poses_equal(a, c) for a, c in zip(b3.results(), ref))
        with pytest.raises(P.TMError):
            b3.set_form(9, 4)
        with pytest.raises(P.TMError):
            b3.set_form(planned["variant"], planned["waves_per_chunk"], 1)  # 360 chunks: beyond the scratch
