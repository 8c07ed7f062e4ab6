"""Edge cases of the detection path on the GPU against the FP64 oracle:
inputs with no edges, the smallest image a pyramid allows, instances cut by
the image border, partial angle ranges (clamped, not wrapped, in the
refinement), the largest candidate count with every local maximum kept, and
a model with very few points at the top level."""
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

    P.lib()
    return P


def _P():
    import paper_2112_05576_amd as P

    return P


def _detect_both(img, model, L, tau_s, tau_m, **kw):
    P = _P()
    osp = O.SearchParams(**kw)
    tr = O.detect(img, model, O.PyrParams(L, tau_s), O.PyrParams(L, tau_m), osp)
    gm = P.Model(model, L, tau_m)
    pyr = P.Pyramid(img, L, tau_s)
    got = P.detect(gm, pyr, P.SearchParams(**kw))
    return got, tr, osp


def _match(got, tr, osp, L):
    ref = tr.detections
    assert len(got) == len(ref), (len(got), len(ref))
    st = O.level_step(osp, L, 0)
    ml = tr.model.levels[0]
    for g, r in zip(got, ref):
        if (int(g["x"]), int(g["y"]), int(g["k"])) == (r.x, r.y, r.k):
            assert abs(g["sw"] - r.sw) <= TOL and abs(g["s1"] - r.s1) <= TOL
            continue
        a = O.score(tr.fields[0], ml.t, ml.d, int(g["x"]), int(g["y"]), O.theta(osp.theta_min, st, int(g["k"])))
        assert abs(a[0] - r.sw) <= TOL and abs(a[1] - r.s1) <= TOL, (g, r)


def _model(seed=0, size=64):
    rng = np.random.default_rng(20211200 + 900 + seed)
    return synth.render_model(synth.make_model_shape("polygon", size, rng), size)


def test_blank_image_gives_no_detection():
    case("blank image")
    img = np.full((120, 160), 90, np.uint8)
    got, tr, _ = _detect_both(img, _model(), 2, 30.0, 30.0, theta_step_top=10.0)
    assert len(got) == 0 and len(tr.detections) == 0
    # every score is 0 on an edge-free field
    mw = tr.top[0]
    assert np.all(mw == 0.0)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_smallest_image_of_a_pyramid(L):
    """3 * 2^(L-1) pixels a side, the least the pyramid accepts."""
    case(f"smallest image L={L}")
    side = 3 * 2 ** (L - 1)
    rng = np.random.default_rng(77 + L)
    img = rng.integers(0, 256, (side, side), dtype=np.uint8)
    model = np.full((side, side), 40, np.uint8)
    model[side // 3: 2 * side // 3 + 1, side // 4: 3 * side // 4 + 1] = 210
    got, tr, osp = _detect_both(img, model, L, 30.0, 30.0, theta_step_top=30.0, min_score=-1.0)
    _match(got, tr, osp, L)
    P = _P()
    with pytest.raises(P.TMError):
        P.Pyramid(img[:side - 1], L, 30.0)


@pytest.mark.parametrize("quarter", [0, 1])
def test_instance_cut_by_the_border(quarter):
    case(f"instance at the border quarter={quarter}")
    model = _model(1)
    # model centre 10 px inside the left / top border: most of it is outside
    img = synth.paste_rot90(model, 200, 160, 10 if quarter == 0 else 100, 80 if quarter == 0 else 6, quarter)
    rng = np.random.default_rng(5)
    img = np.clip(img.astype(np.int64) + rng.integers(-4, 5, img.shape), 0, 255).astype(np.uint8)
    got, tr, osp = _detect_both(img, model, 2, 30.0, 30.0, theta_step_top=4.0, min_score=0.2)
    _match(got, tr, osp, 2)


@pytest.mark.parametrize("theta_min,theta_range", [(-45.0, 90.0), (350.0, 20.0)])
def test_partial_angle_range_clamps(theta_min, theta_range):
    """A partial range holds both end points and clamps the refinement's
    2k+-1 at its ends; instances beyond the range are not wrapped into it."""
    case(f"partial range {theta_min} + {theta_range}")
    sc = synth.scene_for_config(2, 5)
    cfg = sc.config
    got, tr, osp = _detect_both(sc.image, sc.model, 3, cfg["tau_s"], cfg["tau_m"], theta_min=theta_min,
                                theta_range=theta_range, theta_step_top=2.0, min_score=0.3)
    _match(got, tr, osp, 3)
    K0 = O.level_count(osp, O.level_step(osp, 3, 0))
    assert all(0 <= int(d["k"]) < K0 for d in got)


def test_every_local_maximum_with_the_largest_candidate_count():
    """A noise image, no score floor, the largest candidate list: every strict
    local maximum of the top-level map is carried through refinement."""
    case("max_candidates 1024, min_score -1, noise image")
    sc = synth.scene_for_config(2, 6)
    img = np.random.default_rng(3).integers(0, 256, (480, 640), dtype=np.uint8)
    got, tr, osp = _detect_both(img, sc.model, 4, 30.0, sc.config["tau_m"], theta_step_top=4.0, min_score=-1.0,
                                max_candidates=1024, max_matches=64, nms_min_dist=1.0)
    assert len(tr.candidates) > 100 and len(tr.detections) == 64
    _match(got, tr, osp, 4)


def test_model_with_few_top_level_points():
    """A 16-pixel model has 4 points at level 2."""
    case("tiny model")
    model = np.full((16, 16), 40, np.uint8)
    model[5:11, 4:12] = 200
    om = O.build_model(model, O.PyrParams(3, 30.0))
    print(f"points per level {[len(l.t) for l in om.levels]}")
    assert len(om.levels[2].t) <= 4
    img = synth.paste_rot90(model, 96, 96, 50, 41, 1)
    got, tr, osp = _detect_both(img, model, 3, 30.0, 30.0, theta_step_top=8.0)
    _match(got, tr, osp, 3)


def test_zero_length_inputs_enqueue_nothing():
    """Every call that takes a list of poses accepts an empty one and returns
    an empty result; a map with nothing above the score floor selects nothing;
    the library keeps working afterwards (no error is left behind)."""
    P = _P()
    case("zero-length inputs")
    sc = synth.scene_for_config(1, 0)
    cfg = sc.config
    gm = P.Model(sc.model, 1, cfg["tau_m"])
    pyr = P.Pyramid(sc.image, 1, cfg["tau_s"])
    assert P.score_poses(gm, pyr, 0, [], [], []).shape == (0, 2)
    assert len(P.refine(gm, pyr, P.SearchParams(theta_step_top=5.0), np.zeros(0, P.POSE_DTYPE), 0)) == 0
    none = torch.zeros((0, 3), dtype=torch.float32)
    assert P.cont_score(gm, pyr, 0, none).shape == (0,)
    assert P.cont_score_backward(gm, pyr, 0, none).shape == (0, 3)
    moved, scores = P.cont_line_search(gm, pyr, 0, none, none, [0.0, 1.0])
    assert moved.shape == (0, 3) and scores.shape == (0,)
    flat = torch.zeros((6, 8), dtype=torch.float32, device="cuda")
    out, n = P.select(flat, flat, torch.zeros((6, 8), dtype=torch.int32, device="cuda"), 1, 1, 0, 0.5, 0.0, 16)
    assert int(n.item()) == 0
    # and a real call after them: one pose against the oracle
    g = O.edge_field(sc.image, cfg["tau_s"])
    ml = O.build_model(sc.model, O.PyrParams(1, cfg["tau_m"])).levels[0]
    x, y, th = sc.instances[0].x, sc.instances[0].y, 10.0
    want = O.score(g, ml.t, ml.d, int(round(x)), int(round(y)), th)
    got = P.score_poses(gm, pyr, 0, [int(round(x))], [int(round(y))], [th]).cpu().numpy()[0]
    assert abs(got[0] - want[0]) <= TOL and abs(got[1] - want[1]) <= TOL
