"""FP16 detections take the FP32 decisions.  The FP16 search is certified:
every translation whose FP32 value could change the candidate selection is
re-scored in FP32 over the angles left open by the FP16 bound, and the
refinement works on the pyramid's FP32 twin, so an FP16 detection returns the
FP32 detection bit for bit.  Checked:

* the 64 scenes of the benchmark's batch (640x480, 4 levels, 1 degree at the
  top): FP16 batch (graph launch) = FP32 batch, every detection bit for bit,
  and every image's detections equal to the FP64 oracle's (stored by
  tests/golden/make_oracle_detections.py) under the tie rule: the same pose,
  or a pose whose oracle S_w and S_1 are within 1e-5 of the oracle's match;
  scores within 1e-5 of the oracle's at the reported pose;
* single FP16 detections (the unbatched plan, small angle chunks) = FP32;
* the 2048x2048 five-level configuration, two images: FP16 = FP32, and the
  oracle's top match under the same rule;
* the similarity search, the edge-taps vote and the generic search (steps
  of 3 pixels): FP16 = FP32."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
HERE = os.path.dirname(os.path.abspath(__file__))


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


def _same(a, b):
    return len(a) == len(b) and a.tobytes() == b.tobytes()


def _golden():
    import importlib.util

    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_oracle_detections.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    g = json.load(open(os.path.join(HERE, "golden", "c2_bench_oracle.json")))
    return mk, g


def _match_oracle(dets, ref, fields0, ml, theta_of):
    """Every detection against the oracle's list: equal poses, or ties under
    the oracle's own key within 1e-5 (S_w and S_1)."""
    assert len(dets) == len(ref), (len(dets), len(ref))
    ties = 0
    for d, r in zip(dets, ref):
        rx, ry, rk, rsw, rs1 = int(r[0]), int(r[1]), int(r[2]), float(r[4]), float(r[5])
        if (int(d["x"]), int(d["y"]), int(d["k"])) == (rx, ry, rk):
            assert abs(float(d["sw"]) - rsw) <= TOL and abs(float(d["s1"]) - rs1) <= TOL, (d, r)
            continue
        sw, s1 = O.score(fields0, ml.t, ml.d, int(d["x"]), int(d["y"]), theta_of(int(d["k"])))
        assert abs(sw - rsw) <= TOL and abs(s1 - rs1) <= TOL, (d, r, sw, s1)
        assert abs(float(d["sw"]) - sw) <= TOL and abs(float(d["s1"]) - s1) <= TOL, (d, sw, s1)
        ties += 1
    return ties


def test_bench_batch_fp16_equals_fp32_and_oracle():
    P = _P()
    mk, gold = _golden()
    cfg = synth.CONFIGS[2]
    L = cfg["levels"]
    case("64 benchmark scenes: FP16 batch = FP32 batch = oracle")
    scenes = [synth.scene_for_config(2, i) for i in range(64)]
    for sc, g in zip(scenes, gold["images"]):
        assert mk.scene_hash(sc) == g["scene"], "the stored oracle detections are stale: rerun the golden script"
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    model = P.Model(scenes[0].model, L, cfg["tau_m"])
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    b16 = P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=P.TM_FP16)
    b32 = P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=P.TM_FP32)
    b16.run(graph=True)
    b32.run(graph=True)
    r16, r32 = b16.results(), b32.results()
    diff = [i for i in range(64) if not _same(r16[i], r32[i])]
    assert not diff, f"FP16 differs from FP32 on images {diff}"
    om = O.build_model(scenes[0].model, O.PyrParams(L, cfg["tau_m"]))
    ml = om.levels[0]
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    step0 = O.level_step(osp, L, 0)
    ties = 0
    for i, (sc, g) in enumerate(zip(scenes, gold["images"])):
        f0 = O.edge_field(sc.image, cfg["tau_s"])
        ties += _match_oracle(r16[i], g["detections"], f0, ml, lambda k: O.theta(0.0, step0, k))
    print(f"64 images, {sum(len(r) for r in r16)} detections equal to the oracle's ({ties} ties within 1e-5)")
    # the same batch again, and a second run of the graph, give the same bits
    b16.run(graph=True)
    assert all(_same(a, b) for a, b in zip(b16.results(), r16))


def test_single_fp16_detections_equal_fp32():
    P = _P()
    cfg = synth.CONFIGS[2]
    L = cfg["levels"]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    sc0 = synth.scene_for_config(2, 0)
    gm = P.Model(sc0.model, L, cfg["tau_m"])
    for i in range(8):
        case(f"single FP16 detection, image {i}")
        sc = synth.scene_for_config(2, i)
        a = P.detect(gm, P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP16), sp)
        b = P.detect(gm, P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP32), sp)
        assert _same(a, b), (i, a, b)


@pytest.mark.parametrize("index", [0, 1])
def test_c3_fp16_equals_fp32_and_oracle(index):
    P = _P()
    sc = synth.scene_for_config(3, index)
    cfg = sc.config
    L, st = cfg["levels"], cfg["theta_step_top"]
    case(f"C3 image {index}: FP16 = FP32 = oracle")
    gm = P.Model(sc.model, L, cfg["tau_m"])
    sp = P.SearchParams(theta_step_top=st)
    a = P.detect(gm, P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP16), sp)
    b = P.detect(gm, P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP32), sp)
    assert _same(a, b)
    osp = O.SearchParams(theta_step_top=st)
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp)
    ref = [[d.x, d.y, d.k, d.theta, d.sw, d.s1] for d in tr.detections]
    step0 = O.level_step(osp, L, 0)
    ties = _match_oracle(a, ref, tr.fields[0], tr.model.levels[0], lambda k: O.theta(0.0, step0, k))
    print(f"{len(a)} detections equal to the oracle's ({ties} ties)")


def test_variants_fp16_equal_fp32():
    """The similarity search (angles x scales), the edge-taps vote and the
    generic search (3-pixel steps over a partial angle range, one level)."""
    P = _P()
    # similarity, batched
    cfg = synth.CONFIGS[7]
    L = cfg["levels"]
    scenes = [synth.scene_for_config(7, i) for i in range(6)]
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    model = P.Model(scenes[0].model, L, cfg["tau_m"])
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"], scale_min=cfg["scale_min"],
                        scale_step=cfg["scale_step"], scale_count=cfg["scale_count"])
    case("similarity batch FP16 = FP32")
    r = [P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=pr) for pr in (P.TM_FP16, P.TM_FP32)]
    for b in r:
        b.run()
    assert all(_same(x, y) for x, y in zip(r[0].results(), r[1].results()))
    # edge-taps vote, single detections
    cfg = synth.CONFIGS[2]
    L = cfg["levels"]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"], vote=P.TM_VOTE_EDGE)
    for i in (2, 5):
        case(f"edge-taps vote FP16 = FP32, image {i}")
        sc = synth.scene_for_config(2, i)
        gm = P.Model(sc.model, L, cfg["tau_m"])
        a = P.detect(gm, P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP16), sp)
        b = P.detect(gm, P.Pyramid(sc.image, L, cfg["tau_s"], precision=P.TM_FP32), sp)
        assert _same(a, b)
    # generic search: steps of 3 pixels, 90 degrees in 3-degree steps, one level
    sc = synth.scene_for_config(6, 0)
    pc = sc.config
    gm = P.Model(sc.model, 1, pc["tau_m"])
    sp = P.SearchParams(step_x=3, step_y=3, theta_min=0.0, theta_range=90.0, theta_step_top=3.0, max_matches=4,
                        min_score=0.3)
    case("generic search FP16 = FP32")
    a = P.detect(gm, P.Pyramid(sc.image, 1, pc["tau_s"], precision=P.TM_FP16), sp)
    b = P.detect(gm, P.Pyramid(sc.image, 1, pc["tau_s"], precision=P.TM_FP32), sp)
    assert len(b) >= 1 and _same(a, b)
