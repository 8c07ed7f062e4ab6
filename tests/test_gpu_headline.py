"""The benchmark's batched leg as it is timed: 64 C2 scenes of 640x480, FP16
fields, the tuned search form, graph launches, two batches over the same
images in flight on two streams with the steps alternating between them.

Checks at this size: both batches give the same detections on every step;
every reported detection's S_w and S_1 equal the oracle's scores at the
reported pose within 1e-5 (an FP16 detection takes its decisions and its
scores in FP32: the certified search and the FP32 refinement); and for four
of the images the full oracle detection, whose top match the batch must
reproduce (the same pose, or one whose oracle key ties the oracle's within
1e-5)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def case(msg):
    print(f"[case] {msg}", flush=True)


def _same(a, b):
    return len(a) == len(b) and a.tobytes() == b.tobytes()


def test_headline_batch_two_streams_matches_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05576_amd as P

    P.lib()
    cfg = synth.CONFIGS[2]
    L = cfg["levels"]
    case("64 C2 images, FP16, tuned, graph launch, 2 batches on 2 streams")
    scenes = [synth.scene_for_config(2, i) for i in range(64)]
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    model = P.Model(scenes[0].model, L, cfg["tau_m"])
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    b0 = P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=P.TM_FP16)
    b1 = P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=P.TM_FP16)
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    form = b0.tune(iterations=1, partner=b1, partner_stream=streams[1])  # both keep the pipelined step's choice
    assert b1.search_form() == b0.search_form()
    for i in range(6):
        (b0, b1)[i % 2].run(streams[i % 2], graph=True)
    torch.cuda.synchronize()
    r0, r1 = b0.results(), b1.results()
    assert all(_same(a, b) for a, b in zip(r0, r1))
    om = O.build_model(scenes[0].model, O.PyrParams(L, cfg["tau_m"]))
    ml = om.levels[0]
    checked = 0
    for sc, dets in zip(scenes, r0):
        if len(dets) == 0:
            continue
        g0 = O.edge_field(sc.image, cfg["tau_s"])
        for d in dets:
            sw, s1 = O.score(g0, ml.t, ml.d, int(d["x"]), int(d["y"]), float(d["theta"]))
            assert abs(float(d["sw"]) - sw) <= TOL and abs(float(d["s1"]) - s1) <= TOL, (d, sw, s1)
            checked += 1
    print(f"{checked} detections checked against the oracle's scores at their poses; form {form}")
    assert checked >= 64
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    for i in (0, 1, 17, 63):
        case(f"oracle detection of image {i}")
        tr = O.detect(scenes[i].image, scenes[i].model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]),
                      osp, model=om)
        ref, dets = tr.detections, r0[i]
        print(f"  oracle {[(d.x, d.y, d.k, round(d.sw, 4)) for d in ref[:3]]}")
        print(f"  gpu    {[(int(d['x']), int(d['y']), int(d['k']), round(float(d['sw']), 4)) for d in dets[:3]]}")
        assert len(ref) > 0 and len(dets) > 0
        r, g = ref[0], dets[0]
        if (int(g["x"]), int(g["y"]), int(g["k"])) != (r.x, r.y, r.k):
            sw, s1 = O.score(tr.fields[0], ml.t, ml.d, int(g["x"]), int(g["y"]), float(g["theta"]))
            assert abs(sw - r.sw) <= TOL and abs(s1 - r.s1) <= TOL, (i, g, r)
