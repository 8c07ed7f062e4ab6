"""The batched workload at full size: 64 search images of mixed sizes
(640x480, 1280x1024, 2448x2048) against 8 models of 210 to 3900 points, in
one graph launch with FP16 fields (the launch the benchmark's batched leg
times), and the continuous refinement of 4096 poses over the same pairs.

At this size the oracle cannot redo every search, so the checks are:
  * for three 640x480 images with the two models of C2's size (about 750
    and 1100 points), the oracle's full detection, whose top match the batch
    must reproduce (equal, or a tie within 1e-5 under the oracle's own key:
    the FP16 search is certified and the refinement runs in FP32);
  * for every pair, every reported detection's S_w and S_1 recomputed by the
    oracle at the reported pose, within 1e-5;
  * for the continuous score, sampled poses against the oracle's FP64 value
    and gradient, and the refinement never lowering a pose's score."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def c4():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_05576_amd as P

    P.lib()
    cfg = synth.C4
    mods = [synth.c4_model(k) for k in range(len(synth.C4_MODELS))]
    shapes = [m[0] for m in mods]
    scenes = [synth.c4_image(i, shapes) for i in range(cfg["n_images"])]
    return P, cfg, [m[1] for m in mods], scenes


def _oracle_fields(img, L, tau):
    return O.field_pyramid(img, L, tau)


def test_c4_batch_graph_fp16(c4):
    P, cfg, model_imgs, scenes = c4
    L = cfg["levels"]
    case("C4 64 images x 8 models, FP16, graph launch")
    models = [P.Model(m, L, cfg["tau_m"]) for m in model_imgs]
    images = [torch.from_numpy(s.image).cuda() for s in scenes]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    b = P.Batch(models, images, L, cfg["tau_s"], sp, precision=P.TM_FP16)
    b.run(graph=True)
    got = b.results()
    oms = [O.build_model(m, O.PyrParams(L, cfg["tau_m"])) for m in model_imgs]
    nm = len(models)
    checked = 0
    for i, sc in enumerate(scenes):
        g0 = None
        for j in range(nm):
            dets = got[i * nm + j]
            if len(dets) == 0:
                continue
            if g0 is None:
                g0 = O.edge_field(sc.image, cfg["tau_s"])
            ml = oms[j].levels[0]
            for d in dets:
                assert int(d["level"]) == 0
                sw, s1 = O.score(g0, ml.t, ml.d, int(d["x"]), int(d["y"]), float(d["theta"]))
                assert abs(float(d["sw"]) - sw) <= TOL and abs(float(d["s1"]) - s1) <= TOL, (i, j, d, sw, s1)
                checked += 1
    print(f"checked {checked} detections of {sum(len(r) for r in got)}")
    assert checked > 100
    # full oracle detections on the small images with the small models
    small = [i for i, sc in enumerate(scenes) if sc.image.shape == (480, 640)][:3]
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    for i in small:
        for j in (3, 4):
            case(f"C4 oracle detect image {i} model {j}")
            tr = O.detect(scenes[i].image, model_imgs[j], O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]),
                          osp)
            ref, dets = tr.detections, got[i * nm + j]
            print(f"  oracle {[(d.x, d.y, d.k, round(d.sw, 4)) for d in ref[:3]]}")
            print(f"  gpu    {[(int(d['x']), int(d['y']), int(d['k']), round(float(d['sw']), 4)) for d in dets[:3]]}")
            if len(ref) == 0 or len(dets) == 0:  # only a top score at the threshold may be missing on one side
                assert len(ref) == len(dets), (i, j, len(ref), len(dets))
                continue
            r0, g0 = ref[0], dets[0]
            if (int(g0["x"]), int(g0["y"]), int(g0["k"])) != (r0.x, r0.y, r0.k):
                ml = tr.model.levels[0]
                sw, s1 = O.score(tr.fields[0], ml.t, ml.d, int(g0["x"]), int(g0["y"]), float(g0["theta"]))
                assert abs(sw - r0.sw) <= TOL and abs(s1 - r0.s1) <= TOL, (i, j, g0, r0)


def test_c5_continuous_refinement(c4):
    P, cfg, model_imgs, scenes = c4
    L = cfg["levels"]
    case("C5 4096 poses, 10 ascent steps, FP32 fields")
    models = [P.Model(m, L, cfg["tau_m"]) for m in model_imgs]
    images = [torch.from_numpy(s.image).cuda() for s in scenes]
    b = P.Batch(models, images, L, cfg["tau_s"], P.SearchParams(theta_step_top=cfg["theta_step_top"]))
    b.run()
    img_i, mod_i, start, truth = synth.c5_poses(scenes)
    pairs = img_i * len(models) + mod_i
    st32 = torch.from_numpy(start.astype(np.float32)).cuda()
    s0 = b.cont_score(0, st32, pairs).cpu().numpy().astype(np.float64)
    g = b.cont_score_backward(0, st32, pairs).cpu().numpy().astype(np.float64)
    newp, s1 = b.refine_continuous(st32, pairs, steps=10)
    newp = newp.cpu().numpy().astype(np.float64)
    s1 = s1.cpu().numpy().astype(np.float64)
    oms = [O.build_model(m, O.PyrParams(L, cfg["tau_m"])).levels[0] for m in model_imgs]
    rng = np.random.default_rng(505)
    fields = {}
    for j in rng.choice(len(start), 48, replace=False):
        i, k = int(img_i[j]), int(mod_i[j])
        if i not in fields:
            fields[i] = O.edge_field(scenes[i].image, cfg["tau_s"])
        p0 = start[j].astype(np.float32).astype(np.float64)
        ref, gref = O.cont_score(fields[i], oms[k].t, oms[k].d, *p0)
        assert abs(s0[j] - ref) <= 1e-5, (j, s0[j], ref)
        assert np.all(np.abs(g[j] - gref) <= 5e-5 + 1e-5 * np.abs(gref)), (j, g[j], gref)
        after, _ = O.cont_score(fields[i], oms[k].t, oms[k].d, *newp[j])
        assert after >= ref - 1e-6 and abs(s1[j] - after) <= 1e-6, (j, ref, after, s1[j])
    e0 = np.abs(start - truth)
    e1 = np.abs(newp - truth)
    e0[:, 2] = np.abs((start[:, 2] - truth[:, 2] + 180) % 360 - 180)
    e1[:, 2] = np.abs((newp[:, 2] - truth[:, 2] + 180) % 360 - 180)
    for name, e in (("start", e0), ("refined", e1)):
        print(f"{name}: mean |dx| {e[:, 0].mean():.3f} |dy| {e[:, 1].mean():.3f} |dth| {e[:, 2].mean():.3f}; "
              f"p95 {np.percentile(e, 95, axis=0).round(3)}; max {e.max(axis=0).round(3)}")
    assert np.all(s1 >= s0 - 1e-5)
    assert e1[:, :2].mean() < e0[:, :2].mean()
