"""Throughput of the detector's hot path on one MI355X.

Workload: 640x480 industrial scenes, 3 instances of a 128x128 polygon model,
4 levels, 1 degree at the top.  A detection is the full path for one image:
pyramid and edge-field build, exhaustive top-level search over 80x60
translations x 360 angles, candidate selection, refinement through 3 levels,
final selection.  Images are synthetic, seeded, and resident in device memory
before timing starts.

The headline leg (the timed steps): a step is one graph launch of all
--batch images, FP16 direction storage with FP32 accumulation and a certified
search by default; two such batches are in flight on two streams, the steps
alternating between them (--streams 1: one at a time).  The search schedule
is the autotuner's, chosen on that pipelined step.  Beside it: the batched
leg in the other precision, and the FP32 plain leg (one detection per call),
the bit-for-bit agreement of the legs' detections, top-1 against the oracle
per leg and ground-truth hits.  Prints one JSON line; `value` is pose
evaluations per second of the headline leg (exhaustive top-level poses;
refinement adds 27 x candidates x 3 per detection and is not counted);
detections/s and taps/s are given beside it.

`roofline`: the batched search kernel, its duration from HIP events around
its launches in eager steps after the timed region, on the stream it runs on;
bound by VALU issue: its executed VALU instructions per second (counted by
rocprofv3 for the schedule in use, profiles/dense_c2_valu.json) against the
issue peak of its inner loop's instruction mix (profiles/dense_c2_loop_mix.json),
with its HBM bytes per launch (profiles/dense_c2_traffic.json) and the
measured ceilings of the tm_probe kernels; the FLOP and tap figures beside.
`cpu_baseline`: the FP64 oracle on the host cores over a bounded sample.

--c4 adds the mixed batch (64 images of 640x480 to 2448x2048 against 8 models,
one graph launch per step) and the continuous refinement of 4096 poses over
its pairs (10 ascent steps); --c3 the 2048x2048 frames in FP16 and FP32;
--paper the search of the paper's own experiment shape (812x617, 3 px / 3 px /
3 deg steps over 90 deg, one level); --similarity the similarity pose (angles
x scales); --readings the four combinations of pyramid source (grey image or
gradient maps) and window vote (all taps or edge taps only), with their
ground-truth matches.  With the oracle on (no --no-cpu-baseline) the --c3 and
--c4 legs also time the oracle on their workloads.  --plain-only times the
plain leg alone.  --copy-probe ends the run with one 256 MiB elementwise copy,
the calibration of the HBM byte counters; --traffic-from, --valu-from and
--loop-mix-from turn rocprofv3 counter runs and the kernel's assembly into the
committed records; --trace-summary prints a rocprofv3 kernel trace as a table
with one row per kernel and launch shape.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
FLOP_PER_TAP = 3           # r . g: two products and a sum


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64, help="images per batched step")
    ap.add_argument("--precision", choices=["fp32", "fp16"], default="fp16",
                    help="direction storage of the batched leg (fp16: FP32 accumulation)")
    ap.add_argument("--cpu-seconds", type=float, default=30.0,
                    help="time budget of the oracle CPU baseline (it stops earlier once every image is done)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true", help="batched leg as plain enqueues instead of a graph launch")
    ap.add_argument("--streams", type=int, default=2,
                    help="batches in flight on their own streams in the batched leg (steps alternate between them)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default search-kernel form (no autotuning)")
    ap.add_argument("--c4", action="store_true", help="also time the 64 x 8 mixed batch and the C5 refinement")
    ap.add_argument("--c3", action="store_true",
                    help="also time the 2048x2048 five-level FP16 detection with its per-score error against FP32")
    ap.add_argument("--no-other", action="store_true", help="skip the batched leg of the other precision")
    ap.add_argument("--plain-only", action="store_true",
                    help="time the FP32 plain leg alone and print its figures (a profiling aid, not the bench line)")
    ap.add_argument("--loop-mix-from", metavar="K_SCORE_ASM",
                    help="record the search loop's VALU issue mix from the AMD assembly of k_score.hip")
    ap.add_argument("--valu-from", metavar="VALU_CSV",
                    help="write the search kernel's VALU-instruction entry from a rocprofv3 --pmc SQ_INSTS_VALU CSV "
                         "and exit")
    ap.add_argument("--similarity", action="store_true",
                    help="also time the similarity-pose search (x, y, theta, scale) on 64 scaled 640x480 scenes")
    ap.add_argument("--paper", action="store_true",
                    help="also time the paper's own search shape (812x617, 3 px / 3 deg steps, 90 deg, one level)")
    ap.add_argument("--readings", action="store_true",
                    help="also time and score the four combinations of pyramid source and window vote")
    ap.add_argument("--copy-probe", action="store_true", help="end with a 256 MiB elementwise copy (counter scale)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the search kernel's traffic entry from two rocprofv3 --pmc CSV files and exit")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="print a per-kernel, per-launch-shape table of a rocprofv3 --kernel-trace CSV and exit")
    return ap.parse_args()


COPY_PROBE_BYTES = 256 << 20
KERNEL_SRC = os.path.join(ROOT, "paper_2112_05576_amd", "csrc", "k_score.hip")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "dense_c2_traffic.json")


def _pmc_rows(path, counter):
    """(kernel name, value) per dispatch of one counter, in dispatch order."""
    import csv

    rows = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") == counter:
            rows.append((int(r.get("Dispatch_Id", len(rows))), r.get("Kernel_Name", ""), float(r["Counter_Value"]),
                         int(r.get("Grid_Size", 0)), int(r.get("Workgroup_Size", 0))))
    rows.sort()
    return [(n, v, g, wg) for _, n, v, g, wg in rows]


def trace_summary(path):
    """Markdown table of a rocprofv3 --kernel-trace CSV: one row per kernel
    and launch shape (workgroups x threads), so that launches of one kernel
    made by different legs of the benchmark are told apart."""
    import csv

    groups = {}
    total = 0
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        name = re.sub(r"\(.*$", "", name.replace("(anonymous namespace)::", "").replace("tmk::", ""))
        wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        groups.setdefault((name[:70], grid // max(wg, 1), wg), []).append(ns)
        total += ns
    print("| kernel | workgroups x threads | calls | median us | min us | max us | share % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for (name, nwg, wg), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        v.sort()
        print(f"| `{name}` | {nwg} x {wg} | {len(v)} | {v[len(v) // 2] / 1e3:.2f} | {v[0] / 1e3:.2f} | "
              f"{v[-1] / 1e3:.2f} | {100.0 * sum(v) / max(total, 1):.2f} |")


def traffic_from(fetch_csv, write_csv):
    """HBM bytes per launch of the batched search kernel: its FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the final 256 MiB elementwise copy of --copy-probe (read 256 MiB,
    write 256 MiB).  Run the counter passes with tuning on: the tuner
    dispatches every schedule of the search over the same batch, so one pass
    per counter gives the figure of each schedule, told apart by kernel
    variant, waves per chunk and workgroups per launch; the bench line takes
    the one of the schedule it runs."""
    out = {"kernel_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()}
    per = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _pmc_rows(path, counter)
        probe_name, probe, _, _ = rows[-1]
        if "elementwise" not in probe_name:
            raise SystemExit(f"last dispatch in {path} is not the copy probe: {probe_name[:80]}")
        scale = COPY_PROBE_BYTES / probe  # bytes per counted KiB
        out[f"{key}_probe_kib"] = probe
        out[f"{key}_scale_bytes_per_kib"] = scale
        n = 0
        for name, v, g, wg in rows:
            m = re.search(r"k_dense_fast<([^>]*)>", name)
            if not m:
                continue
            # template arguments: G, R, LC, PREC, VAR (the variant), VOTE[, SCREEN]; the FP16 batch's launches
            targs = [t.strip() for t in m.group(1).split(",")]
            if int(targs[3]) != 1:
                continue
            k = (int(targs[4]), wg // 64, g // wg)
            f = per.setdefault(k, {"variant": k[0], "waves_per_chunk": k[1], "workgroups": k[2]})
            f.setdefault(key, []).append(v * scale)
            n += 1
        if not n:
            raise SystemExit(f"no FP16 k_dense_fast dispatch in {path}")
    forms = []
    for f in per.values():
        if "fetch" not in f or "write" not in f:
            continue
        # the median launch: a batch's first launch after its creation reads
        # its inputs from cold caches and is not the steady state
        fb, wb = float(np.median(f["fetch"])), float(np.median(f["write"]))
        forms.append({"variant": f["variant"], "waves_per_chunk": f["waves_per_chunk"], "workgroups": f["workgroups"],
                      "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                      "launches": len(f["fetch"]), "fetch_bytes_max": max(f["fetch"])})
    out["forms"] = sorted(forms, key=lambda f: (f["variant"], f["waves_per_chunk"], f["workgroups"]))
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    _dump_forms(TRAFFIC_JSON, out)
    print(json.dumps(out))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(scenes, cfg, budget_s, paper=False):
    """The FP64 oracle, as it is, on the host cores: full detections of the
    benchmark's images, each once, in order, until all are done or the time
    budget is spent (and, with paper=True, one detection of the paper-shaped
    search, timed on its own).  Returns the baseline entry and the oracle's
    detections by image index, which the top-1 comparison of the GPU legs
    uses."""
    import oracle as O

    threads = O.default_threads()
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    L = cfg["levels"]
    model = O.build_model(scenes[0].model, O.PyrParams(L, cfg["tau_m"]))
    dets = {}
    poses = 0
    t0 = time.perf_counter()
    for i, sc in enumerate(scenes):
        tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp,
                      nthreads=threads, model=model)
        dets[i] = (tr.detections, tr.fields[0])
        poses += tr.top[0].size * O.level_count(osp, O.level_step(osp, L, L - 1))
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    n_top = len(model.levels[L - 1].t)
    res = {"value": poses / dt, "unit": "pose-evals/s", "cores": threads, "kind": "oracle",
           "taps_per_sec": poses * n_top * 9 / dt,
           "sample": f"{len(dets)} full detections of distinct 640x480 images (4 levels, 360 top angles), "
                     f"{dt:.1f} s",
           "cpu": _cpu_model()}
    # one more detection of the first image on a single thread
    sc = scenes[0]
    t0 = time.perf_counter()
    tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp, nthreads=1,
                  model=model)
    res["single_core_value"] = tr.top[0].size * O.level_count(osp, O.level_step(osp, L, L - 1)) / (
        time.perf_counter() - t0)
    # the single-instance configuration (128x128, one level, 72 angles), one
    # full detection
    import synth

    c1 = synth.CONFIGS[1]
    sc1 = synth.scene_for_config(1, 0)
    dt1, poses1, _, _, _ = oracle_detection(sc1.image, sc1.model, c1, c1["levels"], threads)
    res["configs"] = {"128x128 single instance, 1 level, 72 angles": {
        "ms_per_detection": dt1 * 1e3, "pose_evals_per_sec": poses1 / dt1, "sample": "1 full detection"}}
    if paper:
        sc = synth.scene_for_config(6, 0)
        pc = sc.config
        osp = O.SearchParams(step_x=3, step_y=3, theta_min=0.0, theta_range=90.0, theta_step_top=3.0, max_matches=1)
        t0 = time.perf_counter()
        O.detect(sc.image, sc.model, O.PyrParams(1, pc["tau_s"]), O.PyrParams(1, pc["tau_m"]), osp, nthreads=threads)
        res["paper_shape_ms_per_detection"] = (time.perf_counter() - t0) * 1e3
    return res, (model, dets)


def oracle_detection(image, model_img, cfg, L, threads):
    """One full oracle detection (pyramid, exhaustive top level, refinement,
    selection) timed on `threads` host threads: (seconds, top-level poses,
    detections, level-0 field, oracle model)."""
    import oracle as O

    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    om = O.build_model(model_img, O.PyrParams(L, cfg["tau_m"]))
    t0 = time.perf_counter()
    tr = O.detect(image, model_img, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), osp, nthreads=threads,
                  model=om)
    dt = time.perf_counter() - t0
    return dt, tr.top[0].size * O.level_count(osp, O.level_step(osp, L, L - 1)), tr.detections, tr.fields[0], om


def top1_one(g, ref, f0, om, cfg, L):
    """"identical", "tie" (the GPU top match's oracle S_w and S_1 within 1e-5
    of the oracle's top match), "differs" or "both_empty" for one image."""
    import oracle as O

    if len(ref) == 0 and len(g) == 0:
        return "both_empty"
    if len(ref) == 0 or len(g) == 0:
        return "differs"
    if (int(g[0]["x"]), int(g[0]["y"]), int(g[0]["k"])) == (ref[0].x, ref[0].y, ref[0].k):
        return "identical"
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    ml = om.levels[0]
    sw, s1 = O.score(f0, ml.t, ml.d, int(g[0]["x"]), int(g[0]["y"]),
                     O.theta(0.0, O.level_step(osp, L, 0), int(g[0]["k"])))
    return "tie" if abs(sw - ref[0].sw) <= 1e-5 and abs(s1 - ref[0].s1) <= 1e-5 else "differs"


def top1_vs_oracle(gpu_dets, oracle, cfg):
    """Top-1 of a GPU leg against the oracle's, image by image: the same pose
    ("identical"), a pose whose oracle S_w and S_1 are within 1e-5 of the
    oracle's top match ("tie"), or neither ("differs"); images where neither
    side detects anything are counted apart ("both_empty"), not as
    agreement."""
    import oracle as O

    model, dets = oracle
    ml = model.levels[0]
    L = cfg["levels"]
    osp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    step0 = O.level_step(osp, L, 0)
    out = {"identical": 0, "tie": 0, "differs": 0, "both_empty": 0, "images": len(dets)}
    for i, (ref, f0) in dets.items():
        g = gpu_dets[i]
        if len(ref) == 0 and len(g) == 0:
            out["both_empty"] += 1
        elif len(ref) == 0 or len(g) == 0:
            out["differs"] += 1
        elif (int(g[0]["x"]), int(g[0]["y"]), int(g[0]["k"])) == (ref[0].x, ref[0].y, ref[0].k):
            out["identical"] += 1
        else:
            sw, s1 = O.score(f0, ml.t, ml.d, int(g[0]["x"]), int(g[0]["y"]), O.theta(0.0, step0, int(g[0]["k"])))
            out["tie" if abs(sw - ref[0].sw) <= 1e-5 and abs(s1 - ref[0].s1) <= 1e-5 else "differs"] += 1
    return out


def traffic_entry(form):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source, for the search form now in use."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    d = json.load(open(TRAFFIC_JSON))
    h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if d.get("kernel_sha256") != h:
        return None
    for f in d.get("forms", []):
        if (f["variant"], f["waves_per_chunk"], f.get("workgroups")) == (
                form.get("variant"), form.get("waves_per_chunk"), form.get("workgroups")):
            return f["bytes_per_launch"]
    return None


def gt_hit(d, sc):
    return len(d) > 0 and any(np.hypot(d[0]["x"] - it.x, d[0]["y"] - it.y) <= 2.0 and
                              abs((d[0]["theta"] - it.theta + 180) % 360 - 180) <= 2.0 for it in sc.instances)


def _ang(a, b):
    return np.abs((a - b + 180.0) % 360.0 - 180.0)


def c4_legs(P, torch, steps, warmup, oracle_threads=0):
    """The mixed batch (FP16, graph launch) and the continuous refinement.
    With oracle_threads, the oracle's full detections of a 2-image x 8-model
    subset of the batch are timed on that many host threads and the batch's
    top-1 of those pairs compared with them."""
    import synth

    cfg = synth.C4
    L = cfg["levels"]
    mods = [synth.c4_model(k) for k in range(len(synth.C4_MODELS))]
    scenes = [synth.c4_image(i, [m[0] for m in mods]) for i in range(cfg["n_images"])]
    models = [P.Model(m[1], L, cfg["tau_m"]) for m in mods]
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    K = int(np.ceil(360.0 / cfg["theta_step_top"]))
    b = P.Batch(models, imgs, L, cfg["tau_s"], sp, precision=P.TM_FP16)
    tuned = b.tune(iterations=1)
    for _ in range(warmup):
        b.run(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run(graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res = b.results()
    nm = len(models)
    poses = sum((s.image.shape[0] >> (L - 1)) * (s.image.shape[1] >> (L - 1)) for s in scenes) * nm * K
    taps = sum((s.image.shape[0] >> (L - 1)) * (s.image.shape[1] >> (L - 1)) * m.level_info(L - 1)[2]
               for s in scenes for m in models) * K * 9
    found = total = 0
    for i, s in enumerate(scenes):
        for it, k in zip(s.instances, s.models):
            total += 1
            d = res[i * nm + k]
            found += any(np.hypot(x["x"] - it.x, x["y"] - it.y) <= 2.0 and _ang(x["theta"], it.theta) <= 2.0
                         for x in d)
    c4 = {"workload": f"{len(scenes)} images (640x480 / 1280x1024 / 2448x2048) x {nm} models "
                      f"({', '.join(str(m.level_info(0)[2]) for m in models)} level-0 points), FP16, graph launch",
          "ms_per_step": dt * 1e3, "detections_per_sec": len(scenes) * nm / dt, "pose_evals_per_sec": poses / dt,
          "taps_per_sec": taps / dt, "instances_found": f"{found}/{total}", "search_form": tuned}
    if oracle_threads:
        secs, n_o, top1 = 0.0, 0, {}
        for i in range(2):
            for k in range(nm):
                dt_o, poses_o, ref, f0, om = oracle_detection(scenes[i].image, mods[k][1], cfg, L, oracle_threads)
                secs += dt_o
                n_o += poses_o
                r = top1_one(res[i * nm + k], ref, f0, om, cfg, L)
                top1[r] = top1.get(r, 0) + 1
        # linear extrapolation to the whole batch by top-level work (translations x angles x points)
        def work(i, k):
            return (scenes[i].image.shape[0] >> (L - 1)) * (scenes[i].image.shape[1] >> (L - 1)) * \
                models[k].level_info(L - 1)[2]

        scale = sum(work(i, k) for i in range(len(scenes)) for k in range(nm)) / sum(
            work(i, k) for i in range(2) for k in range(nm))
        c4["cpu_oracle"] = {"ms_per_detection": secs / (2 * nm) * 1e3, "pose_evals_per_sec": n_o / secs,
                            "extrapolated_batch_s": secs * scale,
                            "extrapolation": "linear in top-level translations x points over the 512 pairs "
                                             "(not measured)",
                            "cores": oracle_threads,
                            "sample": f"images 0-1 ({scenes[0].image.shape[1]}x{scenes[0].image.shape[0]}, "
                                      f"{scenes[1].image.shape[1]}x{scenes[1].image.shape[0]}) x {nm} models, "
                                      f"full detections"}
        c4["top1_vs_oracle_subset"] = top1
    # C5: 4096 poses near the truth, 10 ascent steps on FP32 fields
    b32 = P.Batch(models, imgs, L, cfg["tau_s"], sp, precision=P.TM_FP32)
    b32.run()
    img_i, mod_i, start, truth = synth.c5_poses(scenes)
    pairs = torch.from_numpy(img_i * nm + mod_i).cuda()
    st = torch.from_numpy(start.astype(np.float32)).cuda()
    b32.refine_continuous(st, pairs, steps=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        newp, _ = b32.refine_continuous(st, pairs, steps=10)
    torch.cuda.synchronize()
    dt5 = (time.perf_counter() - t0) / reps
    newp = newp.cpu().numpy().astype(np.float64)
    e0 = np.abs(start - truth)
    e1 = np.abs(newp - truth)
    e0[:, 2], e1[:, 2] = _ang(start[:, 2], truth[:, 2]), _ang(newp[:, 2], truth[:, 2])

    def stats(e):
        return {k: {"mean": float(e[:, j].mean()), "p95": float(np.percentile(e[:, j], 95)),
                    "max": float(e[:, j].max())} for j, k in enumerate(("dx", "dy", "dtheta_deg"))}

    c5 = {"workload": "4096 poses of the mixed batch's instances, +-1.5 px / +-2 deg, 10 ascent steps (gradient "
                      "kernel + FP64 line search of 6 step lengths per step)",
          "ms_per_refinement": dt5 * 1e3, "poses_per_sec": len(start) / dt5,
          "error_start": stats(e0), "error_refined": stats(e1)}
    return c4, c5


def similarity_leg(P, torch, steps):
    """64 scaled 640x480 scenes (instances scaled by U[0.8, 1.2]) searched over
    5 scales x 90 angles at the top of 3 levels, batched (FP16, graph launch,
    tuned); ground-truth hits within 2 px, 2 degrees and 0.05 in scale."""
    import synth

    cfg = synth.CONFIGS[7]
    L = cfg["levels"]
    scenes = [synth.scene_for_config(7, i) for i in range(64)]
    model = P.Model(scenes[0].model, L, cfg["tau_m"])
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"], scale_min=cfg["scale_min"],
                        scale_step=cfg["scale_step"], scale_count=cfg["scale_count"])
    b = P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=P.TM_FP16)
    tuned = b.tune(iterations=2)
    b.run(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run(graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res = b.results()
    K = int(np.ceil(360.0 / cfg["theta_step_top"]))
    top = (480 >> (L - 1)) * (640 >> (L - 1)) * K * cfg["scale_count"]
    hits = sum(len(d) > 0 and any(np.hypot(d[0]["x"] - it.x, d[0]["y"] - it.y) <= 2.0 and
                                  _ang(d[0]["theta"], it.theta) <= 2.0 and
                                  abs(sp.scale(int(d[0]["j"])) - it.scale) <= 0.05 for it in sc.instances)
               for d, sc in zip(res, scenes))
    return {"workload": f"64 images of 640x480 with 3 instances scaled by U[0.8, 1.2]; {L} levels, top level "
                        f"{640 >> (L - 1)}x{480 >> (L - 1)} x {K} angles x {cfg['scale_count']} scales "
                        f"({cfg['scale_min']} .. {sp.scale(cfg['scale_count'] - 1):.1f}); FP16, graph launch",
            "ms_per_step": dt * 1e3, "detections_per_sec": len(scenes) / dt,
            "pose_evals_per_sec": top * len(scenes) / dt, "top1_ground_truth_hits": f"{hits}/{len(scenes)}",
            "search_form": tuned}


def readings_leg(P, torch, steps):
    """The two readings of the method that the paper leaves open, each on and
    off: the pyramid of the grey image or of the gradient maps, and a window
    vote over all taps or over edge taps only.  Per combination the headline
    batch (64 C2 scenes of 640x480, FP16, graph launch, tuned) is timed, and
    its detections are matched against the ground truth: top-1 hits, the
    instances found by any detection (within 2 px and 2 degrees, and within
    2 px alone) and the detections within 2 px of no instance."""
    import synth

    cfg = synth.CONFIGS[2]
    L = cfg["levels"]
    scenes = [synth.scene_for_config(2, i) for i in range(64)]
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    n_inst = sum(len(sc.instances) for sc in scenes)
    out = {}
    for src_name, src in (("grey", P.TM_PYR_GREY), ("gradient", P.TM_PYR_GRADIENT)):
        model = P.Model(scenes[0].model, L, cfg["tau_m"], source=src)
        for vote_name, vote in (("all", P.TM_VOTE_ALL), ("edge", P.TM_VOTE_EDGE)):
            sp = P.SearchParams(theta_step_top=cfg["theta_step_top"], vote=vote)
            b = P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=P.TM_FP16, source=src)
            b.tune(iterations=2)
            b.run(graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                b.run(graph=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res = b.results()
            found = found_xy = stray = 0
            for d, sc in zip(res, scenes):
                at = [[np.hypot(x["x"] - it.x, x["y"] - it.y) <= 2.0 for it in sc.instances] for x in d]
                near = [[a and _ang(x["theta"], it.theta) <= 2.0 for a, it in zip(row, sc.instances)]
                        for row, x in zip(at, d)]
                found += sum(any(row[i] for row in near) for i in range(len(sc.instances)))
                found_xy += sum(any(row[i] for row in at) for i in range(len(sc.instances)))
                stray += sum(not any(row) for row in at)
            out[f"{src_name}_pyramid+{vote_name}_taps"] = {
                "ms_per_step": dt * 1e3, "detections_per_sec": len(scenes) / dt,
                "top1_ground_truth_hits": f"{sum(gt_hit(d, sc) for d, sc in zip(res, scenes))}/{len(scenes)}",
                "instances_found": f"{found}/{n_inst}", "instances_found_xy_only": f"{found_xy}/{n_inst}",
                "unmatched_detections": stray,
                "model_points_top": model.level_info(L - 1)[2], "search_form": b.search_form()}
    out["workload"] = ("64 images of 640x480 (3 instances each), 4 levels, 1 deg top step, FP16, graph launch; "
                       "matches within 2 px and 2 deg")
    return out


def paper_leg(P, torch, steps):
    """The search of the paper's experiment on synthetic 812x617 frames: every
    3rd pixel, 31 angles over 90 degrees, one level, the single best pose;
    one tm_detect per frame (FP32, the generic search path)."""
    import synth

    scenes = [synth.scene_for_config(6, i) for i in range(8)]
    cfg = scenes[0].config
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    model = P.Model(scenes[0].model, 1, cfg["tau_m"])
    kw = dict(step_x=3, step_y=3, theta_min=0.0, theta_range=90.0, theta_step_top=3.0, max_matches=1)
    sp = P.SearchParams(**kw)
    pyr = P.Pyramid(imgs[0], 1, cfg["tau_s"])
    outs = torch.empty((len(imgs), 1, P.tm.POSE_WORDS), dtype=torch.int32, device="cuda")
    nout = torch.zeros((len(imgs),), dtype=torch.int32, device="cuda")

    def one(i):
        j = i % len(imgs)
        pyr.update(imgs[j])
        P.detect_async(model, pyr, sp, outs[j], nout[j:j + 1])

    for i in range(len(imgs)):
        one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one(i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    dets = [P.poses_to_numpy(outs[j], int(nout[j].item())) for j in range(len(imgs))]
    hits = sum(gt_hit(d, sc) for d, sc in zip(dets, scenes))
    poses = 271 * 206 * 31
    res = {"workload": "812x617 frames, 1 instance of a 96x96 polygon model (847 points), steps 3 px / 3 px / 3 deg "
                       "over 90 deg (271x206x31 poses), 1 level, best pose; FP32, one detection per call",
           "ms_per_detection": dt * 1e3, "pose_evals_per_sec": poses / dt, "top1_ground_truth_hits":
           f"{hits}/{len(imgs)}"}
    return res


VALU_JSON = os.path.join(ROOT, "profiles", "dense_c2_valu.json")
LOOP_MIX_JSON = os.path.join(ROOT, "profiles", "dense_c2_loop_mix.json")
SIMDS = 1024                 # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9             # MI355X peak engine clock (published)
# Issue cycles of one wave64 VALU instruction by class: the packed-half dot
# product, DPP-modified and three-operand max instructions take 4 (the class
# probes measure 4.1 to 4.6 at the clock they run at), the rest 2 (plain
# adds measure 2.2).
SLOW_VALU = ("v_dot2", "v_max3", "v_min3", "v_med3")


def _dump_forms(path, out):
    """A record with its forms one per line (short files for profiles/)."""
    head = {k: v for k, v in out.items() if k != "forms"}
    with open(path, "w") as fh:
        fh.write(json.dumps(head)[:-1] + ', "forms": [\n')
        fh.write(",\n".join(json.dumps(f, separators=(",", ":")) for f in out["forms"]))
        fh.write("\n]}\n")


def _valu_cycles(mnemonic, operands):
    return 4 if mnemonic.startswith(SLOW_VALU) or mnemonic.endswith("_dpp") or "row_" in operands or \
        "wave_sh" in operands or "quad_perm" in operands else 2


def loop_mix_from(asm_path):
    """The VALU mix of the search kernel's innermost loop, per instantiation
    of k_dense_fast, from the AMD assembly of k_score.hip (hipcc
    --cuda-device-only -S): instructions by issue class and the mean issue
    cycles per instruction, which with the SIMD count and the engine clock
    give the issue peak of that loop; recorded with the SHA-256 of the
    source."""
    lines = open(asm_path).read().splitlines()
    fn_re = re.compile(r"^(_ZN3tmk\S*k_dense_fastILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELb([01])E\S*):")
    out = {"kernel_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest(), "clock_hz": CLOCK_HZ,
           "simds": SIMDS, "forms": []}
    i = 0
    while i < len(lines):
        m = fn_re.match(lines[i])
        if not m:
            i += 1
            continue
        j = i + 1
        while j < len(lines) and "s_endpgm" not in lines[j]:
            j += 1
        body = lines[i + 1:j]
        labels = {}
        loops = []
        for k, ln in enumerate(body):
            lm = re.match(r"^(\.LBB\w+):", ln)
            if lm:
                labels[lm.group(1)] = k
            bm = re.match(r"^\s*s_c?branch\w*\s+(\.LBB\w+)", ln)
            if bm and bm.group(1) in labels and labels[bm.group(1)] < k:
                loops.append((labels[bm.group(1)], k))
        # innermost loops (no other loop inside); the search loop is the one
        # with the most cross-lane (DPP) window maxima, then products (dot2,
        # fma, mul), then VALU instructions
        inner = [(a, b) for a, b in loops if not any(a < c and d < b for c, d in loops if (c, d) != (a, b))]
        best = None
        for a, b in inner:
            cls = {}
            n = cyc = lds = prod = dpp = 0
            for ln in body[a:b + 1]:
                t = ln.strip().split(None, 1)
                if t and t[0].startswith("ds_read"):
                    lds += 1
                if not t or not t[0].startswith("v_"):
                    continue
                if t[0].startswith(("v_dot2", "v_fma", "v_mul_f32", "v_pk_fma", "v_pk_mul")):
                    prod += 1
                c = _valu_cycles(t[0], t[1] if len(t) > 1 else "")
                if "dpp" in t[0] or "row_" in ln or "wave_sh" in ln or "quad_perm" in ln:
                    dpp += 1
                cls[t[0]] = cls.get(t[0], 0) + 1
                n += 1
                cyc += c
            if n and (best is None or (dpp, prod, n) > (best["dpp"], best["products"], best["valu"])):
                best = {"valu": n, "cycles": cyc, "lds_reads": lds, "products": prod, "dpp": dpp,
                        "by_mnemonic": dict(sorted(cls.items(), key=lambda kv: -kv[1]))}
        if best:
            G, R, LC, prec, var, vote, screen = (int(x) for x in m.groups()[1:])
            out["forms"].append({"precision": "fp16" if prec else "fp32", "variant": var, "vote": vote,
                                 "screen": bool(screen), "lc": LC, "loop_valu": best["valu"],
                                 "loop_issue_cycles": best["cycles"], "loop_lds_reads": best["lds_reads"],
                                 "cycles_per_instr": best["cycles"] / best["valu"],
                                 "by_mnemonic": best["by_mnemonic"]})
        i = j
    # one entry per form: the smallest field-tile width (the 640x480 batches'), its six most frequent mnemonics
    keep = {}
    for f in out["forms"]:
        k = (f["precision"], f["variant"], f["vote"], f["screen"])
        if k not in keep or f["lc"] < keep[k]["lc"]:
            keep[k] = dict(f, by_mnemonic=dict(list(f["by_mnemonic"].items())[:6]))
    out["forms"] = [keep[k] for k in sorted(keep)]
    _dump_forms(LOOP_MIX_JSON, out)
    print(json.dumps({k: v for k, v in out.items() if k != "forms"} | {"forms": len(out["forms"])}))


def loop_mix_entry(form, precision, vote=0):
    """Mean issue cycles per VALU instruction of the search loop of the form
    in use, if recorded on the current k_score.hip (the loop of the smallest
    field-tile width, the one the 640x480 batches use, is the one recorded)."""
    if not os.path.exists(LOOP_MIX_JSON):
        return None
    d = json.load(open(LOOP_MIX_JSON))
    if d.get("kernel_sha256") != hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest():
        return None
    fs = [f for f in d.get("forms", []) if (f["precision"], f["variant"], f["vote"], f["screen"]) ==
          (precision, form.get("variant"), vote, precision == "fp16")]
    if not fs:
        return None
    f = fs[0]
    return {"cycles_per_instr": f["cycles_per_instr"], "loop_valu": f["loop_valu"],
            "counted_in": os.path.relpath(LOOP_MIX_JSON, ROOT)}


def valu_from(csv_path):
    """Executed VALU instructions per launch of the search kernel, from a
    rocprofv3 --pmc SQ_INSTS_VALU CSV of this benchmark (tuning on, so that
    every schedule of the batched search is dispatched): the median over the
    launches of each schedule (variant, waves per chunk, workgroups per
    launch, precision, screen), with the SHA-256 of k_score.hip they were
    counted on."""
    out = {"kernel_sha256": hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest(), "forms": []}
    rows = _pmc_rows(csv_path, "SQ_INSTS_VALU")
    per = {}
    for n, v, g, wg in rows:
        m = re.search(r"k_dense_fast<([^>]*)>", n)
        if not m:
            continue
        targs = m.group(1).split(",")
        prec, var = int(targs[3]), int(targs[4])
        screen = len(targs) > 6 and targs[6].strip() == "true"
        per.setdefault((var, wg // 64, g // wg, prec, screen), []).append(v)
    for (var, wa, nwg, prec, screen), v in sorted(per.items()):
        out["forms"].append({"variant": var, "waves_per_chunk": wa, "workgroups": nwg,
                             "precision": "fp16" if prec else "fp32", "screen": screen,
                             "valu_instr_per_launch": float(np.median(v)), "launches": len(v)})
    _dump_forms(VALU_JSON, out)
    print(json.dumps(out))


def valu_entry(form, precision):
    """The counted VALU instructions per launch of the form in use, if they
    were counted on the current k_score.hip."""
    if not os.path.exists(VALU_JSON):
        return None
    d = json.load(open(VALU_JSON))
    if d.get("kernel_sha256") != hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest():
        return None
    for f in d.get("forms", []):
        if (f["variant"], f["waves_per_chunk"], f.get("workgroups"), f["precision"]) == (
                form.get("variant"), form.get("waves_per_chunk"), form.get("workgroups"), precision) and \
                f["screen"] == (precision == "fp16"):
            return {"valu_instr_per_launch": f["valu_instr_per_launch"], "counted_in": os.path.relpath(VALU_JSON, ROOT)}
    return None


def c3_leg(P, torch, steps, oracle_threads=0):
    """The large-frame precision configuration: 2048x2048 scenes with 5
    instances of a 256x256 model, 5 levels, 8 degrees at the top (0.5 at
    level 0).  One tm_detect per frame in FP16 (certified search, FP32
    refinement) and in FP32, timed; their detections compared bit for bit;
    and the per-score error of the FP16 top-level map against the FP32 map
    (both at the top level, every translation's best angle).  With
    oracle_threads, the oracle's full detection of each frame is timed on
    that many host threads and both legs' top-1 compared with it."""
    import synth

    scenes = [synth.scene_for_config(3, i) for i in range(2)]
    cfg = scenes[0].config
    L = cfg["levels"]
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    model = P.Model(scenes[0].model, L, cfg["tau_m"])
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    out = {"workload": "2048x2048, 5 instances of a 256x256 model, 5 levels, 8 deg top step (45 angles, 0.5 deg at "
                       "level 0), one detection per call"}
    dets = {}
    maps = {}
    for name, prec in (("fp16", P.TM_FP16), ("fp32", P.TM_FP32)):
        pyr = P.Pyramid(imgs[0], L, cfg["tau_s"], precision=prec)
        o = torch.empty((sp.max_matches, P.tm.POSE_WORDS), dtype=torch.int32, device="cuda")
        n = torch.zeros(1, dtype=torch.int32, device="cuda")
        for i in range(2):
            pyr.update(imgs[i % 2])
            P.detect_async(model, pyr, sp, o, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            pyr.update(imgs[i % 2])
            P.detect_async(model, pyr, sp, o, n)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        dets[name] = []
        for im in imgs:
            pyr.update(im)
            dets[name].append(P.detect(model, pyr, sp))
        pyr.update(imgs[0])
        maps[name] = [t.float().cpu().numpy() for t in P.score_map(model, pyr, L - 1, sp)]
        out[name] = {"ms_per_detection": dt * 1e3, "detections_per_sec": 1.0 / dt,
                     "detections": [len(d) for d in dets[name]]}
        pyr.free()
    out["fp16_equals_fp32_bit_for_bit"] = all(a.tobytes() == b.tobytes() for a, b in zip(dets["fp16"], dets["fp32"]))
    if oracle_threads:
        # the oracle's full detection of each frame, timed, and the top-1 of both legs against it
        secs, poses = 0.0, 0
        top1 = {"fp16": {}, "fp32": {}}
        for i, sc in enumerate(scenes):
            dt_o, n_o, ref, f0, om = oracle_detection(sc.image, sc.model, cfg, L, oracle_threads)
            secs += dt_o
            poses += n_o
            for name in ("fp16", "fp32"):
                r = top1_one(dets[name][i], ref, f0, om, cfg, L)
                top1[name][r] = top1[name].get(r, 0) + 1
        out["cpu_oracle"] = {"ms_per_detection": secs / len(scenes) * 1e3, "pose_evals_per_sec": poses / secs,
                             "cores": oracle_threads, "sample": f"{len(scenes)} full detections"}
        out["top1_vs_oracle"] = top1
    e = np.abs(maps["fp16"][0].astype(np.float64) - maps["fp32"][0])
    out["fp16_map_error_vs_fp32"] = {"max": float(e.max()), "mean": float(e.mean()),
                                     "p99": float(np.percentile(e, 99)), "translations": int(e.size),
                                     "angle_differs": int((maps["fp16"][2] != maps["fp32"][2]).sum())}
    return out


def batched_leg(P, torch, model, imgs, L, cfg, sp, prec, args, stream):
    """One batched leg as the headline times it: --streams batches over the
    same images (each with its own pyramids and scratch, the same search
    form) on their own streams of default priority, the steps alternating
    between them, every step one whole pass over its batch.  Returns its
    timing, detections and search form, and the search kernel's launch time
    from HIP events around its launches in eager steps after the timed
    region (one batch, same stream, nothing overlapping it)."""
    ns = max(1, args.streams)
    batches = [P.Batch([model], imgs, L, cfg["tau_s"], sp, precision=prec) for _ in range(ns)]
    batch = batches[0]
    streams = [stream] + [torch.cuda.Stream() for _ in range(ns - 1)]
    graph = not args.eager
    # the autotuner picks the search's schedule (variant, waves per chunk,
    # angles per chunk); with two batches in flight it times the chunkings on
    # their pipelined step, and both keep its choice (all schedules give the
    # same detections)
    tuned = None
    if not args.no_tune:
        if ns >= 2:
            tuned = batch.tune(iterations=3, partner=batches[1], partner_stream=streams[1])
            for b in batches[2:]:
                b.set_form(tuned["variant"], tuned["waves_per_chunk"], tuned["chunk_angles"])
        else:
            tuned = batch.tune(iterations=3)
    form = dict(batch.search_form(), workgroups=batch.search_launch()["workgroups"])
    chosen_by = "default" if tuned is None else ("autotuner, pipelined step" if ns >= 2 else "autotuner, search launch")
    for i in range(max(args.warmup, ns)):
        batches[i % ns].run(streams[i % ns], graph=graph)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for st in streams[1:]:
        st.wait_event(ev0)
    for i in range(args.steps):
        batches[i % ns].run(streams[i % ns], graph=graph)
    for st in streams[1:]:
        e = torch.cuda.Event()
        e.record(st)
        stream.wait_event(e)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    elapsed = max(wall, ev0.elapsed_time(ev1) / 1e3)
    dets = batch.results()
    for b in batches[1:]:  # the same images give the same detections on every batch
        assert all(len(x) == len(y) and (x.tobytes() == y.tobytes()) for x, y in zip(b.results(), dets))
    P.timing_read()
    P.timing_enable(True)
    for _ in range(max(5, min(args.steps, 20))):
        batch.run()
    torch.cuda.synchronize()
    P.timing_enable(False)
    dense_ms, launches = P.timing_read()
    for b in batches:
        b.free()
    return {"elapsed": elapsed, "dets": dets, "form": dict(form, tuned=tuned is not None, chosen_by=chosen_by),
            "launch_s": dense_ms / max(launches, 1) / 1e3, "ns": ns, "nb": len(imgs)}


def progress(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ceilings(P):
    """Measured ceilings of the search kernel's roofs (tm_probe): its VALU
    instruction mix, each instruction class of it, plain FP32 adds, its LDS
    read pattern and an HBM copy."""
    return {"valu_mix_wave_instr_per_s": P.probe_rate(P.tm.PROBE_VALU_MIX, 4000),
            "valu_dot2_wave_instr_per_s": P.probe_rate(P.tm.PROBE_DOT2, 4000),
            "valu_max_dpp_wave_instr_per_s": P.probe_rate(P.tm.PROBE_MAX_DPP, 4000),
            "valu_max3_wave_instr_per_s": P.probe_rate(P.tm.PROBE_MAX3, 4000),
            "valu_add_wave_instr_per_s": P.probe_rate(P.tm.PROBE_VALU_ADD, 4000),
            "lds_bytes_per_s": P.probe_rate(P.tm.PROBE_LDS, 4000),
            "hbm_bytes_per_s": P.probe_rate(P.tm.PROBE_HBM, 1)}


def main():
    args = parse()
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.traffic_from:
        traffic_from(*args.traffic_from)
        return
    if args.valu_from:
        valu_from(args.valu_from)
        return
    if args.loop_mix_from:
        loop_mix_from(args.loop_mix_from)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is single-GPU by design.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2112_05576_amd as P
    import synth

    cfg = dict(synth.CONFIGS[2])
    L = cfg["levels"]
    nb = args.batch
    scenes = [synth.scene_for_config(2, i) for i in range(nb)]
    imgs = [torch.from_numpy(s.image).cuda() for s in scenes]
    model = P.Model(scenes[0].model, L, cfg["tau_m"])
    sp = P.SearchParams(theta_step_top=cfg["theta_step_top"])
    stream = torch.cuda.current_stream()
    prec_b = P.TM_FP16 if args.precision == "fp16" else P.TM_FP32
    K = int(np.ceil(360.0 / cfg["theta_step_top"]))
    n_top = model.level_info(L - 1)[2]

    # ---- FP32 plain, one detection (pyramid + search) per call
    progress("FP32 plain leg")
    pyr = P.Pyramid(imgs[0], L, cfg["tau_s"], precision=P.TM_FP32)
    H3, W3 = pyr.level_shape(L - 1)
    poses_per_det = H3 * W3 * K
    taps_per_det = poses_per_det * n_top * 9
    cap = sp.max_matches
    outs = torch.empty((nb, cap, P.tm.POSE_WORDS), dtype=torch.int32, device="cuda")
    nout = torch.zeros((nb,), dtype=torch.int32, device="cuda")

    def plain(i):
        j = i % nb
        pyr.update(imgs[j])
        P.detect_async(model, pyr, sp, outs[j], nout[j:j + 1])

    for i in range(max(args.warmup, nb)):
        plain(i)
    torch.cuda.synchronize()
    plain_steps = max(args.steps, 1) * 4
    t0 = time.perf_counter()
    for i in range(plain_steps):
        plain(i)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    # the search kernel's duration from events around it, in calls of their
    # own (the events stay out of the timed detections above)
    P.timing_read()
    P.timing_enable(True)
    for i in range(nb):
        plain(i)
    torch.cuda.synchronize()
    P.timing_enable(False)
    plain_dense_ms, plain_launches = P.timing_read()
    plain_dets = [P.poses_to_numpy(outs[j], int(nout[j].item())) for j in range(nb)]
    pyr.free()
    plain_res = {"pose_evals_per_sec": poses_per_det * plain_steps / plain_s,
                 "detections_per_sec": plain_steps / plain_s,
                 "us_per_detection": plain_s / plain_steps * 1e6,
                 "search_kernel_us": plain_dense_ms / max(plain_launches, 1) * 1e3}
    if args.plain_only:
        print(json.dumps({"fp32_plain": plain_res, "detections": plain_steps,
                          "workload": "one 640x480 image per call, pyramid + detection, FP32"}), flush=True)
        return

    # ---- the headline: the batched leg in the asked precision (FP16 by
    # default); beside it the other precision's batched leg
    progress(f"{args.precision} batched leg")
    head = batched_leg(P, torch, model, imgs, L, cfg, sp, prec_b, args, stream)
    other_prec = P.TM_FP32 if prec_b == P.TM_FP16 else P.TM_FP16
    other_name = "fp32" if other_prec == P.TM_FP32 else "fp16"
    if not args.no_other:
        progress(f"{other_name} batched leg")
    other = batched_leg(P, torch, model, imgs, L, cfg, sp, other_prec, args, stream) if not args.no_other else None
    bdets = head["dets"]
    elapsed = head["elapsed"]
    hits = {"fp32_plain": sum(gt_hit(d, sc) for d, sc in zip(plain_dets, scenes)),
            f"{args.precision}_batched": sum(gt_hit(d, sc) for d, sc in zip(bdets, scenes))}
    same_bits = {f"{args.precision}_batched_vs_fp32_plain":
                 sum(a.tobytes() == b.tobytes() for a, b in zip(bdets, plain_dets))}
    if other is not None:
        hits[f"{other_name}_batched"] = sum(gt_hit(d, sc) for d, sc in zip(other["dets"], scenes))
        same_bits[f"{args.precision}_batched_vs_{other_name}_batched"] = sum(
            a.tobytes() == b.tobytes() for a, b in zip(bdets, other["dets"]))

    dense_avg_s = head["launch_s"]
    flops = taps_per_det * nb * FLOP_PER_TAP
    achieved = flops / dense_avg_s / 1e12
    dets_per_s = nb * args.steps / elapsed
    progress("ceiling probes")
    ceil = ceilings(P)
    # the search is bound by VALU issue: the roofline is its executed VALU
    # instructions per second (counted by SQ_INSTS_VALU for the schedule in
    # use) against the issue peak of its inner loop's instruction mix (SIMDs x
    # engine clock / issue cycles per instruction of that loop); the FLOP and
    # tap figures are given beside it (they count the method's 9 n taps per
    # pose, which the kernel shares between neighbouring translations, so they
    # can exceed the vector peak)
    roof = {"kernel": "k_dense_fast (exhaustive top-level search, all images of the step)", "bound": "alu",
            "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic_entry(head["form"]),
            "launch_us": dense_avg_s * 1e6}
    valu = valu_entry(head["form"], args.precision)
    mix = loop_mix_entry(head["form"], args.precision)
    if valu is not None and mix is not None:
        rate = valu["valu_instr_per_launch"] / dense_avg_s
        peak = SIMDS * CLOCK_HZ / mix["cycles_per_instr"]
        roof.update({"achieved": rate / 1e12, "peak": peak / 1e12, "unit": "T VALU wave-instr/s", "frac": rate / peak,
                     "peak_basis": f"{SIMDS} SIMDs x {CLOCK_HZ / 1e9:.1f} GHz / {mix['cycles_per_instr']:.3f} issue "
                                   f"cycles per instruction of the search loop ({mix['loop_valu']} VALU: dot2, DPP "
                                   f"and 3-operand max at 4 cycles, the rest at 2)",
                     "valu_instr_per_launch": valu["valu_instr_per_launch"],
                     "counted_in": [valu["counted_in"], mix["counted_in"]]})
    roof.update({"flop": {"achieved_tflops": achieved, "peak_tflops": PEAK_FP32_TFLOPS,
                          "frac": achieved / PEAK_FP32_TFLOPS, "flop_per_launch": flops,
                          "note": "3 FLOP per algorithmic tap (9 n per pose)"},
                 "taps_per_s": taps_per_det * nb / dense_avg_s,
                 "lds_tap_ceiling_taps_per_s": ceil["lds_bytes_per_s"] / (4 if prec_b == P.TM_FP16 else 8),
                 "measured_ceilings": ceil})
    if valu is not None:
        roof["executed_valu_vs_mix_probe"] = valu["valu_instr_per_launch"] / dense_avg_s / ceil[
            "valu_mix_wave_instr_per_s"]
    res = {
        "metric": "pose-evals/sec and detections/sec at 640x480 (FP32 plain vs FP16 batched, equal top-1)",
        "value": poses_per_det * dets_per_s,
        "unit": "pose-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 (f32 accumulation)" if args.precision == "fp16" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{nb} images of 640x480 (3 instances of a 128x128 polygon model each) per step, "
                               "4 levels, 1 deg top step (80x60x360 top poses per image), full detection",
                   "images_per_step": nb, "levels": L, "top_angles": K, "model_points_top": n_top,
                   "path": f"{args.precision}-batched" + ("" if args.eager else ", graph launch")
                           + (f", {head['ns']} batches in flight on {head['ns']} streams" if head["ns"] > 1 else "")
                           + (", certified FP16 search, FP32 refinement" if args.precision == "fp16" else ""),
                   "search_form": head["form"]},
        "detections_per_sec": dets_per_s,
        "taps_per_sec": taps_per_det * dets_per_s,
        "fp32_plain": plain_res,
        "same_detections_bit_for_bit": same_bits,
        "top1_ground_truth_hits": {k: f"{v}/{nb}" for k, v in hits.items()},
        "roofline": roof,
    }
    if other is not None:
        res[f"{other_name}_batched"] = {"ms_per_step": other["elapsed"] * 1e3 / args.steps,
                                        "detections_per_sec": nb * args.steps / other["elapsed"],
                                        "pose_evals_per_sec": poses_per_det * nb * args.steps / other["elapsed"],
                                        "search_launch_us": other["launch_s"] * 1e6, "search_form": other["form"]}
    oracle_threads = 0
    if not args.no_cpu_baseline:
        import oracle as O

        oracle_threads = O.default_threads()
    if args.c4:
        progress("c4 leg")
        res["c4"], res["c5"] = c4_legs(P, torch, max(2, args.steps // 10), 1, oracle_threads)
    if args.c3:
        progress("c3 leg")
        res["c3"] = c3_leg(P, torch, max(5, args.steps // 5), oracle_threads)
    if args.paper:
        progress("paper leg")
        res["paper_shape"] = paper_leg(P, torch, max(8, args.steps))
    if args.similarity:
        progress("similarity leg")
        res["similarity"] = similarity_leg(P, torch, max(5, args.steps // 4))
    if args.readings:
        progress("readings leg")
        res["readings"] = readings_leg(P, torch, max(5, args.steps // 4))
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        res["cpu_baseline"], oracle = cpu_baseline(scenes, cfg, args.cpu_seconds, paper=args.paper)
        res["top1_vs_oracle"] = {"fp32_plain": top1_vs_oracle(plain_dets, oracle, cfg),
                                 f"{args.precision}_batched": top1_vs_oracle(bdets, oracle, cfg)}
        if other is not None:
            res["top1_vs_oracle"][f"{other_name}_batched"] = top1_vs_oracle(other["dets"], oracle, cfg)
    if args.copy_probe:
        x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
