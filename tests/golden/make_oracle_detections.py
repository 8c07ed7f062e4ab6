"""Writes tests/golden/c2_bench_oracle.json: the FP64 oracle's detections
(O1-O11: Sec. II of the paper with the readings the oracle states) of the 64
seeded 640x480 scenes of the benchmark's batch (config 2: 4 levels, 1 degree
at the top, the scenes' own model), with a hash of each scene so that a
change of the generator is detected instead of compared against.

Calls only the oracle and the seeded input generator:
    python tests/golden/make_oracle_detections.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "c2_bench_oracle.json")


def scene_hash(sc):
    h = hashlib.sha256()
    h.update(sc.image.tobytes())
    h.update(sc.model.tobytes())
    return h.hexdigest()[:16]


def main(n=64):
    cfg = synth.CONFIGS[2]
    L = cfg["levels"]
    sp = O.SearchParams(theta_step_top=cfg["theta_step_top"])
    model = None
    out = {"config": "C2 640x480, 4 levels, 1 deg top step, tau_m 30, tau_s 80; detections at level 0 as "
                     "[x, y, k, theta_deg, S_w, S_1]",
           "images": []}
    t0 = time.time()
    for i in range(n):
        sc = synth.scene_for_config(2, i)
        if model is None:
            model = O.build_model(sc.model, O.PyrParams(L, cfg["tau_m"]))
        tr = O.detect(sc.image, sc.model, O.PyrParams(L, cfg["tau_s"]), O.PyrParams(L, cfg["tau_m"]), sp, model=model)
        out["images"].append({"index": i, "scene": scene_hash(sc),
                              "detections": [[d.x, d.y, d.k, d.theta, d.sw, d.s1] for d in tr.detections]})
        print(f"image {i}: {len(tr.detections)} detections ({time.time() - t0:.1f} s)", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
