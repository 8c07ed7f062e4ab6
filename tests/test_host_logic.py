"""Host-side logic, on the CPU: the binding's structures against the C
header's layout (compiled with gcc), the pose record dtypes, the benchmark's
counter arithmetic, and the determinism of the seeded workloads."""
import csv
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of `fields` in `struct`, from a gcc build of tm.h."""
    src = tmp_path / f"{struct}.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tm.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / struct
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("cls,struct", [("PyrParamsC", "tm_pyr_params"), ("SearchParamsC", "tm_search_params")])
def test_binding_structs_match_the_header(tmp_path, cls, struct):
    from paper_2112_05576_amd import tm

    c = getattr(tm, cls)
    names = [f[0] for f in c._fields_]
    size, offs = _c_layout(tmp_path, struct, names)
    assert ctypes.sizeof(c) == size
    assert [getattr(c, n).offset for n in names] == offs


@pytest.mark.parametrize("dtype,struct,fields", [
    ("POSE_DTYPE", "tm_pose", ["x", "y", "k", "level", "theta_deg", "score_w", "score_1", "j"]),
    ("EVAL_DTYPE", "tm_eval_pose", ["x", "y", "theta_deg"]),
])
def test_pose_dtypes_match_the_header(tmp_path, dtype, struct, fields):
    from paper_2112_05576_amd import tm

    dt = getattr(tm, dtype)
    size, offs = _c_layout(tmp_path, struct, fields)
    assert dt.itemsize == size
    assert [dt.fields[n][1] for n in dt.names] == offs


def test_search_params_pack_every_field():
    from paper_2112_05576_amd import tm

    sp = tm.SearchParams(step_x=2, step_y=3, theta_min=-5.0, theta_range=90.0, theta_step_top=2.5,
                         neighbourhood=5, min_score=0.25, nms_min_dist=7.0, max_candidates=17, max_matches=4,
                         scale_min=0.9, scale_step=0.05, scale_count=5, vote=1)
    c = sp.c()
    assert (c.step_x, c.step_y, c.theta_min_deg, c.theta_range_deg, c.theta_step_top_deg) == (2, 3, -5.0, 90.0, 2.5)
    assert (c.neighbourhood, c.max_candidates, c.max_matches, c.scale_count, c.vote) == (5, 17, 4, 5, 1)
    assert abs(c.min_score - 0.25) == 0 and abs(c.nms_min_dist - 7.0) == 0
    assert (c.scale_min, c.scale_step) == (0.9, 0.05)
    assert abs(sp.scale(4) - 1.1) < 1e-12


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size",
                               "Workgroup_Size"])
        w.writeheader()
        for i, (name, value, grid, wg) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value,
                        "Grid_Size": grid, "Workgroup_Size": wg})


def test_traffic_figures_from_counter_runs(tmp_path, monkeypatch):
    """Per schedule of the FP16 batched search (variant, waves per chunk,
    workgroups per launch): the median dispatch, scaled by what the counter
    read for the 256 MiB copy; FP32 dispatches (single images, the other
    leg) are left out; the figure is reported only for the recorded source
    and the schedule in use."""
    sys.path.insert(0, ROOT)
    import bench

    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "traffic.json"))
    k = ("void tmk::(anonymous namespace)::k_dense_fast<32, 8, 64, {}, {}, 0, true>"
         "(tmk::(anonymous namespace)::FastArgs)")
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>(int)"
    fetch = [(k.format(0, 3), 99.0, 900 * 256, 256),           # FP32: not the batched FP16 search
             (k.format(1, 4), 1000.0, 1280 * 256, 256), (k.format(1, 4), 1002.0, 1280 * 256, 256),
             (k.format(1, 4), 90000.0, 1280 * 256, 256),       # a cold first launch: the median ignores it
             (k.format(1, 4), 700.0, 1920 * 256, 256),         # another chunking: its own figure
             (k.format(1, 2), 1500.0, 1280 * 512, 512),
             (copy, 131072.0, 1 << 26, 256)]
    write = [(n, v / 2, g, wg) for n, v, g, wg in fetch[:-1]] + [(copy, 262144.0, 1 << 26, 256)]
    _write_counters(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write_counters(tmp_path / "w.csv", "WRITE_SIZE", write)
    bench.traffic_from(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    forms = {(f["variant"], f["waves_per_chunk"], f["workgroups"]): f for f in
             __import__("json").load(open(tmp_path / "traffic.json"))["forms"]}
    assert set(forms) == {(4, 4, 1280), (4, 4, 1920), (2, 8, 1280)}
    f44 = forms[(4, 4, 1280)]
    assert f44["fetch_bytes"] == 1002.0 * 2048.0 and f44["write_bytes"] == 1002.0 / 2 * 1024.0
    assert f44["launches"] == 3
    assert forms[(4, 4, 1920)]["fetch_bytes"] == 700.0 * 2048.0
    form = {"variant": 4, "waves_per_chunk": 4, "workgroups": 1280}
    assert bench.traffic_entry(form) == f44["bytes_per_launch"]
    assert bench.traffic_entry(dict(form, workgroups=640)) is None
    assert bench.traffic_entry(dict(form, waves_per_chunk=16)) is None
    monkeypatch.setattr(bench, "KERNEL_SRC", str(tmp_path / "f.csv"))  # another source: no figure
    assert bench.traffic_entry(form) is None


def test_trace_summary_groups_by_launch_shape(tmp_path, capsys):
    """One row per kernel and launch shape, with the median over its
    dispatches; rows ordered by total time."""
    sys.path.insert(0, ROOT)
    import bench

    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X", "Workgroup_Size_Y",
            "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    k = "void tmk::(anonymous namespace)::k_dense_fast<32, 8, 64, 1, 4, 0>(tmk::(anonymous namespace)::FastArgs)"
    rows = [(k, 0, 3000, 256, 1, 1, 1280 * 256, 1, 1), (k, 5000, 9000, 256, 1, 1, 1280 * 256, 1, 1),
            (k, 10000, 13200, 256, 1, 1, 1280 * 256, 1, 1),
            (k, 20000, 20070, 256, 1, 1, 900 * 256, 1, 1),          # another shape: its own row
            ("k_select(SelectArgs)", 30000, 30016, 1024, 1, 1, 1024, 1, 1)]
    with open(tmp_path / "t.csv", "w") as f:
        f.write(",".join(cols) + "\n")
        for r in rows:
            f.write(",".join(f'"{v}"' if isinstance(v, str) else str(v) for v in r) + "\n")
    bench.trace_summary(str(tmp_path / "t.csv"))
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("| `")]
    assert len(lines) == 3
    cells = [[c.strip() for c in ln.strip("|").split("|")] for ln in lines]
    assert cells[0][:4] == ["`void k_dense_fast<32, 8, 64, 1, 4, 0>`", "1280 x 256", "3", "3.20"]
    assert cells[0][4:6] == ["3.00", "4.00"]
    assert cells[1][:4] == ["`void k_dense_fast<32, 8, 64, 1, 4, 0>`", "900 x 256", "1", "0.07"]
    assert cells[2][:4] == ["`k_select`", "1 x 1024", "1", "0.02"]


def test_workloads_are_seeded():
    import synth

    a = synth.scene_for_config(2, 5)
    b = synth.scene_for_config(2, 5)
    c = synth.scene_for_config(2, 6)
    assert a.image.dtype == np.uint8 and a.image.shape == (480, 640)
    assert np.array_equal(a.image, b.image) and np.array_equal(a.model, b.model)
    assert not np.array_equal(a.image, c.image)
    assert [(i.x, i.y, i.theta) for i in a.instances] == [(i.x, i.y, i.theta) for i in b.instances]
    assert len(a.instances) == 3


def test_bench_refuses_more_than_one_gpu():
    """The measured path is one GPU's share: --gpus N > 1 exits with a message
    before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_integer_distance_test_equals_the_fp64_one():
    """The suppression test d2 * 4^level < dmin^2 (FP64, as the oracle takes
    it) and d2 * 4^level < ceil(dmin^2) (integers, as the GPU takes it) agree
    for integer squared distances and FP32 distances, at the boundaries too."""
    rng = np.random.default_rng(3)
    dmin = np.concatenate([rng.uniform(0, 200, 20000).astype(np.float32),
                           np.float32([0.0, 1.0, 2.5, 3.0, 7.0710678, 31.999998, 32.0, 1e6])])
    dmin2 = dmin.astype(np.float64) ** 2
    lim = np.ceil(dmin2).astype(np.int64)
    for level in (0, 1, 3, 5):
        # the 32-bit form for coordinates below 2^15: the unscaled distance
        # against ceil(lim / 4^level), capped at 2^32 - 1
        s = 2 * level
        lim32 = np.minimum((lim >> s) + ((lim & ((1 << s) - 1)) != 0), 0xFFFFFFFF)
        for dx in range(-20, 21):
            for dy in (0, 1, 7, 19):
                d2 = (dx * dx + dy * dy) << (2 * level)
                assert np.array_equal(float(d2) < dmin2, d2 < lim), (level, dx, dy)
                assert np.array_equal(d2 < lim, (dx * dx + dy * dy) < lim32), (level, dx, dy)
    # exact squares land on the boundary: not too close in either form
    d = np.float32(5.0)
    assert not (25.0 < float(d) ** 2) and not (25 < int(np.ceil(float(d) ** 2)))


def test_unit_direction_rounds_as_fp64_sqrt_and_division():
    """The edge field's (gx, gy)/|g| in FP32: over the Sobel range |gx|, |gy| <=
    1020 every quotient lies at least 2^-44 (relative) from the midpoint of
    two FP32 neighbours, and two Newton steps in FP64 from an FP32 estimate
    of 1/|g| (even one 2^-15 off; the hardware's is within 2^-22) reach 2^-50,
    so the products round as FP64 square root and division do, for every
    pair."""
    g = np.arange(-1020, 1021, dtype=np.int64)
    gx, gy = (a.ravel() for a in np.meshgrid(g, g, indexing="ij"))
    m2 = gx * gx + gy * gy
    gx, gy, m2 = gx[m2 > 0], gy[m2 > 0], m2[m2 > 0]
    md = m2.astype(np.float64)
    m = np.sqrt(md)
    ref_x, ref_y = (gx / m).astype(np.float32), (gy / m).astype(np.float32)
    # distance of each positive quotient to the nearest FP32 midpoint (the
    # FP64 quotient is within 2^-52 of the exact one)
    q = (gx / m)[gx > 0]
    f = q.astype(np.float32)
    lo = np.where(f.astype(np.float64) <= q, f, np.nextafter(f, np.float32(-1)))
    mid = (lo.astype(np.float64) + np.nextafter(lo, np.float32(2)).astype(np.float64)) / 2
    assert np.min(np.abs(q - mid) / q) > 2.0 ** -44
    exact = 1.0 / m
    for rel in (2.0 ** -22, -(2.0 ** -22), 2.0 ** -15):
        r = (exact * (1 + rel)).astype(np.float32).astype(np.float64)
        for _ in range(2):
            r = (0.5 * r) * (1.0 - (md * r) * r) + r
        assert np.max(np.abs(r - exact) / exact) < 2.0 ** -50
        assert np.array_equal((gx * r).astype(np.float32), ref_x)
        assert np.array_equal((gy * r).astype(np.float32), ref_y)


def test_valu_counts_per_form(tmp_path, monkeypatch):
    """The search kernel's executed VALU instructions per launch come from a
    SQ_INSTS_VALU counter run: the median over the launches of each schedule
    (variant, waves, workgroups per launch, precision, screen); reported
    only for the recorded source and the schedule and precision in use (an
    FP16 detection runs the screen form)."""
    sys.path.insert(0, ROOT)
    import bench

    monkeypatch.setattr(bench, "VALU_JSON", str(tmp_path / "valu.json"))
    k = ("void tmk::(anonymous namespace)::k_dense_fast<32, 8, 64, {}, {}, 0, {}>"
         "(tmk::(anonymous namespace)::FastArgs)")
    rows = [(k.format(0, 3, "false"), 5.0, 900 * 256, 256),        # a single image: its own schedule
            (k.format(1, 4, "true"), 1.5e9, 1920 * 256, 256), (k.format(1, 4, "true"), 1.6e9, 1920 * 256, 256),
            (k.format(1, 4, "true"), 1.4e9, 1920 * 256, 256),
            (k.format(0, 4, "false"), 2.0e9, 1920 * 512, 512)]
    _write_counters(tmp_path / "v.csv", "SQ_INSTS_VALU", rows)
    bench.valu_from(str(tmp_path / "v.csv"))
    forms = __import__("json").load(open(tmp_path / "valu.json"))["forms"]
    by = {(f["variant"], f["waves_per_chunk"], f["workgroups"], f["precision"], f["screen"]): f for f in forms}
    assert set(by) == {(3, 4, 900, "fp32", False), (4, 4, 1920, "fp16", True), (4, 8, 1920, "fp32", False)}
    assert by[(4, 4, 1920, "fp16", True)]["valu_instr_per_launch"] == 1.5e9
    f16 = {"variant": 4, "waves_per_chunk": 4, "workgroups": 1920}
    assert bench.valu_entry(f16, "fp16")["valu_instr_per_launch"] == 1.5e9
    assert bench.valu_entry({"variant": 4, "waves_per_chunk": 8, "workgroups": 1920}, "fp32")[
        "valu_instr_per_launch"] == 2.0e9
    assert bench.valu_entry({"variant": 4, "waves_per_chunk": 8, "workgroups": 1920}, "fp16") is None
    assert bench.valu_entry(dict(f16, workgroups=1280), "fp16") is None
    monkeypatch.setattr(bench, "KERNEL_SRC", str(tmp_path / "v.csv"))  # another source: no figure
    assert bench.valu_entry(f16, "fp16") is None


def test_loop_mix_from_assembly(tmp_path, monkeypatch):
    """The search loop of each k_dense_fast instantiation is its innermost
    loop with the most DPP window maxima; its VALU instructions are costed 4
    issue cycles (dot2, DPP, 3-operand max) or 2 (the rest)."""
    sys.path.insert(0, ROOT)
    import bench

    monkeypatch.setattr(bench, "LOOP_MIX_JSON", str(tmp_path / "mix.json"))
    asm = "\n".join([
        "_ZN3tmk12_GLOBAL__N_112k_dense_fastILi32ELi8ELi64ELi1ELi4ELi0ELb1EEEvNS0_8FastArgsEPKNS_8PairDescE:",
        "\ts_load_dwordx2 s[0:1], s[4:5], 0x0",
        ".LBB0_1:",                                       # the epilogue-like loop: products, no DPP
        "\tv_fma_f32 v1, v2, v3, v4",
        "\tv_fma_f32 v1, v2, v3, v4",
        "\tv_fma_f32 v1, v2, v3, v4",
        "\ts_cbranch_scc0 .LBB0_1",
        ".LBB0_2:",                                       # the search loop
        "\tds_read2st64_b32 v[0:1], v5 offset1:1",
        "\tv_dot2_f32_f16 v6, s0, v0, 0",
        "\tv_max_f32_dpp v7, v6, v6 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1",
        "\tv_max3_f32 v8, v7, v6, v9",
        "\tv_add_f32_e32 v10, v10, v8",
        "\ts_cbranch_scc0 .LBB0_2",
        "\ts_endpgm",
    ])
    (tmp_path / "k.s").write_text(asm + "\n")
    bench.loop_mix_from(str(tmp_path / "k.s"))
    f = __import__("json").load(open(tmp_path / "mix.json"))["forms"]
    assert len(f) == 1 and (f[0]["precision"], f[0]["variant"], f[0]["screen"]) == ("fp16", 4, True)
    assert f[0]["loop_valu"] == 4 and f[0]["loop_issue_cycles"] == 4 + 4 + 4 + 2
    assert bench.loop_mix_entry({"variant": 4}, "fp16")["cycles_per_instr"] == 14 / 4
    assert bench.loop_mix_entry({"variant": 3}, "fp16") is None
