"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic
byte model of each step kernel, the rooflines of the dominant kernel and of
the whole step, and the rule that measured traffic is reported only for the
kernel sources it was taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def headline():
    from workloads import workload
    return workload("sg_gap_m8_q12_n3e7", precision="fp64")


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_kernel_bytes_of_the_headline_workload():
    cfg = headline()
    N, P, Q, nk = cfg["n_particles"], 9, 12, cfg["nk"]
    assert (N, nk) == (30_000_000, 256)
    cand = 350_000
    b = bench.kernel_bytes(cfg, P, Q, n_drift=1, cand=cand)
    # every coefficient read once; the drifted mode written for the non-candidates
    assert b["stream"] == 2 * P * 8 * N + (N - cand) * 1 * 8
    # H^n written and the overflow grid cleared
    assert b["finalize"] == 2 * Q * nk * nk * 4
    # the candidates' coefficients read and written
    assert b["collide"] == cand * 4 * P * 8
    b32 = bench.kernel_bytes(dict(cfg, precision="fp32"), P, Q, n_drift=1, cand=cand)
    assert b32["stream"] * 2 == b["stream"] and b32["collide"] * 2 == b["collide"]


def _run(kernels, wall=2.0, steps=1000):
    return {"n_drift": 1, "cand": (350_000.0,), "kernels": kernels, "wall": wall, "steps": steps,
            "symbols": {"stream": "sgpm::k1_pairs", "finalize": "sgpm::k3_finalize",
                        "collide": "sgpm::k2_lanes"}}


def test_roofline_is_the_longest_kernel():
    cfg = headline()
    r = _run({"stream": (1.50, 1000), "finalize": (0.05, 1000), "collide": (1.00, 1000)})
    roof, per, step = bench.roofline_of(cfg, r, 9, 12)
    assert roof["kernel"] == "sgpm::k1_pairs"
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    want = per["stream"]["bytes_per_launch"] / 1.5e-3 / 1e9
    assert roof["achieved"] == pytest.approx(want)
    assert roof["frac"] == pytest.approx(want / 8000.0)
    # no margin in favour of any kernel: a collider 1 % longer takes the roofline
    r["kernels"]["collide"] = (1.515, 1000)
    roof, _, _ = bench.roofline_of(cfg, r, 9, 12)
    assert roof["kernel"] == "sgpm::k2_lanes"


def test_roofline_of_the_whole_step():
    """The step's algorithmic bytes (the three launches) over the wall time
    per step."""
    cfg = headline()
    r = _run({"stream": (1.50, 1000), "finalize": (0.05, 1000), "collide": (1.00, 1000)},
             wall=2.4, steps=1000)
    _, per, step = bench.roofline_of(cfg, r, 9, 12)
    total = sum(v["bytes_per_launch"] for v in per.values())
    assert step["bytes_per_step"] == total
    assert step["ms_per_step"] == pytest.approx(2.4)
    assert step["achieved"] == pytest.approx(total / 2.4e-3 / 1e9)
    assert step["frac"] == pytest.approx(step["achieved"] / 8000.0)


def test_matched_error_is_per_observable():
    import numpy as np
    t = 5
    ref = {o: np.linspace(1.0, 2.0, t) for o in bench.OBSERVABLES}
    ref.update({"SE_" + o: np.full(t, 0.1) for o in bench.OBSERVABLES})
    other = {o: ref[o].copy() for o in bench.OBSERVABLES}
    other["E_vx"][3] += 0.25          # 2.5 SE at one time
    other["Var_vx"][0] += 9.0         # time 0 (the shared initial datum) is not compared
    dev = bench.max_dev_over_se(ref, other)
    assert dev["E_vx"] == pytest.approx(2.5) and dev["Var_vx"] == 0.0


def test_traffic_only_for_the_profiled_sources(monkeypatch, tmp_path):
    rec = {"source_sha256": "the profiled sources", "calibration": {"fetch_factor": 2.0,
                                                                      "write_factor": 1.0},
           "kernels": {"stream": {"fetch_bytes": 4.3e9, "write_bytes": 0.4e9}}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "not the profiled sources")
    assert bench.measured_traffic("stream") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["source_sha256"])
    k = rec["kernels"]["stream"]
    assert bench.measured_traffic("stream") == k["fetch_bytes"] + k["write_bytes"]
    # the calibration factors of a plain copy are recorded beside the figures
    assert rec["calibration"]["fetch_factor"] > 0 and rec["calibration"]["write_factor"] > 0


def test_entry_points_exist():
    import __graft_entry__ as e
    assert callable(e.build) and callable(e.smoke)


def test_pmc_summary_scales_by_the_copy(tmp_path):
    """Synthetic counter files: the copy reads half its bytes on FETCH_SIZE and
    all of them on WRITE_SIZE; the kernels' medians are scaled accordingly."""
    head = "Kernel_Name,Counter_Name,Counter_Value\n"
    copy_kib = 268435456 / 1024
    fetch = [("__amd_rocclr_copyBuffer", copy_kib / 2)] * 5 + [
        ("void sgpm::k1_stream<double, 9, 12>(x)", v) for v in (1000.0, 1100.0, 900.0)] + [
        ("sgpm::k3_finalize(x)", 50.0), ("void sgpm::k2_collide_wide<double, 9, 1>(x)", 20.0),
        ("void sgpm::k1_stream<float, 9, 12>(x)", 1e9)]   # another precision: ignored
    write = [("__amd_rocclr_copyBuffer", copy_kib)] * 5 + [
        ("void sgpm::k1_stream<double, 9, 12>(x)", 300.0), ("sgpm::k3_finalize(x)", 4.0),
        ("void sgpm::k2_collide_wide<double, 9, 1>(x)", 6.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    fp.write_text(head + "".join(f'"{k}",FETCH_SIZE,{v}\n' for k, v in fetch))
    wp.write_text(head + "".join(f'"{k}",WRITE_SIZE,{v}\n' for k, v in write))
    out = bench.pmc_summary(str(fp), str(wp), str(tmp_path / "t.json"))
    assert out["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert out["calibration"]["write_factor"] == pytest.approx(1.0)
    k1 = out["kernels"]["stream"]
    assert k1["dispatches"] == 3
    assert k1["fetch_bytes"] == pytest.approx(1000.0 * 1024 * 2.0)
    assert k1["write_bytes"] == pytest.approx(300.0 * 1024)
    assert out["source_sha256"] == bench.kernel_source_hash()
    assert json.loads((tmp_path / "t.json").read_text()) == out


def test_pmc_summary_keeps_the_timed_passes(tmp_path):
    """With dispatch ids, only the last 2 * steps moving steps count: a stream
    launch followed by the collider before the next stream launch.  Earlier
    launches (another launch shape, as in the autotuner's trials) and bins-only
    passes (no collider) are left out, and the stream workgroups are recorded."""
    head = ("Dispatch_Id,Grid_Size,Workgroup_Size,Kernel_Name,Counter_Name,Counter_Value\n")
    copy_kib = 268435456 / 1024
    k1, k3, k2 = ("void sgpm::k1_stream<double, 9, 12>(x)", "sgpm::k3_finalize(x)",
                  "void sgpm::k2_collide_wide<double, 9, 1>(x)")

    def runs(counter, copy_val):
        rows, d = [], 0
        for _ in range(3):
            d += 1; rows.append((d, 1024, 1024, "__amd_rocclr_copyBuffer", copy_val))
        # a trial shape: 490 workgroups, large values
        for _ in range(4):
            d += 1; rows.append((d, 490 * 1024, 1024, k1, 9000.0))
            d += 1; rows.append((d, 256, 256, k3, 900.0))
            d += 1; rows.append((d, 256, 256, k2, 90.0))
        # a bins-only pass (no collider), then the final shape: 245 workgroups
        d += 1; rows.append((d, 245 * 1024, 1024, k1, 5.0))
        d += 1; rows.append((d, 256, 256, k3, 5.0))
        for s in range(6):
            d += 1; rows.append((d, 245 * 1024, 1024, k1, 100.0 + s))
            d += 1; rows.append((d, 256, 256, k3, 10.0))
            d += 1; rows.append((d, 256, 256, k2, 1.0))
        return head + "".join(f'{a},{g},{wg},"{k}",{counter},{v}\n' for a, g, wg, k, v in rows)

    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    fp.write_text(runs("FETCH_SIZE", copy_kib / 2))
    wp.write_text(runs("WRITE_SIZE", copy_kib))
    out = bench.pmc_summary(str(fp), str(wp), str(tmp_path / "t.json"), steps=2)
    k = out["kernels"]
    assert k["stream"]["dispatches"] == 4          # the last 2 * steps moving steps
    assert k["stream"]["fetch_bytes"] == pytest.approx(103.5 * 1024 * 2.0)   # median of 102..105
    assert k["finalize"]["write_bytes"] == pytest.approx(10.0 * 1024)
    assert k["collide"]["write_bytes"] == pytest.approx(1.0 * 1024)
    assert out["stream_workgroups"] == 245


def test_traffic_only_for_the_same_launch_shape(monkeypatch, tmp_path):
    rec = {"source_sha256": "h", "stream_workgroups": 245,
           "kernels": {"stream": {"fetch_bytes": 1.0, "write_bytes": 2.0},
                       "collide": {"fetch_bytes": 4.0, "write_bytes": 5.0}}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h")
    assert bench.measured_traffic("stream", 245) == 3.0
    assert bench.measured_traffic("stream", 490) is None
    assert bench.measured_traffic("stream") == 3.0
    # the collider's traffic depends on the step window's candidate count
    assert bench.measured_traffic("collide", 245) is None


def test_pmc_summary_sums_the_collider_launches_of_a_step(tmp_path):
    """The lane collider runs as a main and a leftover launch per step: the
    collide row of a step is the sum of both."""
    head = ("Dispatch_Id,Grid_Size,Workgroup_Size,Kernel_Name,Counter_Name,Counter_Value\n")
    copy_kib = 268435456 / 1024
    k1, k3 = "void sgpm::k1_pairs<double, 9, 12, 0>(x)", "sgpm::k3_finalize(x)"
    k2a, k2b = "void sgpm::k2_lanes<double, 9, false>(x)", "void sgpm::k2_lanes<double, 9, true>(x)"

    def runs(counter, copy_val):
        rows, d = [], 0
        for _ in range(3):
            d += 1; rows.append((d, 1024, 1024, "__amd_rocclr_copyBuffer", copy_val))
        for s in range(4):
            d += 1; rows.append((d, 255 * 512, 512, k1, 100.0))
            d += 1; rows.append((d, 256, 256, k3, 10.0))
            d += 1; rows.append((d, 256, 256, k2a, 7.0))
            d += 1; rows.append((d, 256, 256, k2b, 2.0))
        return head + "".join(f'{a},{g},{wg},"{k}",{counter},{v}\n' for a, g, wg, k, v in rows)

    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    fp.write_text(runs("FETCH_SIZE", copy_kib / 2))
    wp.write_text(runs("WRITE_SIZE", copy_kib))
    out = bench.pmc_summary(str(fp), str(wp), str(tmp_path / "t.json"), steps=2)
    k = out["kernels"]
    assert k["collide"]["dispatches"] == 4
    assert k["collide"]["write_bytes"] == pytest.approx(9.0 * 1024)
    assert k["stream"]["write_bytes"] == pytest.approx(100.0 * 1024)
    assert out["stream_workgroups"] == 255
