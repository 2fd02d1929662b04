"""Benchmark of the sG-PM hot path on one MI355X.

Headline workload: sg_gap_m8_q12_n3e7 -- the largest single-GPU workload:
3e7 particles, uncertain band gap Delta(z) = 0.25 eV (1 + 0.2 z), Legendre
order M = 8 (9 modes), 12 Gauss nodes, E = 40 kV/cm, dt = 2 fs, FP64
particle state (the plain form), the paper's rates and the Pauli acceptance
on a 256 x 256 grid rebuilt every step.  A step is one pass of the whole hot
path (drift, node evaluation, histogram, moments, collision decision, nodal
collisions, projection) over every particle, launched the library's default
way (captured HIP graphs of 16 steps).

The same K steps are then run once more with a HIP event after every kernel
launch (on the library's stream) to time each kernel.  ``roofline`` is that
of the longest kernel, from its algorithmic bytes per launch;
``roofline_step`` is the whole step's, from the algorithmic bytes of one
step over the wall time per step.  Beside the headline: the same workload
with FP32 particle state (compared per observable against the Monte Carlo
standard error), the 8-node workload (1e6 particles) in FP64, and the
64-instance sweep in FP32 batched (one launch per kernel and step), in FP64
batched and in FP64 plain (each instance alone), compared per instance and
observable.  The CPU baseline is the plain FP64 oracle on a bounded sample of
the headline workload, on the host cores.

Prints one JSON line.  Throughput is particle-node updates per second with
the state resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "sg_gap_m8_q12_n3e7"
SECONDARY = "sg_gap_m5_q8_n1e6"
# kernel-name patterns of the headline's FP64 launches in a profiler's output
# (the stream kernel in its generic or mirror-pair form, the collider with a
# group of lanes or a lane per candidate)
HEADLINE_KERNELS = {"stream": r"k1_(stream|pairs)<double", "finalize": r"k3_finalize",
                    "collide": r"k2_(collide|collide_wide|lanes)<double"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_sg_gap_m8_q12_n3e7.json")
OBSERVABLES = ("E_vx", "Var_vx", "E_jx", "Var_jx", "E_energy")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sgpm_kernels.hip", "sgpm_internal.h"):
        with open(os.path.join(ROOT, "paper_2404_19602_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_symbols(sim, inst: int = 0) -> dict:
    """The kernel each step role of instance inst is launched as (template
    arguments left out: precision, mode and node buckets)."""
    return {"stream": "sgpm::k1_pairs" if sim.node_pairs(inst) else "sgpm::k1_stream",
            "finalize": "sgpm::k3_finalize",
            "collide": "sgpm::k2_lanes" if sim.collider_lanes(inst) else "sgpm::k2_collide"}


def kernel_bytes(cfg: dict, P: int, Q: int, n_drift: int, cand: float) -> dict:
    """Algorithmic HBM bytes of one launch of each step kernel.

    stream: read every coefficient (2 P s per particle) and write back the
      drifted modes of the particles that cannot collide (n_drift s each);
    finalize: write H^n (Q nk^2 uint32) and clear the overflow counts of the
      next one (the same size);
    collide: read and write all 2 P coefficients of every candidate."""
    s = 4 if cfg.get("precision") == "fp32" else 8
    N = cfg["n_particles"]
    grid = Q * cfg.get("nk", 240) ** 2 * 4
    return {"stream": 2 * P * s * N + (N - cand) * n_drift * s,
            "finalize": 2 * grid,
            "collide": cand * 4 * P * s}


def run_gpu(cfgs, steps: int, warmup: int, profile: bool = True, tune: bool = True):
    """Warm-up, the autotuned launch shape (trials from the warmed-up state,
    which is put back), K timed steps in
    the default launch mode, then the same K steps once more from the same
    state and step (the random streams are keyed by the step, so the run is
    replayed exactly) with a HIP event around every kernel: the per-kernel
    means describe the timed steps.  cfgs: one workload or a list (batched
    instances)."""
    import numpy as np
    import torch
    import paper_2404_19602_amd as sg

    many = isinstance(cfgs, list)
    sim = sg.Simulation(cfgs, max_steps=warmup + 2 * steps)
    sim.init_particles()
    dt = (cfgs[0] if many else cfgs)["dt"]
    if warmup:
        sim.step(warmup, dt)
    tuned_ms = sim.autotune(trial_steps=10, dt=dt) if tune else None
    shape = sim.launch_shape(0)
    s0 = sim.step_count
    saved = [sim.get_state(j) for j in range(sim.n_inst)] if profile else None
    c0 = [sim.counters(j) for j in range(sim.n_inst)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = sim.last_step_ms()
    c1 = [sim.counters(j) for j in range(sim.n_inst)]
    out = dict(sim=sim, wall=wall, steps=steps, dev_ms=dev_ms, shape=shape, tuned_ms=tuned_ms,
               cand=[(b["candidates"] - a["candidates"]) / steps for a, b in zip(c0, c1)])
    # the record of the timed steps: their last steps + 1 recorded times (the
    # autotuner may have restarted the record at the tuned time)
    out["moments_all"] = [sim.moments(sim.record_length(j) - steps - 1, steps + 1, inst=j)
                          for j in range(sim.n_inst)]
    if not many:
        out["moments"] = out["moments_all"][0]
        t = sim.tables()
        out["n_drift"] = int(np.count_nonzero(t["ehat"]))
    if profile:
        for j, (kx, ky) in enumerate(saved):
            sim.set_state(kx, ky, step=s0, inst=j)
        sim.set_profiling(True)
        sim.step(steps, dt)
        out["kernels"] = sim.kernel_times()
        sim.set_profiling(False)
    out["symbols"] = kernel_symbols(sim)
    return out


def roofline_of(cfg, r, P, Q) -> tuple:
    """Per-kernel achieved GB/s, the roofline object of the dominant kernel (the
    one with the largest mean launch time) and that of the whole step (the
    algorithmic bytes of the three launches of a step over the wall time per
    graph-replayed step)."""
    b = kernel_bytes(cfg, P, Q, r["n_drift"], r["cand"][0])
    per = {}
    for k, (ms, n) in r["kernels"].items():
        per[k] = {"avg_ms": ms, "launches": n, "bytes_per_launch": b[k],
                  "GBps": b[k] / (ms * 1e-3) / 1e9 if ms > 0 else None}
    dom = max(per, key=lambda k: per[k]["avg_ms"])
    ach = per[dom]["GBps"]
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": r["symbols"][dom],
            "kernel_ms": per[dom]["avg_ms"], "bytes_per_launch": per[dom]["bytes_per_launch"],
            "timing": "HIP events around each launch on the library's stream, "
                      "in a replay of the timed steps from the same state"}
    shape = r.get("shape") or {}
    traffic = measured_traffic(dom, shape.get("stream_workgroups"))
    if traffic is not None:
        roof["traffic"] = traffic
    step_bytes = sum(b.values())
    step_ms = r["wall"] * 1e3 / r["steps"]
    step = {"bound": "hbm", "achieved": step_bytes / (step_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "bytes_per_step": step_bytes, "ms_per_step": step_ms}
    step["frac"] = step["achieved"] / HBM_PEAK_GBS
    return roof, per, step


def measured_traffic(kernel: str, stream_workgroups=None):
    """HBM bytes per launch of a kernel from the committed PMC summary, if the
    kernel source is the one the counters were taken on and, when both are
    known, the launch shape (stream workgroups) is the same: the window slabs
    the stream kernel writes and the finalize kernel reads scale with it.  The
    collider's traffic scales with the candidate count, which grows through a
    run: the counters, taken over the first 40 steps, do not hold for another
    window, so none is reported for it."""
    if kernel == "collide" or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    taken = rec.get("stream_workgroups")
    if taken is not None and stream_workgroups is not None and taken != stream_workgroups:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def uq_timings(cfg: dict, steps: int = 100, n: int = 50_000, samples: int = 256) -> dict:
    """Sec. 5 Test 4 shapes: Monte Carlo sampling of z with `samples`
    deterministic runs of n particles (one batched launch per kernel and step)
    against the sG-PM of the headline workload at the same n, and the rate of
    the evaluation of the particle expansion at points z."""
    import numpy as np
    import torch
    import paper_2404_19602_amd as sg
    from paper_2404_19602_amd import uq

    log(f"uq: MC-MC with {samples} samples x {n} particles vs MC-sG, {steps} steps")
    z = uq.sample_z(samples, 1, 7)
    cfgs = uq.deterministic_at(cfg, z)
    for k, c in enumerate(cfgs):
        c.update(instance=k, n_particles=n)
    res = {}
    for name, cf in (("mc_mc", cfgs), ("mc_sg", dict(cfg, n_particles=n))):
        sim = sg.Simulation(cf, max_steps=steps + 30)
        sim.init_particles()
        sim.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.set_profiling(True)
        sim.step(20)
        kt = sim.kernel_times()
        sim.set_profiling(False)
        res[name] = {"ms_per_step": wall * 1e3 / steps, "instances": sim.n_inst,
                     "kernels_us": {k: round(v[0] * 1e3, 2) for k, v in kt.items()}}
        if name == "mc_sg":
            zz = np.linspace(-1, 1, 256)
            sim.moments_at(zz[:8])
            t0 = time.perf_counter()
            sim.moments_at(zz)
            res["moments_at_256_points_ms"] = (time.perf_counter() - t0) * 1e3
        del sim
    res["cost_ratio_mc_mc_over_mc_sg"] = res["mc_mc"]["ms_per_step"] / res["mc_sg"]["ms_per_step"]
    res["error_versus_cost"] = test4_error_versus_cost()
    res["config"] = {"n_particles": n, "samples": samples, "steps": steps,
                     "sg_modes": cfg["degree"] + 1, "sg_nodes": cfg["nodes_1d"]}
    return res


def test4_error_versus_cost() -> dict:
    """Sec. 5 Test 4 at the paper's sizes: N = 5e4, t = 0.5 ps (200 steps of
    2.5 fs), reference of 5e6 particles at M = 30, MC-sG orders M1 and MC-MC
    sample counts M2, on the uncertain-width problem of Test 3 (W = 6.5 + z'
    nm, z' ~ U(0, 1), E = 0.5 V/um)."""
    from paper_2404_19602_amd import uq
    cfg = dict(dim_z=1, gap_mode=1, gap_dim=0, gap0=7.0, gap_rel=1.0 / 14.0, field_dim=-1,
               field0=5e5, field_rel=0.0, fermi_eV=0.4, temp_K=300.0, alpha=0.1, nk=240,
               lk_eV=5.0, pauli=1, final_state=0, rate_scale=(1.0,) * 6, seed=2404196034,
               instance=0, c_max=32, dt=2.5e-15, precision="fp64")
    log("Test 4: reference 5e6 particles M = 30, MC-sG M1 in 0..8, MC-MC M2 up to 64, N = 5e4")
    r = uq.error_versus_cost(cfg, n=50_000, steps=200, sg_orders=[0, 1, 2, 3, 4, 6, 8],
                             mc_samples=[1, 2, 4, 8, 16, 32, 64], n_ref=5_000_000, m_ref=30)
    keep = ("M1", "M2", "cost_per_particle", "error", "SE", "SE_samples", "ms_per_step")
    return {"t_ps": r["t_s"] * 1e12, "n": r["n"], "n_ref": r["n_ref"], "m_ref": r["m_ref"],
            "ref_E_vx": r["ref_E_vx"], "ref_SE": r["ref_SE"],
            "ref_ms_per_step": r["ref_ms_per_step"],
            "mc_sg": [{k: v for k, v in row.items() if k in keep} for row in r["mc_sg"]],
            "mc_mc": [{k: v for k, v in row.items() if k in keep} for row in r["mc_mc"]],
            "mc_mc_ms_per_step_64_samples": r["mc_ms_per_step_all_samples"]}


OTHER_CONFIGS = (("gnr_det_n1e4", ("fp64",)),
                 ("sg_gap_field_td4_q64_n4e6", ("fp64", "fp32")))


def other_configs(steps: int = 50) -> dict:
    """The other workloads at their full sizes, each with its autotuned launch
    shape: wall time per step of `steps` graph-replayed steps after 10 warm-up
    steps, in particle-node updates per second."""
    import torch
    import paper_2404_19602_amd as sg
    from workloads import workload

    res = {}
    for name, precs in OTHER_CONFIGS:
        res[name] = {}
        for prec in precs:
            cfg = workload(name, precision=prec)
            log(f"{name} {prec}: 10 warm-up + autotune + {steps} timed steps")
            sim = sg.Simulation(cfg, max_steps=2 * steps + 40)
            sim.init_particles()
            sim.step(10, cfg["dt"])
            sim.autotune(trial_steps=10, dt=cfg["dt"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps, cfg["dt"])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            P, Q = sim.sizes[0]
            res[name][prec] = {"ms_per_step": wall * 1e3 / steps,
                               "value": cfg["n_particles"] * Q * steps / wall,
                               "unit": "particle-node updates/s", "n_particles": cfg["n_particles"],
                               "gpc_modes": P, "nodes": Q, "chunk": sim.launch_shape(0)["chunk"]}
            if Q > 1:
                sim.set_profiling(True)
                sim.step(steps, cfg["dt"])
                kt = sim.kernel_times()
                sim.set_profiling(False)
                res[name][prec]["kernels_us"] = {k: round(v[0] * 1e3, 2) for k, v in kt.items()}
                res[name][prec]["roofline_stream_alu"] = alu_roofline(
                    cfg["n_particles"], P, Q, kt["stream"][0], prec)
            del sim
            torch.cuda.empty_cache()
    return res


FP64_VECTOR_TFLOPS = 78.6     # 256 CUs x 2.4 GHz x 64 FP64 lanes x 2 (FMA)
FP32_VECTOR_TFLOPS = 157.3    # packed FP32 (this build does not emit packed FP32: 78.6 for it)


def alu_roofline(n: int, P: int, Q: int, ms: float, prec: str) -> dict:
    """ALU roofline of the stream kernel from its algorithmic flops: per
    particle-node 4 P (the two components of the node value, P multiply-adds
    each) + 12 (energy, velocity and the three moment terms); the vector peak
    of the state precision."""
    flops = n * Q * (4 * P + 12)
    peak = FP64_VECTOR_TFLOPS if prec == "fp64" else FP32_VECTOR_TFLOPS
    ach = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
            "flops_per_launch": flops, "kernel_ms": ms}


def cpu_baseline(cfg: dict, n_s: int = 100_000, steps_s: int = 250):
    """The FP64 oracle on a bounded sample: n_s of the particles for steps_s
    steps (about ten seconds), every host thread this process may use."""
    import oracle
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))
    scfg = dict(cfg, n_particles=n_s)
    sim = oracle.OracleSim(scfg, threads=threads)
    sim.init()
    t0 = time.perf_counter()
    sim.run(cfg["dt"], steps_s)
    dt = time.perf_counter() - t0
    Q = sim.Q
    return {"value": n_s * Q * steps_s / dt, "unit": "particle-node updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{n_s} of the {cfg['n_particles']} particles, {steps_s} steps, "
                      f"same physical and gPC parameters ({dt:.1f} s of CPU work)"}


def pmc_summary(fetch_csv: str, write_csv: str, out_path: str = TRAFFIC_FILE,
                steps: int = 20) -> dict:
    """The traffic record from two rocprofv3 --pmc runs of this bench with
    --copy-calibration --headline-only (FETCH_SIZE, then WRITE_SIZE; csv
    counter collections),
    scaled by what the same counter reads for the 268435456-byte device copies,
    with the SHA-256 of the kernel sources they were taken on.

    Per step kernel, the median over the last 2 * steps moving steps of the
    headline (its timed and its profiled pass, in the final launch shape): a
    stream launch is a moving step when the collider runs before the next
    stream launch, and that step's finalize and collide launches are the ones
    that follow it.  The autotuner's trials and the bins-only passes, whose
    shapes and traffic differ, are left out.  Without dispatch ids in the files
    every headline dispatch counts."""
    import csv
    import statistics

    names = HEADLINE_KERNELS

    def load(path, counter):
        by, seq = {}, []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                by.setdefault(r["Kernel_Name"], []).append(v)
                key = next((k for k, pat in names.items() if re.search(pat, r["Kernel_Name"])),
                           None)
                if key is not None and r.get("Dispatch_Id"):
                    wgs = None
                    if r.get("Grid_Size") and r.get("Workgroup_Size"):
                        wgs = int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"]))
                    seq.append((int(r["Dispatch_Id"]), key, v, wgs))
        return by, sorted(seq)

    def moving_steps(seq):
        """(stream, finalize, collide) rows of the last 2 * steps moving steps; the
        collide row sums the step's collider launches (the lane collider's main
        and leftover passes)."""
        out = []
        for k, (_, key, _, _) in enumerate(seq):
            if key != "stream":
                continue
            fin, cols = None, []
            for row in seq[k + 1:]:
                if row[1] == "stream":
                    break
                if row[1] == "finalize" and fin is None:
                    fin = row
                if row[1] == "collide":
                    cols.append(row)
            if fin is not None and cols:
                col = (cols[0][0], "collide", sum(r[2] for r in cols), cols[0][3])
                out.append((seq[k], fin, col))
        return out[-2 * steps:]

    copy = 268435456
    (f, fseq), (w, wseq) = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")

    def factor(by):   # counters are in KiB; the copies are the large copyBuffer dispatches
        vals = [v for k, vs in by.items() if "copyBuffer" in k for v in vs if v > 100000]
        return copy / (statistics.median(vals) * 1024)

    cf, cw = factor(f), factor(w)
    fsteps, wsteps = moving_steps(fseq), moving_steps(wseq)
    out = {"workload": WORKLOAD + " (FP64 state)", "source_sha256": kernel_source_hash(),
           "calibration": {"copy_bytes": copy, "fetch_factor": cf, "write_factor": cw},
           "kernels": {}}
    if fsteps and wsteps:
        shapes = sorted({s[0][3] for s in fsteps} | {s[0][3] for s in wsteps})
        out["steps"] = {"fetch_run": len(fsteps), "write_run": len(wsteps)}
        out["stream_workgroups"] = shapes[0] if len(shapes) == 1 else None
    for j, (key, pat) in enumerate(names.items()):
        if fsteps and wsteps:
            fk = [s[j][2] for s in fsteps]
            wk = [s[j][2] for s in wsteps]
        else:
            fk = [v for k, vs in f.items() if re.search(pat, k) for v in vs]
            wk = [v for k, vs in w.items() if re.search(pat, k) for v in vs]
        out["kernels"][key] = {"dispatches": len(fk),
                               "fetch_bytes": statistics.median(fk) * 1024 * cf,
                               "write_bytes": statistics.median(wk) * 1024 * cw}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def max_dev_over_se(ref: dict, other: dict) -> dict:
    """max over the recorded times t >= 1 of |other - ref| / SE(ref), per observable"""
    import numpy as np
    out = {}
    for obs in OBSERVABLES:
        se = np.maximum(ref["SE_" + obs][1:], 1e-300)
        out[obs] = float(np.max(np.abs(ref[obs][1:] - other[obs][1:]) / se))
    return out


def sweep_forms(steps: int, warmup: int = 10) -> dict:
    """The 64-instance sweep three ways, the same steps from the same initial
    data and random streams: FP32 batched and FP64 batched (one launch of each
    kernel per step for every instance of a shape group, graph-replayed), and
    FP64 plain (each instance in a context of its own, one after another; its
    time is the sum).  Every instance's observables of the FP32-batched run
    are compared with its FP64-plain run against the Monte Carlo SE."""
    import numpy as np
    import torch
    import paper_2404_19602_amd as sg
    from workloads import batched_sweep

    cfgs = batched_sweep(steps=steps)
    pn = sum(c["n_particles"] * (c["degree"] + 3) for c in cfgs) * steps
    res = {"workload": "batched_sweep_64 (E 1-50 kV/cm, gap 0.1-0.5 eV +-10 %, M in {2,4,6}, "
                       "Q = M + 3, N log-uniform 1e5-2e6)",
           "instances": len(cfgs), "n_particles": sum(c["n_particles"] for c in cfgs),
           "steps": steps, "unit": "particle-node updates/s"}
    mom = {}
    for form, prec in (("fp32_batched", "fp32"), ("fp64_batched", "fp64")):
        log(f"sweep {form}: {len(cfgs)} instances, {warmup} warm-up + {steps} timed steps")
        r = run_gpu([dict(c, precision=prec) for c in cfgs], steps, warmup, profile=(prec == "fp32"))
        sim = r["sim"]
        mom[form] = r["moments_all"]
        res[form] = {"ms_per_step": r["wall"] * 1e3 / steps, "value": pn / r["wall"],
                     "launch_shape_inst0": r["shape"], "candidates_per_step": sum(r["cand"])}
        if "kernels" in r:
            res[form]["kernels"] = {k: {"avg_ms": ms, "launches": n}
                                    for k, (ms, n) in r["kernels"].items()}
        del r, sim
        torch.cuda.empty_cache()
    log(f"sweep fp64_plain: {len(cfgs)} contexts one after another")
    wall, plain = 0.0, []
    for c in cfgs:
        sim = sg.Simulation(dict(c, precision="fp64"), max_steps=warmup + steps)
        sim.init_particles()
        sim.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        plain.append(sim.moments(warmup, steps + 1))
        del sim
    res["fp64_plain"] = {"ms_per_step": wall * 1e3 / steps, "value": pn / wall}
    worst = {obs: 0.0 for obs in OBSERVABLES}
    worst64 = {obs: 0.0 for obs in OBSERVABLES}
    same = 0
    for j in range(len(cfgs)):
        for obs, v in max_dev_over_se(plain[j], mom["fp32_batched"][j]).items():
            worst[obs] = max(worst[obs], v)
        # FP64 batched against FP64 plain: the same arithmetic, except that a
        # shape group of 2^22 particles or more is stepped by the mirror-pair
        # stream kernel (node values summed in another order), so the two agree
        # to rounding, not always bit for bit
        for obs, v in max_dev_over_se(plain[j], mom["fp64_batched"][j]).items():
            worst64[obs] = max(worst64[obs], v)
        same += int(np.array_equal(plain[j]["E_vx"], mom["fp64_batched"][j]["E_vx"]))
    res["max_abs_dev_over_mc_se"] = worst
    res["fp64_batched_vs_plain_max_abs_dev_over_mc_se"] = worst64
    res["fp64_batched_instances_bit_identical_to_plain"] = same
    res["matched_error"] = all(v < 3.0 for v in worst.values())
    res["speedup_fp32_batched_vs_fp64_plain"] = res["fp64_plain"]["ms_per_step"] / \
        res["fp32_batched"]["ms_per_step"]
    res["speedup_fp32_batched_vs_fp64_batched"] = res["fp64_batched"]["ms_per_step"] / \
        res["fp32_batched"]["ms_per_step"]
    return res


def late_window(cfg: dict, after: int = 1000, steps: int = 100) -> dict:
    """The headline later in a run: `after` steps from the initial datum (the
    distribution heats under the field and the candidate count grows), then
    `steps` graph-replayed steps timed on the wall clock and, again from the
    same state, with a HIP event around every launch."""
    import torch
    import paper_2404_19602_amd as sg
    log(f"late window: {after} steps, then {steps} timed + {steps} profiled steps")
    sim = sg.Simulation(cfg, max_steps=after + 2 * steps)
    sim.init_particles()
    sim.step(after, cfg["dt"])
    s0 = sim.step_count
    kx, ky = sim.get_state()
    c0 = sim.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, cfg["dt"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = sim.counters()
    sim.set_state(kx, ky, step=s0)
    del kx, ky
    sim.set_profiling(True)
    sim.step(steps, cfg["dt"])
    kt = sim.kernel_times()
    sim.set_profiling(False)
    P, Q = sim.P, sim.Q
    out = {"after_steps": after, "t_ps": after * cfg["dt"] * 1e12, "steps": steps,
           "ms_per_step": wall * 1e3 / steps,
           "value": cfg["n_particles"] * Q * steps / wall,
           "kernels_us": {k: round(v[0] * 1e3, 1) for k, v in kt.items()},
           "candidates_per_step": (c1["candidates"] - c0["candidates"]) / steps,
           "collisions_per_step": (c1["collisions"] - c0["collisions"]) / steps}
    del sim
    torch.cuda.empty_cache()
    return out


def secondary_line(steps: int, warmup: int) -> dict:
    """The 8-node workload (1e6 particles, M = 5) in FP64: per-step rate and
    the rooflines of its dominant kernel and of its whole step."""
    from workloads import workload
    cfg = workload(SECONDARY, precision="fp64")
    log(f"{SECONDARY}: FP64, {warmup} warm-up + {steps} timed + {steps} profiled steps")
    r = run_gpu(cfg, steps, warmup)
    P, Q = r["sim"].P, r["sim"].Q
    roof, per, step = roofline_of(cfg, r, P, Q)
    roof["traffic"] = None      # the traffic record is the headline's
    out = {"workload": SECONDARY, "dtype": "f64", "n_particles": cfg["n_particles"],
           "gpc_modes": P, "nodes": Q, "ms_per_step": r["wall"] * 1e3 / steps,
           "value": cfg["n_particles"] * Q * steps / r["wall"], "unit": "particle-node updates/s",
           "roofline": roof, "roofline_step": step, "kernels": per,
           "candidates_per_step": r["cand"][0], "launch_shape": r["shape"]}
    del r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance sweep")
    ap.add_argument("--batched-steps", type=int, default=100)
    ap.add_argument("--late-steps", type=int, default=1000,
                    help="steps before the headline's late window (0: skip it)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 8-node, 1e6-particle FP64 line")
    ap.add_argument("--no-uq", action="store_true", help="skip the MC-MC / moments-at-z timings")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the timings of the other workloads at full size")
    ap.add_argument("--headline-only", action="store_true",
                    help="the headline FP64 run alone (counter runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shape of the headline (counter runs: "
                         "the traffic record then holds for that shape)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run five plain 256 MiB device copies (calibrates the HBM "
                         "byte counters of a profiler run)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record from two counter runs and exit (no GPU); "
                         "--steps gives the timed steps of those runs")
    args = ap.parse_args()
    if args.pmc_summary:
        print(json.dumps(pmc_summary(*args.pmc_summary, steps=args.steps), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs the step on one GPU (asked for {args.gpus}); the path is not "
              "sharded over several GPUs", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_cpu = args.no_fp32 = args.no_batched = args.no_secondary = True
        args.no_uq = args.no_configs = True
        args.late_steps = 0

    from workloads import workload

    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 copies of 268435456 bytes")
        del src, dst

    cfg = workload(WORKLOAD, precision="fp64")
    log(f"{WORKLOAD}: FP64, {args.warmup} warm-up + {args.steps} timed + {args.steps} profiled steps")
    r64 = run_gpu(cfg, args.steps, args.warmup, tune=not args.no_tune)
    P, Q, N = r64["sim"].P, r64["sim"].Q, cfg["n_particles"]
    pn = N * Q * args.steps
    roof, per, step = roofline_of(cfg, r64, P, Q)
    log(f"FP64 {r64['wall'] * 1e3 / args.steps:.4f} ms/step; kernels " +
        ", ".join(f"{k} {v['avg_ms'] * 1e3:.1f} us" for k, v in per.items()))

    out = {
        "metric": "particle-node updates/s + HBM GB/s; FP32-batched vs FP64 plain at matched err",
        "value": pn / r64["wall"],
        "unit": "particle-node updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_particles": N, "gpc_modes": P, "nodes": Q,
                   "grid": cfg["nk"], "dt_fs": cfg["dt"] * 1e15, "field_V_per_m": cfg["field0"],
                   "gap_eV": cfg["gap0"], "gap_rel": cfg["gap_rel"], "state": "fp64",
                   "launch": "hip graphs of 16 steps", "chunk": r64["shape"]["chunk"],
                   "collider_workgroups": r64["shape"]["collider_workgroups"]},
        "roofline": roof,
        "roofline_step": step,
        "kernels": per,
        "device_ms_per_step": r64["dev_ms"],
        "candidates_per_step": r64["cand"][0],
    }
    m64 = r64["moments"]
    del r64
    import torch
    torch.cuda.empty_cache()

    if args.late_steps > 0:
        out["late"] = late_window(cfg, after=args.late_steps)

    if not args.no_fp32:
        log("FP32 run of the same steps")
        r32 = run_gpu(dict(cfg, precision="fp32"), args.steps, args.warmup)
        dev = max_dev_over_se(m64, r32["moments"])
        _, per32, step32 = roofline_of(dict(cfg, precision="fp32"), r32, P, Q)
        out["fp32"] = {
            "value": pn / r32["wall"], "ms_per_step": r32["wall"] * 1e3 / args.steps,
            "kernels": per32, "roofline_step": step32,
            "speedup_vs_fp64": out["ms_per_step"] / (r32["wall"] * 1e3 / args.steps),
            "max_abs_dev_over_mc_se": dev,
            "matched_error": all(v < 3.0 for v in dev.values()),
        }
        del r32
        torch.cuda.empty_cache()

    if not args.no_secondary:
        out["secondary"] = secondary_line(args.steps, args.warmup)
        torch.cuda.empty_cache()

    if not args.no_batched:
        out["batched"] = sweep_forms(args.batched_steps)
        torch.cuda.empty_cache()

    if not args.no_uq:
        out["uq"] = uq_timings(workload(SECONDARY))

    if not args.no_configs:
        out["other_configs"] = other_configs()

    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
