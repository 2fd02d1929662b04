"""Benchmark of the sG-PM hot path on one MI355X.

Workload: sg_gap_m5_q8_n1e6 -- 1e6 particles, uncertain band gap
Delta(z) = 0.2 eV (1 + 0.1 z), Legendre order M = 5 (6 modes), 8 Gauss nodes,
E = 20 kV/cm, dt = 2 fs, FP64 particle state (the plain form), the paper's
rates and Pauli acceptance on a 240 x 240 grid.  A step is one pass of the
whole hot path (drift, node evaluation, collisions, histogram, moments) over
all particles.  The same steps are also run with FP32 particle state and the
two are compared against the Monte Carlo standard error.

Prints one JSON line.  Throughput is particle-node updates per second with the
state resident in HBM; the roofline of the step kernel uses its algorithmic
bytes per launch and its average duration from HIP events on the stream it
runs on.  The CPU baseline is the plain FP64 oracle on a bounded sample of the
same workload, on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "sg_gap_m5_q8_n1e6"


def algorithmic_bytes(cfg: dict, P: int, Q: int, n_drift_modes: int, candidates_per_step: float):
    """Bytes one step must move in HBM: read every coefficient; write back the
    drifted modes of the particles that do not collide and every mode of the
    ones that may; clear the stale histogram of Q nk^2 uint32 cells."""
    s = 4 if cfg.get("precision") == "fp32" else 8
    N = cfg["n_particles"]
    read = 2 * P * s * N
    write = (N - candidates_per_step) * n_drift_modes * s + candidates_per_step * 2 * P * s
    clear = Q * cfg["nk"] ** 2 * 4
    return read + write + clear


def run_gpu(cfg: dict, steps: int, warmup: int):
    import numpy as np
    import torch
    import paper_2404_19602_amd as sg

    sim = sg.Simulation(cfg, max_steps=warmup + steps)
    sim.init_particles()
    if warmup:
        sim.step(warmup, cfg["dt"])
    c0 = sim.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, cfg["dt"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = sim.last_step_ms()        # HIP events on the library's stream
    c1 = sim.counters()
    mom = sim.moments()
    t = sim.tables()
    n_drift = int(np.count_nonzero(t["ehat"]))
    cand = (c1["candidates"] - c0["candidates"]) / steps
    return dict(sim=sim, wall=wall, dev_ms=dev_ms, moments=mom, P=sim.P, Q=sim.Q,
                n_drift=n_drift, cand=cand, counters=c1)


def cpu_baseline(cfg: dict):
    """The FP64 oracle on a bounded sample: 50 000 of the particles for 200
    steps, every host thread the box gives this process."""
    import oracle
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))
    n_s, steps_s = 50_000, 200
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the sharded "
              "design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from workloads import workload

    cfg = workload(WORKLOAD)
    print(f"[bench] {WORKLOAD}: FP64, {args.warmup} warm-up + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    r64 = run_gpu(dict(cfg, precision="fp64"), args.steps, args.warmup)
    P, Q, N = r64["P"], r64["Q"], cfg["n_particles"]
    pn = N * Q * args.steps
    value = pn / r64["wall"]
    bytes64 = algorithmic_bytes(cfg, P, Q, r64["n_drift"], r64["cand"])
    achieved = bytes64 / (r64["dev_ms"] * 1e-3) / 1e9

    out = {
        "metric": "particle-node updates/s + HBM GB/s; FP32-batched vs FP64 plain at matched err",
        "value": value,
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
                   "gap_eV": cfg["gap0"], "gap_rel": cfg["gap_rel"], "state": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sgpm::step_kernel<double,8>",
                     "kernel_ms": r64["dev_ms"], "bytes_per_launch": bytes64},
        "hbm_GBps": achieved,
        "candidates_per_step": r64["cand"],
    }

    if not args.no_fp32:
        print("[bench] FP32 run of the same steps", file=sys.stderr, flush=True)
        r32 = run_gpu(dict(cfg, precision="fp32"), args.steps, args.warmup)
        m64, m32 = r64["moments"], r32["moments"]
        dev = {}
        for obs in ("E_vx", "Var_vx", "E_jx", "Var_jx", "E_energy"):
            se = np.maximum(m64["SE_" + obs][1:], 1e-300)
            dev[obs] = float(np.max(np.abs(m64[obs][1:] - m32[obs][1:]) / se))
        bytes32 = algorithmic_bytes(dict(cfg, precision="fp32"), P, Q, r32["n_drift"], r32["cand"])
        out["fp32"] = {
            "value": pn / r32["wall"], "ms_per_step": r32["wall"] * 1e3 / args.steps,
            "kernel_ms": r32["dev_ms"],
            "hbm_GBps": bytes32 / (r32["dev_ms"] * 1e-3) / 1e9,
            "speedup_vs_fp64": r64["wall"] / r32["wall"],
            "max_abs_dev_over_mc_se": dev,
            "matched_error": all(v < 3.0 for v in dev.values()),
        }
        del r32

    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
