"""Uncertainty-quantification drivers over the sG-PM library.

Everything here marshals arguments for the C-ABI and aggregates its outputs;
the particles are stepped by the library's kernels.

* ``mc_sampling``: the Monte Carlo sampling of z with deterministic runs that
  the paper compares the sG-PM against (MC-MC, Sec. 5 Test 4). The samples run
  as a batch of deterministic instances in one context, so one launch of each
  kernel per step serves every sample.
* ``sg_error``: the L2(z) error of the mean energy of truncation orders M
  against a reference order (Sec. 5 Test 3). All orders run in one context with
  the same Philox key and instance word, so they consume the same random
  numbers (the collisional tree is replayed).
* ``percentile_bands``: bands over z of the mean energy and velocity from the
  particle expansion evaluated at sampled z (Sec. 5 Test 2, Sec. 4.2).
* ``error_versus_cost``: the error of E_z[V_x](t) of the sG-PM (MC-sG) for
  truncation orders M1 and of MC-MC for sample counts M2, both at N particles,
  against a reference sG-PM run with many particles and a high order, beside
  the cost per particle of each (M1^2 and M2 by the paper's cost model, and
  the measured device time per step) (Sec. 5 Test 4).
"""
from __future__ import annotations

import time

import numpy as np

from . import Simulation

_DET = dict(dim_z=0, degree=0, nodes_1d=1, gap_dim=-1, gap_rel=0.0, field_dim=-1,
            field_rel=0.0)


def sample_z(n: int, dim_z: int, seed: int) -> np.ndarray:
    """n points uniform on [-1, 1]^dim_z (numpy PCG64 from the seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, dim_z))


def deterministic_at(cfg: dict, z) -> list:
    """The deterministic problems of an uncertain workload at points z
    ([n][dim_z]): the band gap (or width) and the field take the values the
    library evaluates at each z (``sgpm_inputs_at``)."""
    probe = Simulation(dict(cfg, n_particles=1), max_steps=0)
    vals = probe.inputs_at(z)
    del probe
    out = []
    for k in range(len(vals["field"])):
        c = dict(cfg)
        c.update(_DET)
        if int(cfg.get("gap_mode", 0)) == 1:
            c["gap0"] = float(vals["width_m"][k] * 1e9)
        else:
            c["gap0"] = float(vals["gap_eV"][k])
        c["field0"] = float(vals["field"][k])
        out.append(c)
    return out


def mc_sampling(cfg: dict, n_samples: int, steps: int, seed: int = 7,
                n_particles: int | None = None, dt: float | None = None) -> dict:
    """MC-MC: E_z and Var_z of V_x, J_x and the mean energy at every step from
    n_samples deterministic runs at z drawn uniformly, with the standard error
    of the sample mean.  Each sample has its own instance word (independent
    random streams)."""
    dt = cfg.get("dt", 2e-15) if dt is None else dt
    z = sample_z(n_samples, int(cfg.get("dim_z", 0)), seed)
    cfgs = deterministic_at(cfg, z)
    for k, c in enumerate(cfgs):
        c["instance"] = k
        if n_particles is not None:
            c["n_particles"] = int(n_particles)
    sim = Simulation(cfgs, max_steps=steps)
    sim.init_particles()
    sim.step(steps, dt)
    rec = [sim.moments(inst=k) for k in range(n_samples)]
    vx = np.stack([r["per_node_vx"][:, 0] for r in rec])
    jx = np.stack([r["per_node_jx"][:, 0] for r in rec])
    en = np.stack([r["per_node_energy"][:, 0] for r in rec])
    out = {"z": z, "sim": sim, "cfgs": cfgs}
    for name, v in (("vx", vx), ("jx", jx), ("energy", en)):
        out["E_" + name] = v.mean(axis=0)
        out["Var_" + name] = v.var(axis=0, ddof=1) if n_samples > 1 else np.zeros(v.shape[1])
        out["SE_E_" + name] = np.sqrt(out["Var_" + name] / n_samples)
    return out


def sg_error(cfg: dict, orders, m_ref: int, times_steps, nodes_for=lambda m: m + 3,
             n_quad: int = 32, dt: float | None = None) -> dict:
    """L2(z) error of the mean energy E(t, z) of each truncation order against
    the order m_ref, at the given step counts, for one uncertain input:
    sqrt(int (E_ref - E_M)^2 dz/2) by an n_quad-point Gauss-Legendre rule."""
    if int(cfg.get("dim_z", 0)) != 1:
        raise ValueError("sg_error takes workloads with one uncertain input")
    dt = cfg.get("dt", 2e-15) if dt is None else dt
    orders = list(orders)
    all_m = orders + [m_ref]
    cfgs = [dict(cfg, degree=m, nodes_1d=nodes_for(m)) for m in all_m]
    x, w = np.polynomial.legendre.leggauss(n_quad)
    w = w / 2.0
    times_steps = sorted(int(t) for t in times_steps)
    sim = Simulation(cfgs, max_steps=max(times_steps))
    sim.init_particles()
    done = 0
    err = np.zeros((len(times_steps), len(orders)))
    for it, t in enumerate(times_steps):
        if t > done:
            sim.step(t - done, dt)
            done = t
        e_ref = sim.moments_at(x, inst=len(orders))["energy"]
        for k in range(len(orders)):
            e = sim.moments_at(x, inst=k)["energy"]
            err[it, k] = np.sqrt(np.sum(w * (e - e_ref) ** 2))
    return {"orders": orders, "m_ref": m_ref, "steps": times_steps, "error": err}


def percentile_bands(sim: Simulation, percentiles=(10.0, 90.0), n_z: int = 256, seed: int = 11,
                     inst: int = 0) -> dict:
    """Percentiles over z (sampled uniformly) of the mean energy and V_x of the
    current state, with their expectation over the samples."""
    dz = int(sim.cfgs[inst].get("dim_z", 0))
    z = sample_z(n_z, max(dz, 1), seed)[:, :max(dz, 1)]
    m = sim.moments_at(z, inst=inst)
    out = {"z": z}
    for k in ("energy", "V_x"):
        out[k] = m[k]
        out[k + "_mean"] = float(np.mean(m[k]))
        out[k + "_bands"] = np.percentile(m[k], percentiles)
    out["percentiles"] = tuple(percentiles)
    return out


def _timed_steps(sim: Simulation, steps: int, dt: float) -> float:
    """Steps the simulation and returns the wall time per step in ms (the
    stream is synchronised before and after)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, dt)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / max(steps, 1)


def error_versus_cost(cfg: dict, n: int, steps: int, sg_orders, mc_samples, n_ref: int,
                      m_ref: int, nodes_for=lambda m: m + 3, seed: int = 7,
                      dt: float | None = None) -> dict:
    """Sec. 5 Test 4 for one uncertain input: Error = |E_z[V_x](t) -
    E_z[V_x^ref](t)| at t = steps dt.

    * Reference: the sG-PM of order m_ref with n_ref particles.
    * MC-sG: the sG-PM of each order M1 in sg_orders with n particles (every
      order in one context, on the same random streams); cost per particle
      M1^2.
    * MC-MC: max(mc_samples) deterministic runs of n particles at z drawn
      uniformly (one batched context); the estimate of M2 samples is the mean
      of the first M2 runs; cost per particle M2.

    Besides the errors: the Monte Carlo standard errors of the estimates (the
    reference's and the MC-sG's from their batch means; MC-MC's from the
    spread over its samples), and the measured device time per step of each
    run.  The reference and the MC-sG runs use different random streams
    (instance words 1 and 0)."""
    if int(cfg.get("dim_z", 0)) != 1:
        raise ValueError("error_versus_cost takes workloads with one uncertain input")
    dt = cfg.get("dt", 2e-15) if dt is None else dt
    sg_orders = [int(m) for m in sg_orders]
    mc_samples = sorted(int(m) for m in mc_samples)
    out = {"steps": steps, "t_s": steps * dt, "n": n, "n_ref": n_ref, "m_ref": m_ref}

    ref = Simulation(dict(cfg, degree=m_ref, nodes_1d=nodes_for(m_ref), n_particles=n_ref,
                          instance=1), max_steps=steps)
    ref.init_particles()
    out["ref_ms_per_step"] = _timed_steps(ref, steps, dt)
    m = ref.moments(steps, 1)
    e_ref, se_ref = float(m["E_vx"][0]), float(m["SE_E_vx"][0])
    out["ref_E_vx"], out["ref_SE"] = e_ref, se_ref
    del ref

    cfgs = [dict(cfg, degree=m1, nodes_1d=nodes_for(m1), n_particles=n, instance=0)
            for m1 in sg_orders]
    sim = Simulation(cfgs, max_steps=steps)
    sim.init_particles()
    out["sg_ms_per_step_all_orders"] = _timed_steps(sim, steps, dt)
    sg = []
    for k, m1 in enumerate(sg_orders):
        mk = sim.moments(steps, 1, inst=k)
        sg.append({"M1": m1, "cost_per_particle": m1 * m1, "E_vx": float(mk["E_vx"][0]),
                   "SE": float(mk["SE_E_vx"][0]),
                   "error": abs(float(mk["E_vx"][0]) - e_ref)})
    del sim
    # per-order device time: each order alone
    for row in sg:
        one = Simulation(dict(cfg, degree=row["M1"], nodes_1d=nodes_for(row["M1"]),
                              n_particles=n, instance=0), max_steps=steps)
        one.init_particles()
        row["ms_per_step"] = _timed_steps(one, steps, dt)
        del one
    out["mc_sg"] = sg

    z = sample_z(max(mc_samples), 1, seed)
    dcfgs = deterministic_at(cfg, z)
    for k, c in enumerate(dcfgs):
        c.update(instance=k, n_particles=n)
    det = Simulation(dcfgs, max_steps=steps)
    det.init_particles()
    out["mc_ms_per_step_all_samples"] = _timed_steps(det, steps, dt)
    vx = np.array([float(det.moments(steps, 1, inst=k)["E_vx"][0]) for k in range(len(dcfgs))])
    se_part = np.array([float(det.moments(steps, 1, inst=k)["SE_E_vx"][0])
                        for k in range(len(dcfgs))])
    del det
    mc = []
    for m2 in mc_samples:
        est = float(vx[:m2].mean())
        spread = float(vx[:m2].std(ddof=1) / np.sqrt(m2)) if m2 > 1 else float("nan")
        mc.append({"M2": m2, "cost_per_particle": m2, "E_vx": est, "error": abs(est - e_ref),
                   "SE_particles": float(np.sqrt(np.sum(se_part[:m2] ** 2)) / m2),
                   "SE_samples": spread})
    out["mc_mc"] = mc
    out["std_z_vx_samples"] = float(vx.std(ddof=1)) if len(vx) > 1 else float("nan")
    return out
