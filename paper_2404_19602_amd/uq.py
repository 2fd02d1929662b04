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
"""
from __future__ import annotations

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
