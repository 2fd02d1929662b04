"""Seeded synthetic workloads of the sG-PM hot path.

Plain parameter dictionaries, shared by the product binding, the oracle, the
tests and the benchmark.  This module holds no arithmetic of the method: only
the physical and numerical parameters of each workload and the seed.

Units: gap0 in eV (gap_mode 0) or nm (gap_mode 1), fields in V/m, dt in s.
The uncertain variables z are uniform on [-1, 1]; ``gap_dim``/``field_dim``
name the z component (-1 = deterministic) that drives the band gap / field
linearly: gap(z) = gap0 (1 + gap_rel z), E(z) = field0 (1 + field_rel z).
"""
from __future__ import annotations

import copy

BASE_SEED = 2404196020

_COMMON = dict(fermi_eV=0.4, temp_K=300.0, alpha=0.1, nk=240, lk_eV=5.0, pauli=1,
               final_state=0, rate_scale=(1.0,) * 6, instance=0, c_max=32,
               gap_mode=0, dt=2e-15)

WORKLOADS = {
    # deterministic GNR (Algorithm 1): M = 0, one node
    "gnr_det_n1e4": dict(_COMMON, dim_z=0, degree=0, nodes_1d=1, n_particles=10_000,
                         gap0=0.2, gap_rel=0.0, gap_dim=-1, field0=1.0e6, field_rel=0.0,
                         field_dim=-1, steps=1000, precision="fp64", seed=BASE_SEED + 1),
    # sG-PM, uncertain gap, Legendre M = 5, 8 Gauss nodes, 1e6 particles, 2 ps
    "sg_gap_m5_q8_n1e6": dict(_COMMON, dim_z=1, degree=5, nodes_1d=8, n_particles=1_000_000,
                              gap0=0.2, gap_rel=0.1, gap_dim=0, field0=2.0e6, field_rel=0.0,
                              field_dim=-1, steps=1000, precision="fp64", seed=BASE_SEED + 2),
    # sG-PM, uncertain gap and field, total degree 4 (15 modes), 8x8 nodes, 4e6 particles
    "sg_gap_field_td4_q64_n4e6": dict(_COMMON, dim_z=2, degree=4, nodes_1d=8,
                                      n_particles=4_000_000, gap0=0.3, gap_rel=0.15, gap_dim=0,
                                      field0=1.5e6, field_rel=0.2, field_dim=1, steps=1000,
                                      precision="fp32", seed=BASE_SEED + 3),
    # large single instance, 256 x 256 grid, 10 ps
    "sg_gap_m8_q12_n3e7": dict(_COMMON, dim_z=1, degree=8, nodes_1d=12, n_particles=30_000_000,
                               gap0=0.25, gap_rel=0.2, gap_dim=0, field0=4.0e6, field_rel=0.0,
                               field_dim=-1, nk=256, steps=5000, precision="fp32",
                               seed=BASE_SEED + 5),
}


def workload(name: str, **overrides) -> dict:
    """A copy of a named workload with some parameters replaced."""
    cfg = copy.deepcopy(WORKLOADS[name])
    cfg.update(overrides)
    return cfg


def batched_sweep(n_inst: int = 64, n_min: float = 1e5, n_max: float = 2e6,
                  seed: int = BASE_SEED + 4, precision: str = "fp32", steps: int = 2500) -> list:
    """The batched parameter sweep: n_inst independent instances with the field
    uniform over 1-50 kV/cm, the mean band gap uniform over 0.1-0.5 eV with a
    +-10 % uniform uncertainty, Legendre order M drawn from {2, 4, 6} with
    Q = M + 3 Gauss nodes, and particle counts log-uniform in [n_min, n_max].
    The draws come from numpy's PCG64 seeded with ``seed``; every instance
    shares the Philox key and has its own instance word, so the random
    streams of the method are independent."""
    import math

    import numpy as np

    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_inst):
        field = float(rng.uniform(1.0e5, 5.0e6))
        gap0 = float(rng.uniform(0.1, 0.5))
        M = int(rng.choice([2, 4, 6]))
        N = int(round(10.0 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
        out.append(dict(_COMMON, dim_z=1, degree=M, nodes_1d=M + 3, n_particles=N, gap0=gap0,
                        gap_rel=0.1, gap_dim=0, field0=field, field_rel=0.0, field_dim=-1,
                        steps=steps, precision=precision, seed=seed, instance=j))
    return out
