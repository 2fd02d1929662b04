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
