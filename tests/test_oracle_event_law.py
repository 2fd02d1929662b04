"""Pins of the oracle's collision event law (CPU only).

The free flight and the mechanism selection of the collision loop (Sec. 3:
eq. dt, eq. gamma_tot, eq. lambda, eq. update; Sec. 4.1: eq. deltat) are
checked against what they must produce statistically, with the total rates
taken from the Section 2 transition rates integrated by the test itself
(``sec2_rates``), not from the oracle:

* with one collision iteration at most (c_max = 1) the iteration happens
  within dt with probability 1 - exp(-G dt), G = (1 + alpha) max_q S_q, and
  at node q it is a real event with probability S_q / G; the real events
  split over the mechanisms as Gamma^nu / S_q, read from the energy change;
* over many iterations the number of real events of an elastic-only gas is
  Poisson with mean S dt per particle and the iterations Poisson with mean
  G dt;
* with the Pauli acceptance off, no field and one phonon branch, every
  particle's energy moves on its lattice eps_i(0) + m hbar omega, so the
  relaxed mean energy at the lattice temperature is the Boltzmann average
  over each particle's lattice (detailed balance of the Appendix rates),
  reached from a hotter (or colder) Fermi-Dirac start.

A mistake in the law (normalising the selection by S_q instead of G,
dropping (1 + alpha) from the free flight, swapping emission and
absorption) fails at least one of them; ``test_oracle_mutants.py`` checks
that on mutated copies of the oracle.
"""
import math

import numpy as np
import pytest

from test_oracle_pins import sec2_rates, small

K_B_EV = 1.380649e-23 / 1.602176634e-19      # Boltzmann constant in eV/K
HW_O, HW_K = 0.1646, 0.124                     # Table 1 phonon energies, eV


def _state(n, eps, angle, e0):
    k = math.sqrt(eps * eps - e0 * e0)
    return (np.full((n, 1), k * math.cos(angle)), np.full((n, 1), k * math.sin(angle)))


def _z(count, n, p):
    """binomial z-score of count successes in n trials of probability p"""
    return (count - n * p) / math.sqrt(n * p * (1.0 - p))


@pytest.mark.parametrize("eps,angle,alpha", [(0.6, 0.7, 0.1), (0.35, 2.1, 0.1), (0.6, 0.7, 0.5)])
def test_single_iteration_law(orc, eps, angle, alpha):
    """c_max = 1, Pauli off, no field, M = 0: P(iteration in dt) = 1 - exp(-G dt);
    P(real event | iteration) = S/G; mechanism shares Gamma^nu / S by the
    energy change (elastic AC + edge, -/+ hbar w_O, -/+ hbar w_K)."""
    e0 = 0.1
    cfg = small(field0=0.0, pauli=0, c_max=1, gap0=2 * e0, alpha=alpha, n_particles=4, seed=31)
    s = orc.OracleSim(cfg)
    W = s.tables()["width"][0]
    R = sec2_rates(eps, math.cos(angle), math.sqrt(eps * eps - e0 * e0), e0, W)
    S = R.sum()
    G = (1.0 + alpha) * S
    n = 200_000
    dt = 1.0 / G
    kx, ky = _state(n, eps, angle, e0)
    ox, oy, nc = s.step_particles(np.arange(n), kx, ky, 0, dt)
    it = nc == 1
    assert set(np.unique(nc)) <= {0, 1}
    assert abs(_z(it.sum(), n, 1.0 - math.exp(-G * dt))) < 4.5
    changed = (ox[:, 0] != kx[:, 0]) | (oy[:, 0] != ky[:, 0])
    assert not np.any(changed & ~it)
    assert abs(_z(changed.sum(), it.sum(), S / G)) < 4.5
    de = np.sqrt(ox[:, 0] ** 2 + oy[:, 0] ** 2 + e0 * e0) - eps
    n_ev = int(changed.sum())
    classes = {"elastic": (0.0, R[0] + R[5]), "O-": (-HW_O, R[1]), "O+": (HW_O, R[2]),
               "K-": (-HW_K, R[3]), "K+": (HW_K, R[4])}
    total = 0
    for name, (shift, rate) in classes.items():
        hit = changed & (np.abs(de - shift) < 1e-9)
        total += int(hit.sum())
        p = rate / S
        if p == 0.0:
            assert hit.sum() == 0, name
        else:
            assert abs(_z(hit.sum(), n_ev, p)) < 4.5, (name, hit.sum() / n_ev, p)
    assert total == n_ev


def test_single_iteration_node_acceptance(orc):
    """sG with Q = P (projection is invertible): one iteration, shared s, node
    q accepts a real event with probability S_q / G, G = (1 + alpha) max_q S_q
    (eq. deltat with the maximum over the nodes, eq. update normalised by it)."""
    cfg = small(dim_z=1, degree=3, nodes_1d=4, gap_dim=0, gap0=0.2, gap_rel=0.4, field0=0.0,
                pauli=0, c_max=1, n_particles=4, seed=77)
    s = orc.OracleSim(cfg)
    t = s.tables()
    psi, w = t["psi"], t["w"]
    Q = psi.shape[0]
    eps, angle = 0.55, 1.1
    e0 = t["eps0"]
    kabs = np.sqrt(eps * eps - e0 * e0)            # the same nodal energy at every node
    nodes_x, nodes_y = kabs * math.cos(angle), kabs * math.sin(angle)
    cx = (w[:, None] * psi).T @ nodes_x            # project the nodal values
    cy = (w[:, None] * psi).T @ nodes_y
    Sq = np.array([sec2_rates(eps, math.cos(angle), kabs[q], e0[q], t["width"][q]).sum()
                   for q in range(Q)])
    G = 1.1 * Sq.max()
    n = 120_000
    dt = 1.0 / G
    ox, oy, nc = s.step_particles(np.arange(n), np.tile(cx, (n, 1)), np.tile(cy, (n, 1)), 0, dt)
    it = nc == 1
    assert abs(_z(it.sum(), n, 1.0 - math.exp(-1.0))) < 4.5
    vx, vy = ox @ psi.T, oy @ psi.T                 # node values after the step [n][Q]
    for q in range(Q):
        moved = (np.abs(vx[:, q] - nodes_x[q]) > 1e-9) | (np.abs(vy[:, q] - nodes_y[q]) > 1e-9)
        assert not np.any(moved & ~it)
        assert abs(_z(moved.sum(), it.sum(), Sq[q] / G)) < 4.5, (q, moved[it].mean(), Sq[q] / G)
    # the node with the smallest rate (largest band minimum) is left out more often
    assert Sq.min() < 0.9 * Sq.max()


def test_elastic_event_counts_are_poisson(orc):
    """AC only (elastic, rate fixed by the energy): over a step of length dt
    each particle has Poisson(S dt) real events among Poisson(G dt) iterations,
    and the cap is never reached."""
    e0, eps, angle = 0.1, 0.45, 0.3
    cfg = small(field0=0.0, pauli=0, c_max=255, rate_scale=(1, 0, 0, 0, 0, 0), n_particles=4,
                seed=91)
    s = orc.OracleSim(cfg)
    W = s.tables()["width"][0]
    S = sec2_rates(eps, math.cos(angle), math.sqrt(eps * eps - e0 * e0), e0, W)[0]
    G = 1.1 * S
    n = 40_000
    dt = 3.0 / S
    kx, ky = _state(n, eps, angle, e0)
    ox, oy, nc = s.step_particles(np.arange(n), kx, ky, 0, dt)
    iters = nc.astype(np.float64)
    assert abs(iters.mean() - G * dt) < 4.5 * math.sqrt(G * dt / n)
    assert abs(iters.var() - G * dt) < 0.05 * G * dt          # Poisson: variance = mean
    e_after = np.sqrt(ox[:, 0] ** 2 + oy[:, 0] ** 2 + e0 * e0)
    assert np.allclose(e_after, eps, rtol=1e-13)
    # real events: the counters of a run of the same particles through the oracle's step
    cfg2 = dict(cfg, n_particles=n)
    r = orc.OracleSim(cfg2)
    r.set_state(np.tile(kx[:, 0], (1, 1)), np.tile(ky[:, 0], (1, 1)), step=0)
    r.run(dt, 1)
    c = r.counters()
    assert c["collisions"] == int(nc.sum())             # the same random streams
    assert c["cmax_hits"] == 0
    assert abs(c["events"] - n * S * dt) < 4.5 * math.sqrt(n * S * dt)
    assert abs(c["collisions"] - n * G * dt) < 4.5 * math.sqrt(n * G * dt)


def _orbit_boltzmann(eps, e0, hw, kT):
    """Per particle: mean and variance of the energy under the Boltzmann
    weights eps exp(-eps/kT) (density of states ~ eps, Sec. 2 dispersion) on
    the lattice eps_i + m hw, eps >= e0, that its phonon events can reach."""
    m0 = np.ceil((e0 - eps) / hw - 1e-12)
    lev = eps[:, None] + (m0[:, None] + np.arange(80)[None, :]) * hw
    wgt = lev * np.exp(-(lev - lev[:, :1]) / kT)
    wgt /= wgt.sum(axis=1, keepdims=True)
    mean = (wgt * lev).sum(axis=1)
    return mean, (wgt * (lev - mean[:, None]) ** 2).sum(axis=1)


@pytest.mark.parametrize("branch,T_lattice,T_init,dt,steps", [
    ("O", 300.0, 900.0, 1e-14, 400),     # hot start relaxes to the 300 K lattice
    ("K", 300.0, 900.0, 5e-14, 400),
    ("O", 1500.0, 300.0, 1e-14, 400),    # cold start heated by a hot lattice
])
def test_relaxation_to_the_lattice_temperature(orc, branch, T_lattice, T_init, dt, steps):
    """No field, Pauli off, one phonon branch plus the elastic mechanisms: the
    energy of each particle changes by +/- hbar w per event, emission and
    absorption obey detailed balance at the lattice temperature, so the mean
    energy relaxes from the Fermi-Dirac datum at T_init to the Boltzmann
    average at T_lattice over each particle's energy lattice."""
    e0 = 0.1
    scale = (1, 1, 1, 0, 0, 1) if branch == "O" else (1, 0, 0, 1, 1, 1)
    hw = HW_O if branch == "O" else HW_K
    n = 20_000
    cfg = small(field0=0.0, pauli=0, c_max=64, n_particles=n, temp_K=T_lattice,
                init_temp_K=T_init, rate_scale=scale, seed=5)
    s = orc.OracleSim(cfg, threads=8)
    s.init()
    kx, ky = s.get_state()
    eps0 = np.sqrt(kx[0] ** 2 + ky[0] ** 2 + e0 * e0)
    mean, var = _orbit_boltzmann(eps0, e0, hw, K_B_EV * T_lattice)
    target = mean.mean()
    s.run(dt, steps)
    e = np.array([r[0][2] for r in s.record])
    late = e[-100:].mean()
    # the start is far from the target, the end is on it: each particle's
    # late energy is a draw from its lattice distribution
    assert abs(e[0] - target) > 0.015
    tol = 4.0 * math.sqrt(var.mean() / n) + 1e-5 * target
    assert abs(late - target) < tol, (late, target, tol)
    kx, ky = s.get_state()
    k = (np.sqrt(kx[0] ** 2 + ky[0] ** 2 + e0 * e0) - eps0) / hw
    assert np.max(np.abs(k - np.round(k))) < 1e-9        # every particle on its lattice


def test_initial_temperature_sets_only_the_datum(orc):
    """init_temp_K changes the Fermi-Dirac datum (its mean energy and the
    density used for J), not the lattice rates."""
    a = orc.OracleSim(small(n_particles=3000, init_temp_K=900.0))
    b = orc.OracleSim(small(n_particles=3000))
    ra = a.rates(0, [0.4, 0.7], [0.1, 0.0])
    rb = b.rates(0, [0.4, 0.7], [0.1, 0.0])
    assert np.array_equal(ra, rb)
    a.init(); b.init()
    assert a.record[0][0][2] > b.record[0][0][2] + 0.03
    ta, tb = a.tables(), b.tables()
    assert ta["density"][0] != tb["density"][0]
    kT9 = K_B_EV * 900.0
    assert abs(ta["density"][0] - orc.density_closed(0.1, 0.4, kT9)) < 1e-10 * ta["density"][0]
