"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

FP64 path: trajectories per particle to 1e-10 relative (scale: the
particle's coefficient norm, at least 1 meV), up to rare branch flips that
are counted and bounded; integer outputs (histograms, counters) bit-exact
when no flip occurred.  FP32 path: observables within 3 Monte Carlo
standard errors of the FP64 path.
"""
import math
import os

import numpy as np
import pytest

from workloads import workload

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def sg():
    import paper_2404_19602_amd as sg
    return sg


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def rel_err(gx, gy, ox, oy):
    """per-particle max |difference| over modes / max(coefficient norm, 1 meV)"""
    scale = np.maximum(np.sqrt((ox ** 2 + oy ** 2).sum(axis=0)), 1e-3)
    return np.maximum(np.abs(gx - ox).max(axis=0), np.abs(gy - oy).max(axis=0)) / scale


def announce(name, cfg):
    print(f"\n[gpu case] {name}: N={cfg['n_particles']} dim_z={cfg.get('dim_z')} "
          f"M={cfg.get('degree')} Q1={cfg.get('nodes_1d')} prec={cfg.get('precision', 'fp64')}",
          flush=True)


def small_cfg(**kw):
    base = dict(dim_z=0, degree=0, nodes_1d=1, n_particles=2000, gap_mode=0, gap_dim=-1,
                gap0=0.2, gap_rel=0.0, field_dim=-1, field0=1e6, field_rel=0.0, fermi_eV=0.4,
                temp_K=300.0, alpha=0.1, nk=240, lk_eV=5.0, pauli=1, final_state=0,
                rate_scale=(1.0,) * 6, seed=4242, instance=0, c_max=32, dt=2e-15,
                precision="fp64", steps=400)
    base.update(kw)
    return base


# ------------------------------------------------------------------ RNG
def test_philox_device_matches_oracle(sg, orc):
    rng = np.random.default_rng(0)
    n = 100_000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0; key[0] = 0
    ctr[1] = 0xFFFFFFFF; key[1] = 0xFFFFFFFF
    assert np.array_equal(sg.philox_device(ctr, key), orc.philox(ctr, key))


# ---------------------------------------------------------------- tables
@pytest.mark.parametrize("cfg", [
    small_cfg(),
    small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1),
    small_cfg(dim_z=2, degree=4, nodes_1d=8, gap_dim=0, gap0=0.3, gap_rel=0.15, field_dim=1,
              field0=1.5e6, field_rel=0.2),
    small_cfg(dim_z=1, degree=3, nodes_1d=5, gap_mode=1, gap0=7.0, gap_rel=1 / 14, gap_dim=0),
])
def test_tables_match_oracle(sg, orc, cfg):
    g = sg.Simulation(cfg).tables()
    o = orc.OracleSim(cfg).tables()
    for k in ("z", "w", "psi", "ehat", "eps0", "width", "field", "density"):
        a, b = g[k], o[k]
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * (np.abs(b).max() + 1e-300)), k


# ------------------------------------------------------------------ init
INIT_CASES = {
    "det": small_cfg(n_particles=10_000),
    "sg_gap": small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1, n_particles=20_000,
                        field0=2e6),
    "sg_2d": small_cfg(dim_z=2, degree=4, nodes_1d=8, gap_dim=0, gap0=0.3, gap_rel=0.15,
                       field_dim=1, field0=1.5e6, field_rel=0.2, n_particles=3_000),
    "width": small_cfg(dim_z=1, degree=3, nodes_1d=5, gap_mode=1, gap0=7.0, gap_rel=1 / 14,
                       gap_dim=0, n_particles=4_097),
    # a Fermi-Dirac datum hotter than the lattice
    "hot_start": small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1,
                           n_particles=6_000, init_temp_K=900.0),
}


@pytest.mark.parametrize("name", list(INIT_CASES))
def test_init_parity(sg, orc, name):
    cfg = INIT_CASES[name]
    announce("init " + name, cfg)
    sim = sg.Simulation(cfg)
    sim.init_particles()
    gx, gy = sim.get_state()
    ref = orc.OracleSim(cfg)
    ref.init()
    ox, oy = ref.get_state()
    err = rel_err(gx, gy, ox, oy)
    assert err.max() <= TOL, err.max()
    H, M = sim.histogram()
    Ho, Mo = ref.histogram()
    assert np.array_equal(H, Ho) and np.array_equal(M, Mo)
    m = sim.moments()
    rec = np.asarray(ref.record)
    assert np.allclose(m["per_node_vx"][0], rec[0, :, 0], rtol=1e-9, atol=1e-6)
    assert np.allclose(m["per_node_energy"][0], rec[0, :, 2], rtol=1e-12)


# ---------------------------------------------------------------- steps
STEP_CASES = {
    "strang_sg_gap": (small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1,
                                n_particles=20_001, field0=5e6, splitting=1), 120, 1024),
    "det_n1e4": (small_cfg(n_particles=10_000), 300, None),
    # a fine grid (0.0083 eV cells): the Fermi disk spans about +-48 cells while the LDS
    # window of eight nodes spans +-31, so much of H^n goes through the overflow grid
    "window_overflow": (small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1,
                                  n_particles=20_001, field0=2e6, lk_eV=1.0), 80, 1024),
    "sg_gap_ragged": (small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1,
                                n_particles=20_001, field0=2e6), 120, 1024),
    "sg_2d_q64": (small_cfg(dim_z=2, degree=4, nodes_1d=8, gap_dim=0, gap0=0.3, gap_rel=0.15,
                            field_dim=1, field0=1.5e6, field_rel=0.2, n_particles=3_000), 25, None),
    # 28 modes: the kernels' largest mode bucket (32)
    "sg_2d_td6_p28": (small_cfg(dim_z=2, degree=6, nodes_1d=7, gap_dim=0, gap0=0.3, gap_rel=0.15,
                                field_dim=1, field0=1.5e6, field_rel=0.2, n_particles=1_500),
                      20, None),
    # 81 nodes: two nodes per collider lane
    "sg_2d_q81": (small_cfg(dim_z=2, degree=3, nodes_1d=9, gap_dim=0, gap0=0.3, gap_rel=0.15,
                            field_dim=1, field0=1.5e6, field_rel=0.2, n_particles=2_000), 25, None),
    "hot_field_small_grid": (small_cfg(dim_z=1, degree=2, nodes_1d=3, gap_dim=0, gap_rel=0.2,
                                       field0=3e7, n_particles=5_000, nk=64, lk_eV=1.2), 120, 1024),
    "pauli_off_literal": (small_cfg(dim_z=1, degree=3, nodes_1d=4, gap_dim=0, gap_rel=0.1,
                                    pauli=0, final_state=1, field0=5e6, n_particles=5_000), 80,
                          None),
    "single_particle": (small_cfg(n_particles=1, rate_scale=(30.0,) * 6), 200, None),
    # hot start at zero field relaxing toward the lattice temperature
    "hot_start_relaxation": (small_cfg(dim_z=1, degree=3, nodes_1d=4, gap_dim=0, gap_rel=0.2,
                                       field0=0.0, init_temp_K=900.0, n_particles=8_000), 150,
                             None),
    "field_uncertain_m8": (small_cfg(dim_z=1, degree=8, nodes_1d=12, field_dim=0, field0=4e6,
                                     field_rel=0.5, gap_dim=0, gap0=0.25, gap_rel=0.2,
                                     nk=256, n_particles=6_000), 60, None),
}


@pytest.mark.parametrize("name", list(STEP_CASES))
def test_step_parity(sg, orc, name):
    cfg, steps, chunk = STEP_CASES[name]
    announce("step " + name, cfg)
    ref = orc.OracleSim(cfg, threads=8)
    ref.init()
    kx0, ky0 = ref.get_state()
    sim = sg.Simulation(cfg, max_steps=steps)
    if chunk:
        sim.set_chunk(chunk)
    sim.set_state(kx0, ky0, step=0)
    H0, M0 = sim.histogram()
    Ho, Mo = ref.histogram()
    assert np.array_equal(H0, Ho) and np.array_equal(M0, Mo)
    sim.step(steps, cfg["dt"])
    ref.run(cfg["dt"], steps)
    gx, gy = sim.get_state()
    ox, oy = ref.get_state()
    err = rel_err(gx, gy, ox, oy)
    flips = int(np.count_nonzero(err > TOL))
    print(f"  max rel err (non-flipped) {err[err <= TOL].max() if flips < err.size else 0:.2e}, "
          f"flipped particles {flips}, counters {sim.counters()}", flush=True)
    assert flips <= max(2, cfg["n_particles"] // 10_000)
    gc, oc = sim.counters(), ref.counters()
    if flips == 0:
        for k in ("collisions", "events", "pauli_rejected", "edge_exhausted", "cmax_hits"):
            assert gc[k] == oc[k], (k, gc[k], oc[k])
        H, M = sim.histogram()
        Ho, Mo = ref.histogram()
        assert np.array_equal(H, Ho) and np.array_equal(M, Mo)
        # particles above the maximum occupation number, every step (Pauli violation)
        assert np.array_equal(sim.occupancy_excess(), np.asarray(ref.excess, dtype=np.uint32))
    assert gc["collisions"] > 0 or cfg["n_particles"] == 1
    m = sim.moments()
    rec = np.asarray(ref.record)
    tol_v = 1e-9 if flips == 0 else 2e6 * flips / cfg["n_particles"]
    assert np.allclose(m["per_node_vx"], rec[:, :, 0], rtol=1e-9, atol=tol_v)
    assert np.allclose(m["per_node_energy"], rec[:, :, 2], rtol=1e-9,
                       atol=(1e-12 if flips == 0 else 5.0 * flips / cfg["n_particles"]))
    q = ref.qoi()
    assert np.allclose(m["E_vx"], q["E_vx"], rtol=1e-8, atol=tol_v)
    assert np.allclose(m["E_jx"], q["E_jx"], rtol=1e-8, atol=1e-9 * np.abs(q["E_jx"]).max() + 1e-6)


@pytest.mark.parametrize("degree,nodes", [(5, 8), (4, 7)])
def test_window_counts_beyond_16_bits(sg, orc, degree, nodes):
    """The mirror-pair stream kernel packs two nodes' window counts as 16-bit
    halves of a word.  One workgroup here takes all 200 000 particles: 70 000
    sit at k = 0 and 70 000 at an odd-mode offset (mirror cells at nodes p and
    Q-1-p, and k = 0 again at the middle node of an odd Q), so at every node
    one window cell gets more than 65535 of that workgroup's counts, in the low
    and in the high halves.  The histogram is still the oracle's, after the
    state is set and after two steps."""
    n = 200_000
    cfg = small_cfg(dim_z=1, degree=degree, nodes_1d=nodes, gap_dim=0, gap_rel=0.1,
                    n_particles=n, field0=2e6)
    announce(f"window counts beyond 16 bits, Q={nodes}", cfg)
    ref = orc.OracleSim(cfg, threads=8)
    P = ref.P
    rng = np.random.default_rng(9)
    kx = np.zeros((P, n)); ky = np.zeros((P, n))
    kx[1, 70_000:140_000] = 0.15
    kx[0, 140_000:] = rng.normal(0.0, 0.1, n - 140_000)
    ky[0, 140_000:] = rng.normal(0.0, 0.1, n - 140_000)
    kx[1:, 140_000:] = rng.normal(0.0, 0.01, (P - 1, n - 140_000))
    sim = sg.Simulation(cfg, max_steps=4)
    sim.set_node_pairs(True)
    assert sim.node_pairs()
    sim.set_chunk(200_704)
    assert sim.launch_shape()["stream_workgroups"] == 1
    # the concentrated cells (|k| < 0.3 eV) lie inside the LDS window
    dk = 2 * cfg["lk_eV"] / cfg["nk"]
    assert sim.window()["cells"] >= 2 * math.ceil(0.3 / dk) + 2
    ref.set_state(kx, ky, step=0)
    sim.set_state(kx, ky, step=0)
    H, M = sim.histogram()
    Ho, Mo = ref.histogram()
    assert Ho.max() >= 70_000 and np.all(Ho.sum(axis=(1, 2)) == n)
    assert np.array_equal(H, Ho) and np.array_equal(M, Mo)
    sim.step(2, cfg["dt"])
    ref.run(cfg["dt"], 2)
    gx, gy = sim.get_state()
    ox, oy = ref.get_state()
    flips = int(np.count_nonzero(rel_err(gx, gy, ox, oy) > TOL))
    print(f"  flipped particles {flips}, counters {sim.counters()}", flush=True)
    assert flips <= max(2, n // 10_000)
    H, M = sim.histogram()
    Ho, Mo = ref.histogram()
    assert Ho.max() > 65_535
    if flips == 0:
        assert np.array_equal(H, Ho) and np.array_equal(M, Mo)
    else:
        assert np.abs(H.astype(np.int64) - Ho).sum() <= 2 * flips * ref.Q


def test_chunk_invariance(sg):
    """The launch shape does not change any particle's trajectory."""
    cfg = small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1, n_particles=30_000,
                    field0=2e6)
    states = []
    for chunk in (1024, 2048, 8192):
        sim = sg.Simulation(cfg, max_steps=60)
        sim.set_chunk(chunk)
        sim.init_particles()
        sim.step(60)
        states.append((sim.get_state(), sim.histogram(), sim.counters(), sim.moments()))
    for other in states[1:]:
        assert np.array_equal(other[0][0], states[0][0][0])
        assert np.array_equal(other[0][1], states[0][0][1])
        assert np.array_equal(other[1][0], states[0][1][0])
        assert other[2] == states[0][2]
        assert np.allclose(other[3]["E_vx"], states[0][3]["E_vx"], rtol=1e-12)


def test_repeatable(sg):
    cfg = small_cfg(n_particles=5000)
    out = []
    for _ in range(2):
        sim = sg.Simulation(cfg, max_steps=50)
        sim.init_particles()
        sim.step(50)
        out.append(sim.get_state()[0])
    assert np.array_equal(out[0], out[1])


# ------------------------------------------------- full-size, sampled
FULL = {
    "sg_gap_m5_q8_n1e6": dict(),
    "gnr_det_n1e4": dict(),
    "sg_gap_field_td4_q64_n4e6": dict(precision="fp64"),
    "sg_gap_m8_q12_n3e7": dict(precision="fp64"),
}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled(sg, orc, name):
    """At the workload's full size: the initial coefficients of sampled
    particles, and one step of sampled particles (every particle's step
    depends only on its own state and on H^n), against the oracle."""
    cfg = workload(name, **FULL[name])
    announce("full " + name, cfg)
    N = cfg["n_particles"]
    sim = sg.Simulation(cfg, max_steps=4)
    sim.init_particles()
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([rng.integers(0, N, 1500), [0, N - 1]]))
    ref = orc.OracleSim(dict(cfg, n_particles=1))
    ix, iy = ref.init_particles(idx)
    gx, gy = sim.get_state()
    err = rel_err(gx[:, idx], gy[:, idx], ix.T, iy.T)
    assert err.max() <= TOL, err.max()
    sim.step(3)
    bx, by = sim.get_state()
    H, M = sim.histogram()
    n_now = sim.step_count
    sim.step(1)
    ax, ay = sim.get_state()
    # number conservation: every node counts every in-grid particle once
    t = sim.tables()
    L, nk = cfg["lk_eV"], cfg["nk"]
    dk = 2 * L / nk
    for q in range(sim.Q):
        nx = t["psi"][q] @ bx
        ny = t["psi"][q] @ by
        r = np.floor((nx + L) / dk); l = np.floor((ny + L) / dk)
        inside = (r >= 0) & (r < nk) & (l >= 0) & (l < nk)
        assert int(H[q].sum()) == int(inside.sum())
        assert M[q] == H[q].max()
    # colliders of the last step plus a random sample
    drift = (1e6 * cfg["dt"]) * t["ehat"]
    moved = np.abs(ax - (bx - drift[:, None])).max(axis=0) + np.abs(ay - by).max(axis=0)
    coll = np.nonzero(moved > 1e-12)[0]
    sample = np.unique(np.concatenate([coll[:1500], rng.integers(0, N, 1500)]))
    assert coll.size > 0
    ref = orc.OracleSim(dict(cfg, n_particles=1))
    ref.set_histogram(H.reshape(sim.Q, -1), M)
    nxp, nyp, _ = ref.step_particles(sample, bx[:, sample].T, by[:, sample].T, n_now, cfg["dt"])
    err = rel_err(ax[:, sample], ay[:, sample], nxp.T, nyp.T)
    flips = int(np.count_nonzero(err > TOL))
    print(f"  sampled {sample.size} particles ({coll.size} colliders), flips {flips}", flush=True)
    assert flips <= 1


# ------------------------------------------------------------- FP32
def test_fp32_within_monte_carlo_error(sg):
    base = workload("sg_gap_m5_q8_n1e6", n_particles=200_000)
    res = {}
    for prec in ("fp64", "fp32"):
        sim = sg.Simulation(dict(base, precision=prec), max_steps=300)
        sim.init_particles()
        sim.step(300)
        res[prec] = sim.moments()
    a, b = res["fp64"], res["fp32"]
    for obs in ("E_vx", "Var_vx", "E_jx", "Var_jx", "E_energy"):
        se = np.maximum(a["SE_" + obs], 1e-300)
        dev = np.abs(a[obs] - b[obs]) / se
        print(f"  {obs}: max |fp32 - fp64| / SE = {dev[1:].max():.3f}", flush=True)
        assert dev[1:].max() < 3.0, obs


# ------------------------------------------------------- reconstruction
def test_reconstruct_f_parity(sg, orc):
    cfg = small_cfg(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1, n_particles=8000,
                    field0=2e6)
    ref = orc.OracleSim(cfg)
    ref.init()
    ref.run(2e-15, 40)
    kx, ky = ref.get_state()
    sim = sg.Simulation(cfg, max_steps=1)
    sim.set_state(kx, ky, step=40)
    nodes, modes = sim.reconstruct_f(256, 0.0, 2.56)
    onodes, omodes = ref.reconstruct_f(256, 0.0, 2.56)
    assert np.array_equal(np.rint(nodes * 8000 * 0.01), np.rint(onodes * 8000 * 0.01))
    assert np.allclose(modes, omodes, rtol=1e-12, atol=1e-12)
    zs = np.linspace(-1, 1, 7)
    f = sim.reconstruct_f_at(zs, 256, 0.0, 2.56)
    for k, z in enumerate(zs):
        fo = ref.reconstruct_f_at([z], 256, 0.0, 2.56)
        assert np.all(f[k] >= 0)
        assert abs(f[k].sum() * 0.01 - 1.0) < 1e-12
        assert np.abs(f[k] - fo).max() * 8000 * 0.01 <= 2.0   # at most a bin-edge flip


# ------------------------------------------------------------ errors
def test_error_paths(sg):
    cfg = small_cfg(n_particles=500)
    sim = sg.Simulation(cfg, max_steps=5)
    with pytest.raises(sg.SgpmError):
        sim.step(1)                          # before init
    sim.init_particles()
    with pytest.raises(sg.SgpmError):
        sim.step(1, dt=-1e-15)
    with pytest.raises(sg.SgpmError):
        sim.step(6)                          # beyond the record
    kx, ky = sim.get_state()
    kx[0, 3] = np.nan
    with pytest.raises(sg.SgpmError):
        sim.set_state(kx, ky)
    sim.step(5)
    assert sim.record_length() == 6
    with pytest.raises(sg.SgpmError):
        sg.Simulation(small_cfg(n_particles=0))


@pytest.mark.parametrize("kw", [
    dict(dim_z=1, degree=5, nodes_1d=8, gap_dim=0, gap_rel=0.1, n_particles=30_000, field0=2e6),
    dict(dim_z=2, degree=4, nodes_1d=8, gap_dim=0, gap0=0.3, gap_rel=0.15, field_dim=1,
         field0=1.5e6, field_rel=0.2, n_particles=6_000),
])
def test_moments_at_parity(sg, orc, kw):
    """Moments of the particle expansion at points z between the nodes, on a
    state taken from the oracle after 30 steps."""
    cfg = small_cfg(**kw)
    announce("moments_at", cfg)
    ref = orc.OracleSim(cfg, threads=8)
    ref.init()
    ref.run(cfg["dt"], 30)
    kx, ky = ref.get_state()
    sim = sg.Simulation(cfg)
    sim.set_state(kx, ky, step=30)
    rng = np.random.default_rng(5)
    dz = cfg["dim_z"]
    z = np.concatenate([rng.uniform(-1, 1, size=(19, dz)), -np.ones((1, dz)), np.ones((1, dz))])
    g = sim.moments_at(z)
    o = ref.moments_at(z)
    for k in ("V_x", "V_y"):
        assert np.allclose(g[k], o[k], rtol=1e-12, atol=1e-12 * np.abs(o[k]).max()), k
    assert np.allclose(g["energy"], o["energy"], rtol=1e-13)
    assert np.allclose(g["J_x"], o["J_x"], rtol=1e-9, atol=1e-9 * np.abs(o["J_x"]).max())


def test_occupancy_excess_parity_without_pauli(sg, orc):
    """A degenerate gas pushed hard with the Pauli acceptance off: many cells
    exceed the maximum occupation; the per-step excess matches the oracle."""
    cfg = small_cfg(n_particles=20_000, field0=3e7, nk=60, fermi_eV=0.6, pauli=0,
                    rate_scale=(20.0,) * 6)
    announce("occupancy excess", cfg)
    ref = orc.OracleSim(cfg, threads=8)
    ref.init()
    kx, ky = ref.get_state()
    sim = sg.Simulation(cfg, max_steps=30)
    sim.set_state(kx, ky, step=0)
    sim.step(30, cfg["dt"])
    ref.run(cfg["dt"], 30)
    gx, gy = sim.get_state()
    ox, oy = ref.get_state()
    assert int((rel_err(gx, gy, ox, oy) > TOL).sum()) == 0
    g = sim.occupancy_excess()
    o = np.asarray(ref.excess, dtype=np.uint32)
    assert g.max() > 0
    assert np.array_equal(g, o)
