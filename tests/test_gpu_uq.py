"""GPU checks of the uncertainty-quantification drivers: Monte Carlo sampling
of z with deterministic runs (MC-MC) against the sG-PM and the oracle, the
truncation-order error with replayed random streams, percentile bands."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uq():
    from paper_2404_19602_amd import uq
    return uq


def gap_cfg(**kw):
    base = dict(dim_z=1, degree=5, nodes_1d=8, n_particles=20_000, gap_mode=0, gap_dim=0,
                gap0=0.2, gap_rel=0.3, field_dim=-1, field0=2e6, field_rel=0.0, fermi_eV=0.4,
                temp_K=300.0, alpha=0.1, nk=240, lk_eV=5.0, pauli=1, final_state=0,
                rate_scale=(1.0,) * 6, seed=31337, instance=0, c_max=32, dt=2e-15,
                precision="fp64", steps=300)
    base.update(kw)
    return base


def test_mc_sampling_agrees_with_sg(uq):
    """E_z[V_x](t) by 48 deterministic runs at sampled z and by the sG-PM
    (M = 8) agree within their combined Monte Carlo errors."""
    import paper_2404_19602_amd as sg
    cfg = gap_cfg(degree=8, nodes_1d=11, gap_rel=0.2)
    steps = 150
    print("\n[gpu case] MC-MC 48 samples vs sG", flush=True)
    mc = uq.mc_sampling(cfg, n_samples=48, steps=steps)
    sim = sg.Simulation(cfg, max_steps=steps)
    sim.init_particles()
    sim.step(steps)
    m = sim.moments()
    idx = np.array([40, 80, 120])
    diff = np.abs(m["E_vx"][idx] - mc["E_vx"][idx])
    se = np.sqrt(m["SE_E_vx"][idx] ** 2 + mc["SE_E_vx"][idx] ** 2)
    print(f"  sG {m['E_vx'][idx]}, MC-MC {mc['E_vx'][idx]}, |diff|/se {diff / se}", flush=True)
    assert np.all(diff < 4.0 * se)


def test_mc_sampling_runs_match_oracle(uq):
    """Two sample instances of the batched MC-MC run against oracle
    deterministic runs at the same z and instance word."""
    import oracle
    from test_gpu_parity import TOL, rel_err
    cfg = gap_cfg(n_particles=5_000)
    mc = uq.mc_sampling(cfg, n_samples=6, steps=40)
    for k in (1, 4):
        gx, gy = mc["sim"].get_state(k)
        ref = oracle.OracleSim(mc["cfgs"][k], threads=8)
        ref.init()
        ref.run(cfg["dt"], 40)
        ox, oy = ref.get_state()
        err = rel_err(gx, gy, ox, oy)
        assert int((err > TOL).sum()) <= 2, (k, err.max())


def test_sg_error_decreases_with_order(uq):
    """With the same random streams for every order, the L2(z) error of the
    mean energy against M = 10 falls as the order grows: spectrally for the
    initial datum (smooth in z), then more slowly once collisions, which act
    on the nodes through indicator functions of z, have occurred."""
    cfg = gap_cfg(n_particles=10_000)
    r = uq.sg_error(cfg, orders=[0, 1, 2, 4], m_ref=10, times_steps=[0, 25, 50])
    print(f"\n  sG error (rows: steps {r['steps']}; cols: M {r['orders']}):\n{r['error']}", flush=True)
    e = r["error"]
    assert e[0, 3] < 1e-3 * e[0, 0]
    assert np.all(e[1:, 0] > e[1:, 1]) and np.all(e[1:, 1] > e[1:, 2]) and np.all(e[1:, 2] > e[1:, 3])


def test_percentile_bands(uq):
    import paper_2404_19602_amd as sg
    sim = sg.Simulation(gap_cfg(n_particles=8_000))
    sim.init_particles()
    sim.step(20)
    b = uq.percentile_bands(sim, percentiles=(10, 50, 90), n_z=128)
    for k in ("energy", "V_x"):
        lo, med, hi = b[k + "_bands"]
        assert lo < med < hi and lo < b[k + "_mean"] < hi, k
    flat = sg.Simulation(gap_cfg(n_particles=8_000, gap_rel=0.0))
    flat.init_particles()
    flat.step(20)
    b = uq.percentile_bands(flat, n_z=32)
    lo, hi = b["energy_bands"]
    assert hi - lo <= 1e-10 * abs(b["energy_mean"])


def test_error_versus_cost(uq):
    """Sec. 5 Test 4 at reduced size (uncertain width of Test 3, N = 2e4,
    0.25 ps, reference M = 12 with 4e5 particles): every estimate of
    E_z[V_x] is consistent with the reference within its Monte Carlo error
    (particle noise of both runs, plus for MC-MC the sampling error over z),
    and the cost columns follow the paper's cost model (M1^2, M2)."""
    from test_gpu_accuracy import _test3_cfg
    cfg = _test3_cfg("width", 20_000)
    print("\n[gpu case] Test 4 error vs cost, N = 2e4, reference 4e5 particles M = 12", flush=True)
    r = uq.error_versus_cost(cfg, n=20_000, steps=100, sg_orders=[0, 1, 2, 4, 6],
                             mc_samples=[1, 2, 4, 8, 16, 32], n_ref=400_000, m_ref=12)
    se_ref = r["ref_SE"]
    for row in r["mc_sg"]:
        print(f"  MC-sG M1={row['M1']}: cost {row['cost_per_particle']}, error {row['error']:.3e}, "
              f"SE {row['SE']:.2e}, {row['ms_per_step']:.3f} ms/step", flush=True)
        assert row["cost_per_particle"] == row["M1"] ** 2
        if row["M1"] >= 4:
            assert row["error"] < 4.0 * np.hypot(row["SE"], se_ref), row
    var_z = r["std_z_vx_samples"] ** 2
    for row in r["mc_mc"]:
        print(f"  MC-MC M2={row['M2']}: error {row['error']:.3e}, SE(z) {row['SE_samples']:.2e}",
              flush=True)
        assert row["cost_per_particle"] == row["M2"]
        bound = 4.0 * np.sqrt(var_z / row["M2"] + row["SE_particles"] ** 2 + se_ref ** 2)
        assert row["error"] < bound, row
    assert r["ref_ms_per_step"] > 0 and r["mc_ms_per_step_all_samples"] > 0


def test_percentile_bands_match_oracle(uq):
    """The bands of a GPU run equal the same percentiles of the oracle's
    particle expansion evaluated at the same z after the same steps (a run
    whose trajectories agree with the oracle's to rounding)."""
    import oracle
    import paper_2404_19602_amd as sg
    cfg = gap_cfg(n_particles=3_000)
    steps = 20
    print("\n[gpu case] percentile bands vs oracle, N = 3000, 20 steps", flush=True)
    sim = sg.Simulation(cfg, max_steps=steps)
    sim.init_particles()
    sim.step(steps)
    pct = (10.0, 50.0, 80.0, 90.0)
    b = uq.percentile_bands(sim, percentiles=pct, n_z=64)
    ref = oracle.OracleSim(cfg, threads=8)
    ref.init()
    ref.run(cfg["dt"], steps)
    m = ref.moments_at(b["z"][:, 0])
    for k in ("energy", "V_x"):
        want = np.percentile(m[k], pct)
        scale = np.max(np.abs(m[k]))
        err = np.max(np.abs(b[k + "_bands"] - want)) / scale
        print(f"  {k}: bands {b[k + '_bands']}, oracle {want}, max rel err {err:.1e}", flush=True)
        assert err < 1e-9, k
        assert abs(b[k + "_mean"] - float(np.mean(m[k]))) < 1e-9 * scale
