"""GPU checks of the launch orchestration: graph replay, batched launches of
many instances, per-kernel profiling.

None of these may change a single bit of the results: the kernels of a
graph are the ones launched eagerly, and an instance stepped inside a batch
runs the same arithmetic on the same random streams as when it is stepped
alone.  So every comparison here is exact (np.array_equal), FP64 and FP32.
The batched instances are also checked against the CPU oracle directly.
"""
import numpy as np
import pytest

from workloads import batched_sweep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import paper_2404_19602_amd as sg
    return sg


def cfg_of(**kw):
    base = dict(dim_z=1, degree=5, nodes_1d=8, n_particles=20_001, gap_mode=0, gap_dim=0,
                gap0=0.2, gap_rel=0.1, field_dim=-1, field0=2e6, field_rel=0.0, fermi_eV=0.4,
                temp_K=300.0, alpha=0.1, nk=240, lk_eV=5.0, pauli=1, final_state=0,
                rate_scale=(1.0,) * 6, seed=777, instance=0, c_max=32, dt=2e-15,
                precision="fp64", steps=400)
    base.update(kw)
    return base


def snapshot(sim, inst=0):
    kx, ky = sim.get_state(inst)
    H, M = sim.histogram(inst)
    return dict(kx=kx, ky=ky, H=H, M=M, cnt=sim.counters(inst),
                rec=sim.moments(inst=inst)["per_node_vx"], agg=sim.moments(inst=inst)["E_jx"])


def assert_same(a, b, what=""):
    for k in a:
        if isinstance(a[k], dict):
            assert a[k] == b[k], (what, k)
        else:
            assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_matches_eager(sg, prec):
    """Graphs of 4 steps replayed many times, with host reads between the
    calls, against the same calls launched eagerly; every call compared."""
    cfg = cfg_of(precision=prec)
    print(f"\n[gpu case] graph replay {prec}", flush=True)
    eager = sg.Simulation(cfg)
    eager.set_graph(0)
    graph = sg.Simulation(cfg)
    graph.set_graph(4)
    for s in (eager, graph):
        s.init_particles()
    for n in (13, 20, 1, 17, 4):
        eager.step(n)
        graph.step(n)
        assert_same(snapshot(eager), snapshot(graph), f"after {n}")
    assert eager.step_count == graph.step_count == 55


def test_graph_survives_rechunk(sg):
    """A new launch shape drops the captured graphs; replays after it match."""
    cfg = cfg_of(n_particles=30_000)
    a = sg.Simulation(cfg)
    b = sg.Simulation(cfg)
    a.set_graph(0)
    b.set_graph(3)
    for s in (a, b):
        s.init_particles()
        s.set_chunk(1024)
        s.step(7)
    assert_same(snapshot(a), snapshot(b))


def mixed_instances():
    """Six instances in four shape groups, two groups with several members of
    different P and Q (P = 6, Q = 8 with P = 5, Q = 7)."""
    return [
        cfg_of(n_particles=30_000, instance=0),
        cfg_of(n_particles=12_345, field0=5e6, instance=1, seed=99),
        cfg_of(dim_z=0, degree=0, nodes_1d=1, gap_dim=-1, gap_rel=0.0, n_particles=5_000,
               instance=2),
        cfg_of(n_particles=20_000, precision="fp32", instance=3),
        cfg_of(degree=2, nodes_1d=5, n_particles=7_000, gap0=0.4, instance=4),
        cfg_of(degree=4, nodes_1d=7, n_particles=9_000, field0=1e5, instance=5),
    ]


def test_batched_matches_single_instances(sg):
    cfgs = mixed_instances()
    print("\n[gpu case] batched 6 instances", flush=True)
    batch = sg.Simulation(cfgs)
    batch.init_particles()
    batch.set_profiling(True)
    batch.step(25)
    t = batch.kernel_times()
    n_groups = t["stream"][1] // 25
    assert n_groups == 4, t
    assert t["finalize"][1] == t["collide"][1] == 25 * n_groups
    assert all(ms > 0 for ms, _ in t.values())
    batch.set_profiling(False)
    batch.step(15)
    for j, cfg in enumerate(cfgs):
        alone = sg.Simulation(cfg)
        alone.init_particles()
        alone.step(25)
        alone.step(15)
        assert_same(snapshot(batch, j), snapshot(alone), f"instance {j}")


def test_batched_instance_matches_oracle(sg):
    """An instance with P = 5, Q = 7 run inside a group whose kernels are
    padded for P <= 6, Q <= 8, against the oracle."""
    import oracle
    from test_gpu_parity import TOL, rel_err
    cfgs = mixed_instances()
    batch = sg.Simulation(cfgs)
    batch.init_particles()
    batch.step(30)
    j = 5
    gx, gy = batch.get_state(j)
    ref = oracle.OracleSim(cfgs[j])
    ref.init()
    ref.run(cfgs[j]["dt"], 30)
    ox, oy = ref.get_state()
    err = rel_err(gx, gy, ox, oy)
    flips = int((err > TOL).sum())
    assert flips <= 2, (flips, err.max())
    if flips == 0:
        H, M = batch.histogram(j)
        Ho, Mo = ref.histogram()
        assert np.array_equal(H, Ho) and np.array_equal(M, Mo)


def test_sweep_of_64_instances(sg):
    """The 64-instance sweep (three shape groups), scaled to 2e3-2e4
    particles, in graphs of 8 steps; sampled instances against runs alone."""
    cfgs = batched_sweep(n_min=2e3, n_max=2e4, steps=100)
    print(f"\n[gpu case] sweep of {len(cfgs)} instances, N={sum(c['n_particles'] for c in cfgs)}",
          flush=True)
    batch = sg.Simulation(cfgs)
    batch.set_graph(8)
    batch.init_particles()
    batch.step(20)
    for j in (0, 17, 40, 63):
        alone = sg.Simulation(cfgs[j])
        alone.init_particles()
        alone.step(20)
        assert_same(snapshot(batch, j), snapshot(alone), f"instance {j}")


@pytest.mark.parametrize("batched", [False, True])
def test_autotune_keeps_the_run(sg, batched):
    """The autotuner's trials leave state, step and counters as they were, and
    the run continued in the chosen shape matches an untuned run exactly."""
    cfgs = mixed_instances()[:3] if batched else cfg_of(n_particles=40_000)
    print(f"\n[gpu case] autotune batched={batched}", flush=True)
    tuned = sg.Simulation(cfgs)
    plain = sg.Simulation(cfgs)
    for s in (tuned, plain):
        s.init_particles()
        s.step(5)
    n = tuned.n_inst
    before = [snapshot(tuned, j) for j in range(n)]
    ms = tuned.autotune(trial_steps=4)
    assert ms > 0
    assert tuned.step_count == 5
    for j in range(n):
        after = snapshot(tuned, j)
        for k in ("kx", "ky", "H", "M", "cnt"):
            if isinstance(after[k], dict):
                assert after[k] == before[j][k], (j, k)
            else:
                assert np.array_equal(after[k], before[j][k]), (j, k)
        shape = tuned.launch_shape(j)
        assert shape["chunk"] % 1024 == 0 and shape["collider_workgroups"] in (512, 1024, 2048)
    for s in (tuned, plain):
        s.step(12)
    for j in range(n):
        a, b = snapshot(tuned, j), snapshot(plain, j)
        for k in ("kx", "ky", "H", "M", "cnt"):
            if isinstance(a[k], dict):
                assert a[k] == b[k], (j, k)
            else:
                assert np.array_equal(a[k], b[k]), (j, k)
        # the maximum occupation number of the initial datum is kept, and the
        # record continues through the tuning unless the chunk changed
        ea, eb = tuned.occupancy_excess(inst=j), plain.occupancy_excess(inst=j)
        assert np.array_equal(ea[-12:], eb[-12:]), j
        if tuned.launch_shape(j)["chunk"] == plain.launch_shape(j)["chunk"]:
            assert tuned.record_length(j) == plain.record_length(j) == 18
            ma, mb = tuned.moments(inst=j), plain.moments(inst=j)
            for k in ("E_vx", "E_energy", "SE_E_vx"):
                assert np.array_equal(ma[k], mb[k]), (j, k)
            assert np.array_equal(ea, eb), j


@pytest.mark.parametrize("kw", [
    dict(),                                                             # 6 modes, 8 nodes
    dict(precision="fp32", degree=8, nodes_1d=12, nk=256, field0=4e6),  # 9 modes, 12 nodes
    dict(dim_z=0, degree=0, nodes_1d=1, gap_dim=-1, gap_rel=0.0),        # one node
    dict(dim_z=2, degree=2, nodes_1d=3, field_dim=1, field_rel=0.2),     # 2-D, 9 nodes
    dict(pauli=0, final_state=1, field0=5e6, degree=3, nodes_1d=4),
    dict(splitting=1, field0=5e6, rate_scale=(3.0,) * 6),
])
def test_collider_lanes_match_node_groups(sg, kw):
    """The collider with a lane per candidate and the one with a group of lanes
    per candidate compute the same quantities by the same expressions: the
    runs are identical bit for bit."""
    cfg = cfg_of(n_particles=20_000, **kw)
    print(f"\n[gpu case] collider lanes vs node groups {kw}", flush=True)
    out = []
    for lanes in (True, False):
        sim = sg.Simulation(cfg, max_steps=60)
        sim.set_collider_lanes(lanes)
        sim.init_particles()
        sim.step(60)
        out.append(snapshot(sim))
    assert out[0]["cnt"]["collisions"] > 0
    assert_same(out[0], out[1], "lanes vs groups")


@pytest.mark.parametrize("prec,degree,nodes", [
    ("fp64", 8, 12), ("fp32", 8, 12),
    ("fp64", 5, 8),                     # four pairs: two kept by each lane of a lane pair
    ("fp64", 4, 7), ("fp32", 2, 5),     # odd node counts: three and two pairs, a middle node
])
def test_node_pairs_match_the_generic_stream_kernel(sg, prec, degree, nodes):
    """The mirror-pair stream kernel against the generic one: the node values
    differ only by rounding (even and odd modes summed apart), so histograms
    and event counters agree exactly and the trajectories to rounding.  The
    candidate count differs: the pair kernel bounds the energies after the
    drift by the bound before it plus the largest drift, a looser bound that
    hands more particles to the collider, whose exact test rejects them."""
    cfg = cfg_of(n_particles=50_000, precision=prec, degree=degree, nodes_1d=nodes, nk=256,
                 field0=4e6)
    print(f"\n[gpu case] node pairs vs generic {prec} degree {degree} nodes {nodes}", flush=True)
    out = []
    for on in (True, False):
        sim = sg.Simulation(cfg, max_steps=40)
        sim.set_node_pairs(on)
        assert sim.node_pairs() == on
        sim.init_particles()
        sim.step(40)
        out.append(snapshot(sim))
    a, b = out
    tol = 1e-9 if prec == "fp64" else 2e-4
    scale = np.maximum(np.sqrt((b["kx"] ** 2 + b["ky"] ** 2).sum(axis=0)), 1e-3)
    err = np.maximum(np.abs(a["kx"] - b["kx"]).max(axis=0), np.abs(a["ky"] - b["ky"]).max(axis=0))
    flips = int(np.count_nonzero(err / scale > tol))
    print(f"  flipped particles {flips}", flush=True)
    assert flips <= (2 if prec == "fp64" else 50)
    if flips == 0:
        assert np.array_equal(a["H"], b["H"]) and np.array_equal(a["M"], b["M"])
        ca, cb = dict(a["cnt"]), dict(b["cnt"])
        assert ca.pop("candidates") >= cb.pop("candidates")
        assert ca == cb
    assert np.allclose(a["rec"], b["rec"], rtol=1e-6 if prec == "fp32" else 1e-9)


@pytest.mark.parametrize("pairs", [True, False])
def test_stream_nontemporal_hints_change_nothing(sg, pairs):
    """The stream kernels' non-temporal state access (chosen for states larger
    than the last-level cache) gives the same run bit for bit as the ordinary
    one, in both stream kernels."""
    cfg = cfg_of(n_particles=60_000, degree=8, nodes_1d=12, nk=256, field0=4e6)
    print(f"\n[gpu case] stream non-temporal hints, pairs {pairs}", flush=True)
    out = []
    for nt in (True, False):
        sim = sg.Simulation(cfg, max_steps=40)
        sim.set_node_pairs(pairs)
        sim.set_stream_nontemporal(nt)
        assert sim.stream_nontemporal() == nt
        sim.init_particles()
        sim.step(40)
        out.append(snapshot(sim))
        sim.set_stream_nontemporal(None)
        assert sim.stream_nontemporal() is False       # 60k particles: far below 1 GiB
    assert out[0]["cnt"]["collisions"] > 0
    assert_same(out[0], out[1], "non-temporal vs ordinary")


def test_automatic_kernel_choice(sg):
    """The mirror-pair stream kernel is chosen by default only for shape
    groups of 2^22 particles or more; either choice can be forced."""
    small = sg.Simulation(cfg_of(degree=8, nodes_1d=12, nk=256), max_steps=4)
    assert small.node_pairs() is False
    small.init_particles()
    small.set_node_pairs(True)
    assert small.node_pairs() is True
    small.step(2)
    del small
    big = sg.Simulation(cfg_of(degree=8, nodes_1d=12, nk=256, n_particles=1 << 22), max_steps=4)
    assert big.node_pairs() is True
    big.init_particles()
    big.set_node_pairs(False)
    assert big.node_pairs() is False
    big.set_node_pairs(None)
    assert big.node_pairs() is True
    big.step(2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pair_kernel_workgroup_sizes_agree(sg, prec):
    """The two workgroup sizes of the mirror-pair stream kernel (the default
    and the other one the autotuner may pick) give the same particle states,
    histograms and counters; the FP64 moment sums, grouped by lane
    differently, agree to rounding."""
    cfg = cfg_of(n_particles=60_000, precision=prec, degree=8, nodes_1d=12, nk=256, field0=4e6)
    print(f"\n[gpu case] pair kernel workgroup sizes {prec}", flush=True)
    out, threads = [], []
    for alt in (0, 1):
        sim = sg.Simulation(cfg, max_steps=40)
        sim.set_node_pairs(True)
        sim.set_pair_block(alt)
        sim.init_particles()
        sim.step(40)
        threads.append(sim.stream_threads())
        out.append(snapshot(sim))
        out[-1]["m"] = sim.moments()
    print(f"  threads per workgroup {threads}", flush=True)
    assert threads[0] != threads[1] and set(threads) <= {512, 768, 1024}
    a, b = out
    for k in ("kx", "ky", "H", "M"):
        assert np.array_equal(a[k], b[k]), k
    assert a["cnt"] == b["cnt"]
    for k, tol in (("E_vx", 1e-12), ("E_energy", 1e-12), ("Var_vx", 1e-9)):
        assert np.allclose(a["m"][k], b["m"][k], rtol=tol, atol=0.0), k
