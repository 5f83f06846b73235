"""GPU side of the ladder initialisation (Initialization): single-ligand
sweeps and state replacement that bpmf_initialize_ladder runs on, random
placements in the site against the oracle, and bpmf_initialize_ladder end
to end -- every selection it made replayed with the oracle's formula, the
ladder's states equal to the schedule at their alpha, the last state's
spreads equal to the oracle's on the samples it left, state 0's spreads
equal to the oracle's on
the oracle's own placements and energies."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, make_context, print_case, require_gpu, torch
from oracle import protocol as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _same_ligand_state(ca, la, cb, lb):
    a, b = ca.get_replicas(la), cb.get_replicas(lb)
    for key in ("x", "state_of_replica", "comps", "counter"):
        assert np.array_equal(a[key], b[key]), key
    xa, cpa = ca.get_samples(la)
    xb, cpb = cb.get_samples(lb)
    assert np.array_equal(xa, xb) and np.array_equal(cpa, cpb)
    sa, sb = ca.get_stats(la), cb.get_stats(lb)
    for key in ("hmc_acc", "hmc_try", "ex_acc", "ex_try"):
        assert np.array_equal(sa[key], sb[key]), key


@pytest.mark.parametrize("scheme,chunk", [(0, 0), (0, 8), (1, 8)])
def test_single_ligand_sweeps_equal_their_share_of_full_sweeps(scheme, chunk):
    print_case("single-ligand sweeps", scheme, chunk)
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    ctx_a, (a0, a1) = make_context(g, [lig, lig], seed=5, capacity=20)
    ctx_b, (b0, b1) = make_context(g, [lig, lig], seed=5, capacity=20)
    for c in (ctx_a, ctx_b):
        c.set_graph(chunk)
    before = ctx_a.get_replicas(a0)
    kw = dict(exchange_every=1, exchange_scheme=scheme, max_sep=3,
              sample_every=2)
    ctx_a.hmc_sweep_ligand(a1, 24, 10, **kw)
    ctx_b.hmc_sweep(24, 10, **kw)
    _same_ligand_state(ctx_a, a1, ctx_b, b1)
    after = ctx_a.get_replicas(a0)
    for key in ("x", "state_of_replica", "comps", "counter"):
        assert np.array_equal(before[key], after[key]), key
    assert ctx_a.get_samples(a0)[0].shape[0] == 0
    assert ctx_a.get_stats(a0)["hmc_try"].sum() == 0
    ctx_a.close()
    ctx_b.close()


def test_replaced_states_equal_states_set_up_from_the_start():
    print_case("set_states")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    K = lig.n_states
    rng = np.random.default_rng(3)
    T2 = rng.uniform(300, 600, size=K)
    w2 = rng.uniform(0, 1, size=(K, 3))
    dt2 = rng.uniform(0.5, 1.2, size=K)
    ctx_a, (la,) = make_context(g, [lig], seed=9, capacity=10)
    ctx_a.set_states(la, T2, w2, dt2)
    lig2 = dataclasses.replace(lig, T=T2, w=w2, dt=dt2)
    ctx_b, (lb,) = make_context(g, [lig2], seed=9, capacity=10)
    for c in (ctx_a, ctx_b):
        c.hmc_sweep(12, 10, exchange_every=1, sample_every=3)
    _same_ligand_state(ctx_a, la, ctx_b, lb)
    info = ctx_a.ligand_info(la)
    assert info == dict(n_atoms=lig.n_atoms, n_states=K, n_channels=3,
                        sample_capacity=10)
    import paper_1507_03703_amd as pkg
    with pytest.raises(pkg.BPMFError):
        ctx_a.set_states(la, np.zeros(K), w2, dt2)
    ctx_a.close()
    ctx_b.close()


def test_graphs_captured_before_a_state_change_replay_the_new_states():
    """Sweep graphs read the state parameters from device memory: replays
    of a graph captured before bpmf_set_states equal plain launches after
    it, bit for bit."""
    print_case("set_states then graph replay")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    K = lig.n_states
    rng = np.random.default_rng(8)
    T2 = rng.uniform(300, 600, size=K)
    w2 = rng.uniform(0, 1, size=(K, 3))
    dt2 = rng.uniform(0.5, 1.2, size=K)
    runs = []
    for chunk in (0, 8):
        ctx, (lid,) = make_context(g, [lig], seed=21, capacity=20)
        ctx.set_graph(chunk)
        ctx.hmc_sweep(16, 10, exchange_every=1, sample_every=2)
        ctx.set_states(lid, T2, w2, dt2)
        ctx.hmc_sweep(16, 10, exchange_every=1, sample_every=2)
        runs.append((ctx.get_replicas(lid), ctx.get_samples(lid),
                     ctx.get_stats(lid)))
        ctx.close()
    (ra, sa, ta), (rb, sb, tb) = runs
    for key in ("x", "state_of_replica", "comps", "counter"):
        assert np.array_equal(ra[key], rb[key]), key
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    for key in ("hmc_acc", "hmc_try", "ex_acc", "ex_try"):
        assert np.array_equal(ta[key], tb[key]), key


def test_single_ligand_sweeps_run_only_that_ligands_moves():
    """External moves inside single-ligand sweep calls touch only that
    ligand; its result equals the same units run over every ligand."""
    print_case("single-ligand sweeps with external moves")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    ctx_a, (a0, a1) = make_context(g, [lig, lig], seed=3)
    ctx_b, (b0, b1) = make_context(g, [lig, lig], seed=3)
    kw = dict(exchange_every=1, external_moves=4, external_k_max=3)
    before = ctx_a.get_replicas(a0)
    ctx_a.hmc_sweep_ligand(a1, 6, 10, **kw)
    ctx_b.hmc_sweep(6, 10, **kw)
    _same_ligand_state(ctx_a, a1, ctx_b, b1)
    sa, sb = ctx_a.get_external_stats(a1), ctx_b.get_external_stats(b1)
    assert np.array_equal(sa["tries"], sb["tries"]) and sa["tries"].sum() > 0
    assert ctx_a.get_external_stats(a0)["tries"].sum() == 0
    after = ctx_a.get_replicas(a0)
    assert np.array_equal(before["x"], after["x"])
    ctx_a.close()
    ctx_b.close()


def test_placements_match_oracle():
    print_case("placements")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    ctx, (lid,) = make_context(g, [lig], seed=77)
    confs = np.ascontiguousarray(lig.x0[:3], np.float32)
    out = ctx.place_poses(lid, dev(confs, torch.float32), 37, 6)
    got = out.cpu().numpy().astype(np.float64)
    ref = P.placements(confs.astype(np.float64),
                       lig.mass.astype(np.float32).astype(np.float64),
                       np.asarray(lig.site_center, np.float32),
                       np.float32(lig.d0), 37, 6, seed=77, lig=lid)
    assert got.shape == ref.shape == (3 * 37 * 6, lig.n_atoms, 3)
    assert np.abs(got - ref).max() < 2e-5
    part = ctx.place_poses(lid, dev(confs, torch.float32), 37, 6, first=101,
                           count=55)
    assert np.array_equal(part.cpu().numpy(), out[101:156].cpu().numpy())
    import paper_1507_03703_amd as pkg
    with pytest.raises(pkg.BPMFError):
        ctx.place_poses(lid, dev(confs, torch.float32), 37, 6, first=600,
                        count=100)
    ctx.close()


def _init_system(n_seeds, capacity):
    system = synth.make_system(1)
    g, (lig,) = synth.add_soft_grids(system.grid, system.ligands[:1])
    init = dataclasses.replace(
        lig, T=np.full(n_seeds, 600.0), w=np.zeros((n_seeds, 5)),
        dt=np.ones(n_seeds),
        x0=np.repeat(lig.x0[:1], n_seeds, axis=0).astype(np.float32))
    return g, init


def test_initialize_ladder_end_to_end():
    print_case("initialize ladder")
    n_seeds, n_trials = 16, 60
    g, init = _init_system(n_seeds, n_trials)
    ctx, (lid,) = make_context(g, [init], seed=31, capacity=n_trials)
    TH, TT = 600.0, 300.0
    res = ctx.initialize_ladder(lid, P.SOFT, TH, TT, speed=0.2,
                                n_trials=n_trials, n_leapfrog=10,
                                dt_start=1.0, dt_min=0.25, max_dt_rounds=6,
                                max_selections=4, n_conf=4, n_com=40,
                                n_orient=8, max_states=400)
    K = res["n_states"]
    print("states", K, "selections", res["n_selections"], "runs",
          res["n_runs"], "removed", res["n_removed"], flush=True)
    assert res["reached_target"]
    al = res["alpha"]
    assert al[0] == 0.0 and al[-1] == 1.0 and np.all(np.diff(al) > 0)
    for k in range(K):
        T, w = P.state_of(al[k], P.SOFT, 5, TH, TT)
        assert res["T"][k] == pytest.approx(T, rel=1e-15)
        assert np.allclose(res["w"][k], w, rtol=1e-14, atol=0)
        assert res["dt"][k] >= 0.25
    # every selection replayed with the oracle's parameter selection
    tr = res["trace"]
    assert len(tr) == res["n_selections"]
    for r in tr:
        a_new = P.next_alpha(r[0], r[1], r[2], r[3], P.SOFT, r[4], TH, TT)
        assert r[5] == pytest.approx(a_new, rel=1e-12, abs=1e-15)
        if r[9] == 1:
            assert r[8] < P.P_LOW
    for prev, cur in zip(tr[:-1], tr[1:]):
        if prev[9] == 1:      # a repeat: same start, speed x 4/5
            assert cur[0] == prev[0]
            assert cur[4] == pytest.approx(prev[4] * P.SPEED_FACTOR,
                                           rel=1e-14)
    kept = tr[tr[:, 9] != 1]
    ladder = [0.0]
    for r in kept:           # outcome 2 replaces the state it came from
        if r[9] == 2:
            ladder[-1] = r[5]
        else:
            ladder.append(r[5])
    assert np.array_equal(np.array(ladder), al)
    assert int((tr[:, 9] == 2).sum()) == res["n_removed"]
    # p_acc of accepted states is >= 0.4 unless the selections ran out
    low = (kept[:, 8] < P.P_LOW).sum()
    assert low <= max(1, len(kept) // 10)
    # the last state's spreads from the samples left in the seed ligand
    xs, comps = ctx.get_samples(lid)
    comps = comps.reshape(-1, 6)
    so = P.state_sigmas(comps, al[-1], P.SOFT, TH, TT)
    assert np.allclose(res["sigma"][-1], so, rtol=1e-12)
    assert np.array_equal(res["x"][-1], ctx.get_replicas(lid)["x"])
    # state 0's spreads from the oracle's placements of the same
    # configurations, with the oracle's energies
    confs = res["x"][0][:4].astype(np.float64)
    ol = oracle.OLigand(init)
    og = oracle.OGrid(g)
    poses = P.placements(confs, init.mass.astype(np.float32).astype(np.float64),
                         np.asarray(init.site_center, np.float32),
                         np.float32(init.d0), 40, 8, seed=31, lig=lid)
    comps0 = oracle.components(og, ol, poses)[0]
    s0 = P.state_sigmas(comps0, 0.0, P.SOFT, TH, TT)
    assert np.allclose(res["sigma"][0], s0, rtol=2e-3), (res["sigma"][0], s0)
    ctx.close()


def test_initialize_ladder_linear_schedule_and_state_cap():
    """The linear schedule on three channels with state 0's own samples (no
    placements): selections replayed with the oracle, the ladder equal to
    the schedule; with room for three states the ladder stops short of
    alpha = 1 and says so."""
    print_case("initialize ladder linear")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    n_seeds = 8
    init = dataclasses.replace(
        lig, T=np.full(n_seeds, 600.0), w=np.zeros((n_seeds, 3)),
        dt=np.ones(n_seeds),
        x0=np.repeat(lig.x0[:1], n_seeds, axis=0).astype(np.float32))
    TH, TT = 600.0, 300.0
    for cap in (400, 3):
        ctx, (lid,) = make_context(g, [init], seed=13, capacity=40)
        res = ctx.initialize_ladder(lid, P.LINEAR, TH, TT, speed=0.5,
                                    n_trials=40, n_leapfrog=10,
                                    dt_start=1.0, dt_min=0.25,
                                    max_dt_rounds=4, max_selections=3,
                                    max_states=cap)
        al = res["alpha"]
        print("cap", cap, "states", res["n_states"], flush=True)
        assert al[0] == 0.0 and np.all(np.diff(al) > 0)
        assert res["reached_target"] == (al[-1] == 1.0)
        if cap == 3:
            assert res["n_states"] <= 3
        else:
            assert res["reached_target"]
        for k in range(res["n_states"]):
            T, w = P.state_of(al[k], P.LINEAR, 3, TH, TT)
            assert res["T"][k] == pytest.approx(T, rel=1e-15)
            assert np.allclose(res["w"][k], w, rtol=1e-15, atol=0)
        for r in res["trace"]:
            a_new = P.next_alpha(r[0], r[1], r[2], r[3], P.LINEAR, r[4], TH,
                                 TT)
            assert r[5] == pytest.approx(a_new, rel=1e-12, abs=1e-15)
        # state 0's spreads from its own recorded samples: the sample set
        # of a state is its last run, so only the last state's is left; for
        # a ladder of one selection the trace's first record carries state
        # 0's spreads
        assert np.allclose(res["trace"][0][1:4], res["sigma"][0], rtol=0)
        ctx.close()


def test_initialize_ladder_argument_errors():
    print_case("initialize ladder errors")
    import paper_1507_03703_amd as pkg
    g, init = _init_system(8, 10)
    ctx, (lid,) = make_context(g, [init], seed=3, capacity=10)
    bad = [dict(n_trials=11), dict(kind=P.LINEAR + 7), dict(n_conf=9,
                                                          n_com=2, n_orient=2),
           dict(max_states=1), dict(dt_min=0.0), dict(speed=-1.0)]
    for kw in bad:
        args = dict(kind=P.SOFT, T_hot=600.0, T_cold=300.0, n_trials=10)
        args.update(kw)
        kind = args.pop("kind")
        with pytest.raises(pkg.BPMFError):
            ctx.initialize_ladder(lid, kind, **args)
    ctx.close()
