"""GPU parity of the learned pose proposal against the FP64 oracle: bf16
MFMA forward pass, backward pass (gradients), pose features, and the
independence Metropolis-Hastings pose move; plus training on poses sampled
by plain HMC.

Tolerances: network outputs and gradients relative L2 <= 2e-2 and cosine
>= 0.999 (bf16 operands, fp32 accumulation, against float64 with the same
bf16-valued weights); poses 1e-4; the pose move's ln alpha within 1e-3 of
the oracle (2e-2 + 1e-4 |ln alpha|: float32 energies and rotations) given
the GPU's network outputs, identical decisions where the margin
|ln u - ln alpha| exceeds 5e-2.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, make_context, print_case, require_gpu, torch
from oracle import learned as Lr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def bf16(a):
    """Round float64/float32 values to bfloat16 (nearest even)."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def flat(p):
    return np.concatenate([p[k].reshape(-1) for k in
                           ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(
                               np.float32)


def unflat(v):
    shapes = [("W1", (16, 256)), ("b1", (256,)), ("W2", (256, 256)),
              ("b2", (256,)), ("W3", (256, 104)), ("b3", (104,))]
    out, o = {}, 0
    for k, s in shapes:
        n = int(np.prod(s))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(s)
        o += n
    return out


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def cosine(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def _ligand(which):
    """The 24-atom config-1 system, or a ligand of 90 or 100 atoms (two
    wavefronts of atoms, as the large batched workload's) on its grid."""
    system = synth.make_system(1)
    if which == "c1":
        return system, system.ligands[0]
    n = int(which[4:])
    lig = synth.make_ligand(np.random.default_rng(n), n, 8, box=9.0)
    return system, lig


def _setup(seed=0, which="c1"):
    rng = np.random.default_rng(seed)
    system, lig = _ligand(which)
    p = Lr.init_weights(rng)
    for k in p:
        p[k] = p[k] + 0.05 * rng.normal(size=p[k].shape)
    ctx, (lid,) = make_context(system.grid, [lig], seed=system.seed)
    cond = lig.tors[lig.cond_tors]
    ctx.proposal_setup(lid, lig.frame_atoms, cond, flat(p))
    return rng, system, lig, p, ctx, lid, cond


def test_forward_matches_oracle():
    print_case("mlp forward")
    rng, system, lig, p, ctx, lid, _ = _setup(1)
    B = 300
    f = rng.uniform(-1, 1, (B, 16)).astype(np.float32)
    out = ctx.proposal_forward(lid, dev(f, torch.float32)).cpu().numpy()
    pb = {k: bf16(v) for k, v in p.items()}
    ref, _ = Lr.forward(pb, f.astype(np.float64))
    assert rel_l2(out, ref) < 2e-2, rel_l2(out, ref)
    assert cosine(out.ravel(), ref.ravel()) > 0.999
    ctx.close()


def test_gradients_match_oracle():
    print_case("mlp gradients")
    rng, system, lig, p, ctx, lid, _ = _setup(2)
    B = 512
    f = rng.uniform(-1, 1, (B, 16)).astype(np.float32)
    t = rng.normal(scale=1.0, size=(B, 3))
    w = rng.normal(scale=0.8, size=(B, 3))
    poses = np.concatenate([t, w], 1).astype(np.float32)
    g, loss = ctx.proposal_grad(lid, dev(f, torch.float32),
                                dev(poses, torch.float32))
    g = unflat(g.cpu().numpy())
    pb = {k: bf16(v) for k, v in p.items()}
    loss64, g64, _ = Lr.nll_grad(pb, f.astype(np.float64),
                                 poses[:, :3].astype(np.float64),
                                 poses[:, 3:].astype(np.float64))
    assert abs(loss - loss64) < 1e-2 * abs(loss64)
    for k in g64:
        a, b = g[k].ravel(), g64[k].ravel()
        assert rel_l2(a, b) < 2e-2, (k, rel_l2(a, b))
        assert cosine(a, b) > 0.999, (k, cosine(a, b))
    ctx.close()


@pytest.mark.parametrize("which", ["c1", "wide90", "wide100"])
def test_pose_features_match_oracle(which):
    print_case("pose features", which)
    rng, system, lig, p, ctx, lid, cond = _setup(3, which)
    assert len(cond) == 8 or which == "c1"
    from scipy.spatial.transform import Rotation
    N = 200
    xs = []
    for i in range(N):
        Q = Rotation.random(random_state=i).as_matrix()
        x = lig.x0[0].astype(np.float64) @ Q.T + rng.normal(scale=1.5,
                                                             size=3)
        x += rng.normal(scale=0.1, size=x.shape)
        xs.append(x)
    xs = np.array(xs, np.float32)
    f, po = ctx.pose_features(lid, dev(xs, torch.float32))
    f, po = f.cpu().numpy(), po.cpu().numpy()
    for i in range(N):
        x = xs[i].astype(np.float64)
        t, R, _ = Lr.pose(x, lig.mass, lig.frame_atoms, lig.site_center)
        assert np.allclose(po[i, :3], t, atol=1e-4)
        # compare rotations (the vector is ambiguous at |omega| = pi)
        assert np.allclose(Lr.rodrigues(po[i, 3:]), R, atol=2e-4)
        assert np.allclose(f[i], Lr.features(x, cond), atol=2e-5)
    ctx.close()


def _check_pose_moves(ctx, og, lig, lid, seed, rounds, sweeps=2):
    """`rounds` times: a few sweeps of every ligand, then one pose move of
    every ligand with a proposal (ligand -1), checked replica by replica on
    `lig` against the oracle's move given the GPU's network outputs.
    Returns the number of replicas whose decision was compared."""
    ol = oracle.OLigand(lig)
    checked = 0
    for rnd in range(rounds):
        ctx.hmc_sweep(sweeps, 10, exchange_every=1)
        st = ctx.get_replicas(lid)
        x = st["x"]
        f, _ = ctx.pose_features(lid, dev(x, torch.float32))
        out = ctx.proposal_forward(lid, f).cpu().numpy()
        ctx.pose_move(-1, 1)
        st2 = ctx.get_replicas(lid)
        la = ctx.get_pose_stats(lid)["last_ln_alpha"]
        mp = Lr.mixture(out)
        for r in range(lig.n_states):
            k = st["state_of_replica"][r]
            beta = 1.0 / (oracle.R_GAS * lig.T[k])

            def energy(xx, k=k):
                t, _, _ = oracle.energy(og, ol, lig.w[k], xx, forces=False)
                return t[:4].sum() + lig.w[k] @ t[4:]
            row = {kk: v[r] for kk, v in mp.items()}
            cnt = st["counter"]
            u0 = oracle.uniform(seed, 0, lid, r, cnt, 4)
            z1 = oracle.normals3(seed, 1, lid, r, cnt, 4)
            z2 = oracle.normals3(seed, 2, lid, r, cnt, 4)
            ua = oracle.uniform(seed, 3, lid, r, cnt, 4)
            xn, acc, ln_a = Lr.pose_move(x[r].astype(np.float64), lig.mass,
                                         lig.frame_atoms, lig.site_center,
                                         row, energy, beta, u0, z1, z2, ua)
            # float32 energies (|dE| <= 1e-5 of the magnitude sum, a few
            # 1e-3 kT here) and float32 rotations enter ln alpha
            assert abs(la[r] - ln_a) < 2e-2 + 1e-4 * abs(ln_a), \
                (lid, r, la[r], ln_a)
            if abs(math.log(ua) - ln_a) > 5e-2:
                moved = not np.array_equal(st2["x"][r], x[r])
                assert moved == acc, (lid, rnd, r)
                if acc:
                    assert np.max(np.abs(st2["x"][r] - xn)) < 1e-4
                checked += 1
    return checked


@pytest.mark.parametrize("which", ["c1", "wide90", "wide100"])
def test_pose_move_matches_oracle(which):
    """One wavefront of atoms (24) and two (90, 100: the pose move's
    two-wavefront centre of mass and evaluation)."""
    print_case("pose move", which)
    rng, system, lig, p, ctx, lid, cond = _setup(4, which)
    og = oracle.OGrid(system.grid)
    checked = _check_pose_moves(ctx, og, lig, lid, system.seed, 4)
    assert checked >= 16
    ctx.close()


@pytest.mark.parametrize("all_props", [True, False])
def test_pose_moves_of_several_ligands_in_one_call(all_props):
    """Three ligands of 24, 57 and 96 atoms, each with its own proposal (or
    the 57-atom one without: units then close with their own finish and
    begin launches), in one context: every pose move call moves all of
    them, each checked against the oracle, and sweep calls with
    pose_move_every = 5 (graph and plain launches) equal the host loop of
    five-sweep calls and pose moves bit for bit."""
    print_case("pose moves, three ligands", all_props)
    system = synth.make_system(1)
    rng = np.random.default_rng(9)
    ligs = [system.ligands[0], synth.make_ligand(rng, 57, 8, box=8.0),
            synth.make_ligand(rng, 96, 8, box=9.0)]
    params = []
    for q, lig in enumerate(ligs):
        p = Lr.init_weights(np.random.default_rng(30 + q))
        for k in p:
            p[k] = p[k] + 0.05 * rng.normal(size=p[k].shape)
        params.append(flat(p))
    has = [True, all_props, True]
    ctx, ids = make_context(system.grid, ligs, seed=system.seed)
    for lid, lig, p, h in zip(ids, ligs, params, has):
        if h:
            ctx.proposal_setup(lid, lig.frame_atoms, lig.tors[lig.cond_tors],
                               p)
    og = oracle.OGrid(system.grid)
    if all_props:
        for lid, lig in zip(ids, ligs):
            checked = _check_pose_moves(ctx, og, lig, lid, system.seed, 2,
                                        sweeps=1)
            assert checked >= 6, (lid, checked)
    ctx.close()
    runs = []
    for mode in ("host", "graph", "plain"):
        ctx, ids = make_context(system.grid, ligs, seed=13, capacity=10)
        for lid, lig, p, h in zip(ids, ligs, params, has):
            if h:
                ctx.proposal_setup(lid, lig.frame_atoms,
                                   lig.tors[lig.cond_tors], p)
        if mode == "plain":
            ctx.set_graph(0)
        if mode == "graph":
            ctx.set_graph(15)  # three units per graph, one left over
        if mode == "host":
            for _ in range(4):
                ctx.hmc_sweep(5, 10, exchange_every=1, sample_every=3)
                ctx.pose_move(-1, 1)
            ctx.hmc_sweep(3, 10, exchange_every=1, sample_every=3)
        else:
            ctx.hmc_sweep(23, 10, exchange_every=1, sample_every=3,
                          pose_move_every=5)
        runs.append([(ctx.get_replicas(i), ctx.get_samples(i),
                      ctx.get_pose_stats(i) if h else None, ctx.get_stats(i))
                     for i, h in zip(ids, has)])
        ctx.close()
    for per in runs[1:]:
        for (st, (xs, cs), ps, ss), (st0, (xs0, cs0), ps0, ss0), lig in zip(
                per, runs[0], ligs):
            for key in ("x", "state_of_replica", "comps", "counter"):
                assert np.array_equal(st[key], st0[key]), key
            assert np.array_equal(xs, xs0) and np.array_equal(cs, cs0)
            for key in ss0:
                assert np.array_equal(ss[key], ss0[key]), key
            if ps0 is None:
                continue
            assert ps0["tries"].sum() == 4 * lig.n_states
            assert np.array_equal(ps["acc"], ps0["acc"])
            assert np.array_equal(ps["tries"], ps0["tries"])


def test_training_on_sampled_poses_improves_the_proposal():
    print_case("training")
    system = synth.make_system(1)
    lig = system.ligands[0]
    # 32 independent chains at the coupled end state (lambda = 1, 300 K)
    import copy
    l1 = copy.deepcopy(lig)
    K = 32
    l1.T = np.full(K, lig.T[-1])
    l1.w = np.repeat(lig.w[-1:], K, axis=0)
    l1.dt = np.full(K, 1.0)
    l1.x0 = np.repeat(lig.x0[:1], K, axis=0)
    ctx, (lid,) = make_context(system.grid, [l1], seed=11, capacity=200)
    rng = np.random.default_rng(0)
    p = Lr.init_weights(rng)
    ctx.proposal_setup(lid, l1.frame_atoms, l1.tors[l1.cond_tors], flat(p))
    ctx.hmc_sweep(200, 10, exchange_every=0)
    ctx.hmc_sweep(400, 10, exchange_every=0, sample_every=2)
    xs, _ = ctx.get_samples(lid)
    xs = dev(xs.reshape(-1, l1.n_atoms, 3), torch.float32)
    f, po = ctx.pose_features(lid, xs)
    # untrained proposal
    ctx.pose_move(lid, 20)
    before = ctx.get_pose_stats(lid)
    losses = ctx.proposal_train(lid, f, po, batch=512, steps=400, lr=2e-3,
                                losses=True)
    assert losses[-20:].mean() < losses[:20].mean() - 1.0
    ctx.pose_move(lid, 20)
    after = ctx.get_pose_stats(lid)
    acc0 = before["acc"].sum() / before["tries"].sum()
    acc1 = (after["acc"].sum() - before["acc"].sum()) / \
        (after["tries"].sum() - before["tries"].sum())
    assert acc1 > acc0
    ctx.close()


def test_pose_moves_inside_sweep_calls_match_host_loop():
    """hmc_sweep(pose_move_every=5) -- units of five sweeps and a pose move,
    replayed from a captured graph or launched plainly -- gives the same bits
    as the host alternating five-sweep calls and pose_move calls."""
    print_case("pose_move_every")
    system = synth.make_system(1)
    lig = system.ligands[0]
    p = flat(Lr.init_weights(np.random.default_rng(4)))
    runs = []
    for mode in ("host", "graph", "plain"):
        ctx, (lid,) = make_context(system.grid, [lig], seed=13, capacity=10)
        ctx.proposal_setup(lid, lig.frame_atoms, lig.tors[lig.cond_tors], p)
        if mode == "plain":
            ctx.set_graph(0)
        if mode == "graph":
            ctx.set_graph(15)  # three units per graph
        if mode == "host":
            for _ in range(6):
                ctx.hmc_sweep(5, 10, exchange_every=1, sample_every=3)
                ctx.pose_move(lid, 1)
            ctx.hmc_sweep(2, 10, exchange_every=1, sample_every=3)
        else:
            ctx.hmc_sweep(32, 10, exchange_every=1, sample_every=3,
                          pose_move_every=5)
        st = ctx.get_replicas(lid)
        xs, cs = ctx.get_samples(lid)
        ps = ctx.get_pose_stats(lid)
        runs.append((st, xs, cs, ps, ctx.get_stats(lid)))
        ctx.close()
    st0, xs0, cs0, ps0, ss0 = runs[0]
    assert ps0["tries"].sum() == 6 * lig.n_states
    for st, xs, cs, ps, ss in runs[1:]:
        for key in ("x", "state_of_replica", "comps", "counter"):
            assert np.array_equal(st[key], st0[key]), key
        assert np.array_equal(xs, xs0) and np.array_equal(cs, cs0)
        assert np.array_equal(ps["acc"], ps0["acc"])
        assert np.array_equal(ps["tries"], ps0["tries"])
        for key in ss0:
            assert np.array_equal(ss[key], ss0[key]), key
