"""The energy matrix without allocation (bpmf_energy_matrix_batch_noalloc):
its job table lives in a fixed device array, so it must give exactly what
bpmf_energy_matrix_batch gives, call after call, including a second call
with a smaller input that overwrites only part of the table; both against
brute-force u_kn from the oracle (|u32 - u64| <= 1e-5 beta_k S_n, S_n the
magnitude sum of sample n's contributions)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, make_context, print_case, require_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _brute(g, lig, xs, u, cols):
    og, ol = oracle.OGrid(g), oracle.OLigand(lig)
    u64 = oracle.ukn(og, ol, xs[cols])
    _, mags = oracle.components(og, ol, xs[cols])
    S = mags.sum(axis=1)
    beta = 1.0 / (oracle.R_GAS * lig.T)
    assert np.all(np.abs(u[:, cols] - u64) <=
                  1e-5 * beta[:, None] * S[None, :] + 1e-12)


def test_noalloc_energy_matrix_equals_the_allocating_call():
    print_case("no-alloc energy matrix")
    system = synth.make_system(1)
    g = system.grid
    rng = np.random.default_rng(5)
    # one and two wavefronts of atoms, so that two job groups are used
    ligs = [system.ligands[0], synth.make_ligand(rng, 57, 6, box=8.0),
            synth.make_ligand(rng, 90, 5, box=9.0)]
    ctx, ids = make_context(g, ligs, seed=3, capacity=12)
    ctx.hmc_sweep(24, 8, exchange_every=1, sample_every=2)
    # call 1: every ligand's recorded samples
    outs = [torch.full((l.n_states, 12 * l.n_states), float("nan"),
                       dtype=torch.float64, device="cuda:0") for l in ligs]
    got = ctx.energy_matrix_batch(ids, outs=outs, noalloc=True)
    ref = ctx.energy_matrix_batch(ids)
    for lig, lid, a, b in zip(ligs, ids, got, ref):
        assert torch.equal(a, b), lid
        xs, _ = ctx.get_samples(lid)
        xs = xs.reshape(-1, lig.n_atoms, 3)
        cols = rng.choice(xs.shape[0], 20, replace=False)
        _brute(g, lig, xs, a.cpu().numpy(), cols)
    # call 2, smaller: one ligand, explicit device samples, fewer columns,
    # into a padded output (leading dimension > N)
    lig, lid = ligs[2], ids[2]
    xs = (lig.x0[0][None].astype(np.float64) +
          rng.normal(scale=0.3, size=(33, lig.n_atoms, 3))).astype(np.float32)
    xd = dev(xs, torch.float32)
    big = torch.full((lig.n_states, 40), float("nan"), dtype=torch.float64,
                     device="cuda:0")
    (u2,) = ctx.energy_matrix_batch([lid], samples=[xd],
                                    outs=[big[:, :33]], noalloc=True)
    (r2,) = ctx.energy_matrix_batch([lid], samples=[xd])
    assert torch.equal(u2, r2)
    assert torch.isnan(big[:, 33:]).all()
    _brute(g, lig, xs, u2.cpu().numpy(), np.arange(33))
    # call 3: the first batch again, after the smaller one
    again = ctx.energy_matrix_batch(ids, noalloc=True)
    for a, b in zip(again, ref):
        assert torch.equal(a, b)
    # limit on the table size, checked before anything is enqueued
    with pytest.raises(RuntimeError, match="exceed the limit"):
        ctx.energy_matrix_batch([ids[0]] * 1025, n_samples=[0] * 1025,
                                noalloc=True)
    ctx.close()
