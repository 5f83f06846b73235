"""GPU parity of the energy/force kernels against the FP64 oracle: the grid
term alone (trilinear interpolation with per-atom scale, quartic transform,
clamp to edge) and the full configuration energy (grid + GAFF bonded terms +
COM restraint) with forces.

Tolerances (float32 kernel vs float64 oracle at identical float32 inputs):
  energy  |E32 - E64| <= 1e-5 * S, S = sum of |contributions| (magnitude sum)
  forces  |F32 - F64| <= 1e-4 * RMS(F64) per configuration, atoms whose
          coordinates sit within float32 rounding of a cell face exempt.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, grid_grad_magnitude, make_context, near_face, \
    print_case, require_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _grid_case(rng, shape=(20, 18, 16), C=3):
    tr = (4, 0, 0, 0, 4)[:C]
    g = synth.random_grid(rng, n=shape, spacing=0.5, origin=(-4.5, -4.0, -3.5),
                          n_channels=C, transform=tr)
    return g


def _check_forces_by_group(F, F64, ok, mag, group=24):
    """The force tolerance |F32 - F64| <= 1e-4 RMS(F64) per configuration,
    with independent points taken as configurations of `group` consecutive
    points (the 24-atom ligand's size), plus 1e-5 of the gradient's
    magnitude sum `mag` (grid_grad_magnitude: deep in the capped region a
    float32 gradient is a difference of large, nearly equal corner values;
    the rounding there is about 2e-6 of that sum); points within float32
    rounding of a cell face are exempt and do not enter the RMS."""
    n = len(F) // group * group
    d = np.abs(F - F64)[:n].reshape(-1, group, 3)
    f2 = np.where(ok[:n, None], F64[:n] ** 2, 0.0).reshape(-1, group, 3)
    cnt = np.maximum(ok[:n].reshape(-1, group).sum(axis=1), 1)
    rms = np.sqrt(f2.sum(axis=(1, 2)) / (3 * cnt))
    allow = 1e-4 * rms[:, None, None] + 1e-5 * mag[:n].reshape(-1, group, 3)
    bad = (d > allow) & ok[:n].reshape(-1, group)[..., None]
    worst = np.max(np.where(ok[:n].reshape(-1, group)[..., None],
                            d / allow, 0))
    assert not bad.any(), (int(bad.sum()), float(worst))


@pytest.mark.parametrize("C", [3, 5])
def test_grid_eval_random_grid(C):
    rng = np.random.default_rng(10 + C)
    g = _grid_case(rng, C=C)
    print_case("grid_eval random grid", C)
    nx, ny, nz = g.n
    lo = np.array(g.origin)
    hi = lo + g.spacing * (np.array([nx, ny, nz]) - 1)
    n = 50000
    pos = rng.uniform(lo - 1.0, hi + 1.0, size=(n, 3))
    # exact nodes and exact faces too
    idx = rng.integers(0, [nx, ny, nz], size=(2000, 3))
    pos[:2000] = lo + g.spacing * idx
    pos = pos.astype(np.float32)
    scale = rng.normal(size=(n, C)).astype(np.float32)
    w = rng.uniform(0.2, 1.0, C)
    ctx, _ = make_context(g, [], seed=1)
    e, F = ctx.grid_eval(dev(pos, torch.float32), dev(scale, torch.float32), w)
    torch.cuda.synchronize()
    e, F = e.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(
        np.float64)
    og = oracle.OGrid(g)
    e64, F64 = oracle.grid_points(og, pos, scale, w)
    gmax = np.abs(g.nodes).max(axis=(0, 1, 2)).astype(np.float64)
    # magnitude of each channel's value: |s| max|g| (|s| max|g|^4 quartic)
    mag = np.abs(scale) * np.where(np.array(g.transform) == 4, gmax ** 4, gmax)
    assert np.all(np.abs(e - e64) <= 1e-5 * mag + 1e-30)
    ok = ~near_face(pos, g)
    _check_forces_by_group(F, F64, ok, grid_grad_magnitude(g, pos, scale, w))
    fscale = np.sqrt(np.mean(F64[ok] ** 2))
    # per-point relative check where the force is not tiny
    big = ok & (np.linalg.norm(F64, axis=1) > 0.1 * fscale)
    rel = np.linalg.norm(F - F64, axis=1)[big] / np.linalg.norm(F64, axis=1)[big]
    assert np.max(rel) < 1e-4
    # exact nodes: the interpolant returns the node value
    assert np.allclose(e[:2000], e64[:2000], rtol=2e-6, atol=0)
    ctx.close()


def test_grid_eval_config1_grid_at_ligand_positions():
    print_case("grid_eval config-1 grid")
    system = synth.make_system(1)
    g = system.grid
    lig = system.ligands[0]
    rng = np.random.default_rng(3)
    n = 200000
    base = lig.x0[0][rng.integers(0, lig.n_atoms, n)].astype(np.float64)
    pos = (base + rng.normal(scale=1.5, size=(n, 3))).astype(np.float32)
    sc = lig.scale[rng.integers(0, lig.n_atoms, n)].astype(np.float32)
    w = np.array([0.3, 0.6, 0.9])
    ctx, _ = make_context(g, [], seed=1)
    e, F = ctx.grid_eval(dev(pos, torch.float32), dev(sc, torch.float32), w)
    e, F = e.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(
        np.float64)
    og = oracle.OGrid(g)
    e64, F64 = oracle.grid_points(og, pos, sc, w)
    S = np.abs(e64).sum(axis=1)
    assert np.all(np.abs(e - e64).sum(axis=1) <= 1e-5 * S + 1e-12)
    ok = ~near_face(pos, g)
    _check_forces_by_group(F, F64, ok, grid_grad_magnitude(g, pos, sc, w))
    ctx.close()


def _configs(lig, rng, N, sigma=0.3, shift=0.0):
    x = lig.x0[0][None].astype(np.float64) + rng.normal(
        scale=sigma, size=(N, lig.n_atoms, 3)) + shift
    return x.astype(np.float32)


def _check_evaluate(g, lig, xs, w, label, waves=0):
    print_case("evaluate", label, lig.n_atoms, len(xs), "waves", waves)
    ctx, (lid,) = make_context(g, [lig], seed=5)
    ctx.set_waves(waves)
    terms, F = ctx.evaluate(lid, dev(xs, torch.float32), dev(w, torch.float64))
    terms, F = terms.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    og, ol = oracle.OGrid(g), oracle.OLigand(lig)
    t64, m64, F64 = oracle.energy_batch(og, ol, xs, w)
    S = m64.sum(axis=1)
    err = np.abs(terms - t64)
    assert np.all(err <= 1e-5 * S[:, None] + 1e-9), \
        (np.max(err / (S[:, None] + 1e-9)), label)
    nf = near_face(xs, g)
    for i in range(len(xs)):
        rms = np.sqrt(np.mean(F64[i] ** 2))
        ok = ~nf[i]
        d = np.abs(F[i] - F64[i])[ok]
        assert d.size == 0 or d.max() <= 1e-4 * rms + 1e-6, \
            (label, i, d.max(), rms)
    ctx.close()


@pytest.mark.parametrize("waves", [1, 2, 4])
def test_evaluate_config1_ligand(waves):
    system = synth.make_system(1)
    lig = system.ligands[0]
    rng = np.random.default_rng(1)
    xs = _configs(lig, rng, 96)
    w = rng.uniform(0, 1, (96, 3))
    _check_evaluate(system.grid, lig, xs, w, "c1", waves=waves)


def test_evaluate_restraint_active_and_outside_grid():
    system = synth.make_system(1)
    lig = system.ligands[0]
    rng = np.random.default_rng(2)
    # COM pushed 7-9 A from the site: restraint on, atoms beyond the grid
    xs = np.concatenate([_configs(lig, rng, 32, 0.2, shift=np.array(
        [7.5, 0.0, 0.0])), _configs(lig, rng, 32, 0.2, shift=np.array(
            [-3.0, 6.0, 5.0]))])
    w = np.ones((64, 3))
    _check_evaluate(system.grid, lig, xs, w, "restraint+outside")


def test_evaluate_two_atoms_per_lane():
    # 100-atom ligand: atoms 64..99 live in the second slot of each lane
    rng = np.random.default_rng(7)
    lig = synth.make_ligand(rng, 100, 3, box=9.0)
    system = synth.make_system(1)
    xs = _configs(lig, rng, 40, 0.2)
    w = rng.uniform(0, 1, (40, 3))
    _check_evaluate(system.grid, lig, xs, w, "100 atoms")
    _check_evaluate(system.grid, lig, xs, w, "100 atoms", waves=4)


def test_evaluate_single_atom_and_five_channels():
    rng = np.random.default_rng(8)
    g = _grid_case(rng, shape=(24, 24, 24), C=5)
    g.origin = (-5.75,) * 3
    lig = synth.make_ligand(rng, 17, 2, n_channels=5)
    lig.scale[:, 3:] = rng.normal(size=(17, 2))
    xs = _configs(lig, rng, 30, 0.3)
    _check_evaluate(g, lig, xs, rng.uniform(0, 1, (30, 5)), "C=5")
    one = synth.toy_ligand(np.zeros((1, 3)), np.zeros((0, 2)), 0.0,
                           [300.0, 400.0], [0.0, 1.0], n_channels=5)
    one.scale = rng.normal(size=(1, 5))
    xs1 = rng.normal(scale=2.0, size=(20, 1, 3)).astype(np.float32)
    _check_evaluate(g, one, xs1, rng.uniform(0, 1, (20, 5)), "1 atom")


def test_evaluate_is_deterministic():
    system = synth.make_system(1)
    lig = system.ligands[0]
    rng = np.random.default_rng(9)
    xs = dev(_configs(lig, rng, 64), torch.float32)
    w = dev(rng.uniform(0, 1, (64, 3)), torch.float64)
    ctx, (lid,) = make_context(system.grid, [lig], seed=5)
    a = ctx.evaluate(lid, xs, w)
    b = ctx.evaluate(lid, xs, w)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    ctx.close()
