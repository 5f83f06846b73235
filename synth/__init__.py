"""Seeded synthetic inputs for the BPMF hot path.

This module produces the *inputs* of the method and nothing else: receptor
grids (from random point atoms), ligand topologies with force-field
parameters, starting coordinates and the thermodynamic-state ladder.  It holds
none of the sampling or energy arithmetic that the GPU library and the CPU
oracle implement; both sides receive the arrays produced here.

Stand-in for the paper's workload.  The paper runs on the Astex Diverse Set
with AMBER/GAFF inputs and APBS grids (Methodology, "Astex diverse set BPMF
calculations"); none of that is available, so every system here is synthetic,
with the structural parameters the paper gives: a three-grid receptor model
(one electrostatic and two van der Waals grids, "Thermodynamic Cycle"), a
flat-bottom binding-site restraint with d0 = 6 A and k = 10000 kJ/(mol nm^2)
(Eq. binding_site), temperatures between 300 and 600 K (Estimation), and
drug-sized ligands.

Grid recipe (readings that the paper leaves open):
  * nodes on an n^3 lattice with spacing h, centred on the binding-site centre
    c0 = 0, origin -(n-1)h/2;
  * LJ grids use the geometric-mean combination rule, which factorises the
    pair energy into a receptor grid times a per-ligand-atom factor:
        G_rep(x) = sum_j 2 sqrt(eps_j) sigma_j^6 / r_s^12
        G_att(x) = sum_j 2 sqrt(eps_j) sigma_j^3 / r_s^6
        G_ele(x) = 1389.35457 sum_j q_j / r_s          (epsilon_r = 1)
    with softened distance r_s^2 = r^2 + delta^2 (delta = 0.5 A);
  * node values are clamped to [-1e4, 1e4];
  * the repulsive grid is stored as G_rep^(1/4) (inverse transformation power
    4, Eq. for Psi_vdW discussion); attractive and electrostatic are stored raw.
Per-atom ligand factors: s_rep = 2 sqrt(eps) sigma^6, s_att = -2 sqrt(eps)
sigma^3, s_ele = q.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional

import numpy as np

COULOMB = 1389.35457  # kJ A / (mol e^2)
C_RELEASE = 0  # format version of the generated arrays

GRID_DELTA = 0.5      # softening length (A)
GRID_CAP = 1.0e4      # node clamp
K_BOND = 1000.0       # kJ/(mol A^2)
K_ANGLE = 250.0       # kJ/(mol rad^2)
BOND_LEN = 1.5        # A
MASS_C = 12.011       # amu
K_RESTRAINT = 100.0   # kJ/(mol A^2) == 10000 kJ/(mol nm^2)
D0 = 6.0              # A


@dataclasses.dataclass
class Grid:
    """Regular grid: nodes[iz, iy, ix, c] (x fastest), float32."""
    n: tuple            # (nx, ny, nz)
    origin: tuple       # (ox, oy, oz)
    spacing: float
    transform: tuple    # per channel: 4 = stored quartic root, 0 = none
    nodes: np.ndarray   # (nz, ny, nx, C) float32

    @property
    def n_channels(self):
        return self.nodes.shape[-1]


@dataclasses.dataclass
class Ligand:
    """One flexible ligand with its force field, ladder and starting replicas."""
    n_atoms: int
    mass: np.ndarray        # (n,) float64
    scale: np.ndarray       # (n, C) float64: rep, att, ele(q)
    bonds: np.ndarray       # (nb, 2) int32
    bond_par: np.ndarray    # (nb, 2) float64: K_r, r0
    angles: np.ndarray      # (na, 3) int32  (i, j=centre, k)
    angle_par: np.ndarray   # (na, 2) float64: K_theta, theta0 (rad)
    tors: np.ndarray        # (nt, 4) int32
    tors_par: np.ndarray    # (nt, 3) float64: V/2, n, gamma
    site_center: np.ndarray  # (3,)
    d0: float
    k_restraint: float
    T: np.ndarray           # (K,) state temperatures (K)
    w: np.ndarray           # (K, C) state grid weights
    dt: np.ndarray          # (K,) time step per state (fs)
    x0: np.ndarray          # (K, n, 3) float32, one replica per state
    frame_atoms: tuple = (0, 1, 2)
    cond_tors: Optional[np.ndarray] = None  # torsion indices used as conditioning
    ligand_seed: int = 0

    @property
    def n_states(self):
        return len(self.T)


@dataclasses.dataclass
class System:
    name: str
    grid: Grid
    ligands: List[Ligand]
    seed: int              # Philox key for the run
    n_sweeps: int
    n_leapfrog: int
    sample_every: int
    exchange_every: int = 1


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

def grid_axes(n, h):
    origin = -(n - 1) * h / 2.0
    ax = origin + h * np.arange(n, dtype=np.float64)
    return origin, ax


def grids_from_points(points, q, sigma, eps, n, h, delta=GRID_DELTA,
                      cap=GRID_CAP, chunk=None, device=None):
    """Receptor grids on an n^3 lattice from point atoms (see module doc).

    Returns float32 nodes (n, n, n, 3) with channels (rep^(1/4), att, ele).
    device: torch device for the float64 sums (default CPU; the large
    lattices are generated on a GPU in seconds).  Both run the same
    operations in the same order; results may differ in the last bits.
    """
    import torch  # float64 elementwise sums; only input generation
    dev = torch.device(device) if device is not None else torch.device("cpu")
    origin, ax = grid_axes(n, h)
    axt = torch.from_numpy(ax).to(dev)
    P = torch.from_numpy(np.asarray(points, np.float64))
    c_rep = torch.from_numpy(2.0 * np.sqrt(eps) * sigma ** 6)
    c_att = torch.from_numpy(2.0 * np.sqrt(eps) * sigma ** 3)
    c_ele = torch.from_numpy(COULOMB * np.asarray(q, np.float64))
    rep = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    att = torch.zeros_like(rep)
    ele = torch.zeros_like(rep)
    d2 = delta * delta
    # slab over z to bound temporaries
    zs = max(1, int(2 ** 22 // (n * n)))
    for z0 in range(0, n, zs):
        z1 = min(n, z0 + zs)
        zz = axt[z0:z1].view(-1, 1, 1)
        yy = axt.view(1, -1, 1)
        xx = axt.view(1, 1, -1)
        r_acc = rep[z0:z1]
        a_acc = att[z0:z1]
        e_acc = ele[z0:z1]
        for j in range(P.shape[0]):
            px, py, pz = P[j, 0].item(), P[j, 1].item(), P[j, 2].item()
            s = (zz - pz) ** 2 + (yy - py) ** 2 + (xx - px) ** 2 + d2
            inv = 1.0 / s
            inv3 = inv * inv * inv
            a_acc.add_(inv3, alpha=c_att[j].item())
            r_acc.add_(inv3 * inv3, alpha=c_rep[j].item())
            e_acc.add_(torch.sqrt(inv), alpha=c_ele[j].item())
    rep.clamp_(-cap, cap)
    att.clamp_(-cap, cap)
    ele.clamp_(-cap, cap)
    out = torch.stack([rep.pow(0.25), att, ele], dim=-1)
    return out.cpu().numpy().astype(np.float32)


def make_receptor(rng, n_points, edge, pocket_radius, avoid_xyz=None,
                  avoid_dist=3.0):
    """Receptor point atoms, uniform in the grid box outside the pocket ball
    and at least avoid_dist from every starting ligand atom."""
    pts = []
    avoid = None if avoid_xyz is None else np.asarray(avoid_xyz, np.float64)
    while len(pts) < n_points:
        p = rng.uniform(-edge / 2, edge / 2, size=3)
        if np.linalg.norm(p) < pocket_radius:
            continue
        if avoid is not None and len(avoid) and \
                np.min(np.linalg.norm(avoid - p, axis=1)) < avoid_dist:
            continue
        pts.append(p)
    pts = np.array(pts)
    q = rng.uniform(-0.5, 0.5, n_points)
    sig = rng.uniform(3.0, 4.0, n_points)
    eps = rng.uniform(0.05, 0.3, n_points)
    return pts, q, sig, eps


def linear_field_grid(n, h, field, phi0):
    """Toy grid set whose electrostatic channel is the linear field
    G_ele(x) = field . x + phi0 and whose LJ channels are zero."""
    origin, ax = grid_axes(n, h)
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    ele = field[0] * xx + field[1] * yy + field[2] * zz + phi0
    nodes = np.zeros((n, n, n, 3), np.float32)
    nodes[..., 2] = ele.astype(np.float32)
    return Grid((n, n, n), (origin,) * 3, h, (4, 0, 0), nodes)


# --------------------------------------------------------------------------
# ligands
# --------------------------------------------------------------------------

def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_tree(rng, n_atoms, box=6.0, bond=BOND_LEN, min_sep=1.2,
                max_angle_deg=165.0, far_sep=None):
    """Random tree-shaped ligand grown in a cube of edge `box` centred on 0.

    Atom 0 sits at the centre; each new atom attaches at distance `bond` in a
    uniform random direction to a random existing atom of degree < 4.  A
    placement is rejected when it leaves the box, comes closer than min_sep
    to another atom, or makes a near-linear angle with a bond of its parent;
    with far_sep, also when it comes closer than far_sep to an atom three or
    more bonds away (every atom but its parent and the parent's neighbours),
    so that no pair the intramolecular nonbonded terms see starts in a
    clash.
    """
    x = [np.zeros(3)]
    deg = [0]
    nbr = [[]]
    bonds = []
    cosmax = math.cos(math.radians(max_angle_deg))
    misses = 0
    while len(x) < n_atoms:
        misses += 1
        if misses > 5000:
            raise RuntimeError("random_tree: no room for atom %d of %d in a "
                               "box of %g" % (len(x) + 1, n_atoms, box))
        cand = [i for i in range(len(x)) if deg[i] < 4]
        p = cand[rng.integers(len(cand))]
        for _ in range(100):
            d = _unit(rng)
            y = x[p] + bond * d
            if np.any(np.abs(y) > box / 2):
                continue
            X = np.array(x)
            dist = np.linalg.norm(X - y, axis=1)
            if np.min(dist) < min_sep:
                continue
            if far_sep is not None:
                near = np.ones(len(x), bool)
                near[p] = False
                near[nbr[p]] = False
                if np.any(dist[near] < far_sep):
                    continue
            ok = True
            for q in nbr[p]:
                u = (x[q] - x[p]) / np.linalg.norm(x[q] - x[p])
                if np.dot(u, d) < cosmax:
                    ok = False
                    break
            if not ok:
                continue
            j = len(x)
            x.append(y)
            deg.append(1)
            nbr.append([p])
            deg[p] += 1
            nbr[p].append(j)
            bonds.append((p, j))
            misses = 0
            break
    return np.array(x), np.array(bonds, np.int32), nbr


def angles_and_torsions(n_atoms, bonds, nbr):
    angles = []
    for j in range(n_atoms):
        nb = nbr[j]
        for a in range(len(nb)):
            for b in range(a + 1, len(nb)):
                angles.append((nb[a], j, nb[b]))
    tors = []
    for (b, c) in bonds:
        for a in nbr[b]:
            if a == c:
                continue
            for d in nbr[c]:
                if d == b:
                    continue
                tors.append((a, b, c, d))
    return (np.array(angles, np.int32).reshape(-1, 3),
            np.array(tors, np.int32).reshape(-1, 4))


def _geom_angle(x, i, j, k):
    a = x[i] - x[j]
    b = x[k] - x[j]
    return math.atan2(np.linalg.norm(np.cross(a, b)), float(np.dot(a, b)))


def _geom_dihedral(x, i, j, k, l):
    b1 = x[j] - x[i]
    b2 = x[k] - x[j]
    b3 = x[l] - x[k]
    n1 = np.cross(b1, b2)
    n2 = np.cross(b2, b3)
    y = np.linalg.norm(b2) * float(np.dot(b1, n2))
    return math.atan2(y, float(np.dot(n1, n2)))


def ladder(K, T_hot=600.0, T_target=300.0, n_channels=3):
    """1-D coupled ladder: lambda_k = k/(K-1), T_k = T_hot + (T_target -
    T_hot) lambda_k, grid weights w_k = lambda_k on every channel."""
    lam = np.linspace(0.0, 1.0, K)
    T = T_hot + (T_target - T_hot) * lam
    w = np.repeat(lam[:, None], n_channels, axis=1)
    return T, w


def soft_schedule(K, T_hot=600.0, T_target=300.0):
    """The paper's switching protocol between milestones C and D
    (Thermodynamic Cycle): alpha_k = k/(K-1),
        alpha_sg = 1 - (2 alpha - 1)^2,
        alpha_g  = (2 alpha - 1)^2 / (1 + exp(-1000 (alpha - 1/2))),
        T = (T_target - T_hot) alpha + T_hot,
    the soft grids switched on first, then the original grids.  Returns T
    (K,) and weights (K, 5) on the channels (rep, att, ele, soft rep, soft
    ele), in float64 (exp(500) overflows float32)."""
    a = np.linspace(0.0, 1.0, K)
    sq = (2.0 * a - 1.0) ** 2
    a_sg = 1.0 - sq
    with np.errstate(over="ignore"):
        a_g = sq / (1.0 + np.exp(-1000.0 * (a - 0.5)))
    T = (T_target - T_hot) * a + T_hot
    w = np.stack([a_g, a_g, a_g, a_sg, a_sg], axis=1)
    return T, w


def add_soft_grids(grid, ligands, cap_energy=10.0):
    """Append the soft repulsive and electrostatic channels v_max tanh(v /
    v_max) to a three-channel receptor grid and the matching per-atom
    factors to the ligands (Thermodynamic Cycle, soft grids).

    Readings: the paper's v_max = 10 is in its own grid units; here the
    repulsive cap makes the soft repulsion of the median ligand atom at most
    cap_energy kJ/mol (v_max = cap_energy / median s_rep), and, as in the
    paper, the electrostatic cap keeps every atom's soft electrostatic
    energy at or below its soft repulsive cap (v_max = v_max_rep x the
    minimum over atoms of s_rep / |q|).  Both soft channels are stored and
    interpolated untransformed."""
    rep = grid.nodes[..., 0].astype(np.float64) ** 4
    ele = grid.nodes[..., 2].astype(np.float64)
    s_rep = np.concatenate([l.scale[:, 0] for l in ligands])
    q = np.concatenate([np.abs(l.scale[:, 2]) for l in ligands])
    vr = cap_energy / float(np.median(s_rep))
    ratio = s_rep[q > 0] / q[q > 0]
    ve = vr * float(ratio.min()) if ratio.size else vr
    soft = np.stack([vr * np.tanh(rep / vr), ve * np.tanh(ele / ve)], axis=-1)
    nodes = np.concatenate([grid.nodes, soft.astype(np.float32)], axis=-1)
    out = Grid(grid.n, grid.origin, grid.spacing, tuple(grid.transform) +
               (0, 0), nodes)
    ligs = []
    for l in ligands:
        l2 = dataclasses.replace(l)
        l2.scale = np.concatenate([l.scale, l.scale[:, [0, 2]]], axis=1)
        T, w = soft_schedule(l.n_states)
        l2.T, l2.w = T, w
        ligs.append(l2)
    return out, ligs


def make_ligand(rng, n_atoms, K, box=6.0, dt=1.0, n_channels=3,
                mass=MASS_C, ligand_seed=0, far_sep=None):
    x, bonds, nbr = random_tree(rng, n_atoms, box=box, far_sep=far_sep)
    x32 = x.astype(np.float32)
    xd = x32.astype(np.float64)
    angles, tors = angles_and_torsions(n_atoms, bonds, nbr)
    bond_par = np.array([[K_BOND, np.linalg.norm(xd[i] - xd[j])]
                         for i, j in bonds], np.float64).reshape(-1, 2)
    angle_par = np.array([[K_ANGLE, _geom_angle(xd, i, j, k)]
                          for i, j, k in angles], np.float64).reshape(-1, 2)
    tp = []
    for (a, b, c, d) in tors:
        vh = rng.uniform(0.0, 5.0)
        nn = int(rng.integers(1, 4))
        phi0 = _geom_dihedral(xd, a, b, c, d)
        tp.append([vh, float(nn), nn * phi0 - math.pi])
    tors_par = np.array(tp, np.float64).reshape(-1, 3)
    q = rng.uniform(-0.5, 0.5, n_atoms)
    sig = rng.uniform(3.0, 4.0, n_atoms)
    eps = rng.uniform(0.05, 0.3, n_atoms)
    scale = np.stack([2 * np.sqrt(eps) * sig ** 6, -2 * np.sqrt(eps) * sig ** 3,
                      q], axis=1)
    if n_channels > 3:
        scale = np.concatenate(
            [scale, np.zeros((n_atoms, n_channels - 3))], axis=1)
    T, w = ladder(K, n_channels=n_channels)
    x0 = np.repeat(x32[None], K, axis=0)
    # conditioning torsions for the learned move: rotatable bonds in BFS order
    # from the root (one torsion per central bond, first 8)
    seen = set()
    cond = []
    for t, (a, b, c, d) in enumerate(tors):
        key = (min(b, c), max(b, c))
        if key in seen:
            continue
        seen.add(key)
        cond.append(t)
    cond = np.array(cond[:8], np.int32)
    return Ligand(n_atoms=n_atoms, mass=np.full(n_atoms, mass),
                  scale=scale, bonds=bonds, bond_par=bond_par,
                  angles=angles, angle_par=angle_par, tors=tors,
                  tors_par=tors_par, site_center=np.zeros(3), d0=D0,
                  k_restraint=K_RESTRAINT, T=T, w=w,
                  dt=np.full(K, float(dt)), x0=x0, frame_atoms=(0, 1, 2)
                  if n_atoms >= 3 else (0, 0, 0), cond_tors=cond,
                  ligand_seed=ligand_seed)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

CONFIGS = {
    # name: grid n, receptor points, ligand atom counts, states, sweeps, L,
    # sample_every
    1: dict(name="c1_plain_small", n=48, n_rec=200, atoms=[24], K=8,
            sweeps=1000, L=10, sample_every=10),
    2: dict(name="c2_plain_production", n=128, n_rec=2000, atoms=[48], K=64,
            sweeps=5000, L=20, sample_every=10),
    3: dict(name="c3_batched_uneven", n=160, n_rec=4000, atoms=("U", 10, 80,
                                                                   256),
            K=32, sweeps=2000, L=10, sample_every=10),
    4: dict(name="c4_learned", n=48, n_rec=200, atoms=[24], K=64,
            sweeps=5000, L=10, sample_every=10),
    5: dict(name="c5_large_batched", n=256, n_rec=8000,
            atoms=("U", 40, 100, 32), K=32, sweeps=10000, L=10,
            sample_every=50),
}


_GRID_CACHE = {}


def make_system(config: int, n_ligands: Optional[int] = None,
                with_grid: bool = True, grid_device=None) -> System:
    """Build config `config` (1..5).  n_ligands truncates the ligand list of
    the batched configs (the first n_ligands ligands are identical to the
    full system's).  grid_device: torch device that sums the receptor grids
    (see grids_from_points)."""
    c = CONFIGS[config]
    gen_seed = 100 + config
    rng = np.random.default_rng(gen_seed)
    atoms = c["atoms"]
    if isinstance(atoms, tuple):
        _, lo, hi, nl = atoms
        counts = rng.integers(lo, hi + 1, size=nl)
    else:
        counts = np.array(atoms)
    if n_ligands is not None:
        counts = counts[:n_ligands]
    ligs = []
    for li, na in enumerate(counts):
        lrng = np.random.default_rng([gen_seed, 1000 + li])
        ligs.append(make_ligand(lrng, int(na), c["K"], ligand_seed=li))
    n, h = c["n"], 0.25
    edge = (n - 1) * h
    if with_grid:
        key = (config, len(counts), str(grid_device))
        # optional on-disk cache of generated grids (a directory named by
        # BPMF_GRID_CACHE): the generation is deterministic, so a cached
        # grid equals a fresh one of the same config, ligand count and
        # summing device
        cdir = os.environ.get("BPMF_GRID_CACHE")
        cfile = (os.path.join(cdir, f"grid_c{config}_l{len(counts)}_"
                              f"{'cpu' if grid_device is None else str(grid_device).replace(':', '')}"
                              f"_v{C_RELEASE}.npy") if cdir else None)
        if key not in _GRID_CACHE and cfile and os.path.exists(cfile):
            _GRID_CACHE[key] = np.load(cfile)
        if key not in _GRID_CACHE:
            rrng = np.random.default_rng([gen_seed, 7])
            avoid = np.concatenate([l.x0[0] for l in ligs], axis=0)
            pts, q, sig, eps = make_receptor(rrng, c["n_rec"], edge,
                                             0.3 * edge, avoid_xyz=avoid)
            _GRID_CACHE[key] = grids_from_points(pts, q, sig, eps, n, h,
                                                 device=grid_device)
            if cfile:
                os.makedirs(cdir, exist_ok=True)
                np.save(cfile + ".tmp.npy", _GRID_CACHE[key])
                os.replace(cfile + ".tmp.npy", cfile)
        nodes = _GRID_CACHE[key].copy()
    else:
        nodes = np.zeros((0, 0, 0, 3), np.float32)
    origin = -(n - 1) * h / 2
    grid = Grid((n, n, n), (origin,) * 3, h, (4, 0, 0), nodes)
    return System(name=c["name"], grid=grid, ligands=ligs, seed=200 + config,
                  n_sweeps=c["sweeps"], n_leapfrog=c["L"],
                  sample_every=c["sample_every"])


def random_grid(rng, n=(6, 5, 4), spacing=0.5, origin=(-1.0, -0.5, -0.25),
                n_channels=3, transform=(4, 0, 0)):
    """Small random grid for interpolation tests (rep channel >= 0)."""
    nx, ny, nz = n
    nodes = rng.normal(size=(nz, ny, nx, n_channels)).astype(np.float32)
    for c, t in enumerate(transform):
        if t == 4:
            nodes[..., c] = np.abs(nodes[..., c])
    return Grid(tuple(n), tuple(origin), spacing, tuple(transform), nodes)


def multilinear_grid(coef, n=(5, 6, 7), spacing=0.5, origin=(-1.0, -1.5, -2.0)):
    """Grid sampling f(x,y,z) = a + bx + cy + dz + exy + fxz + gyz + hxyz on
    every channel (all untransformed); coef = (a..h) per channel (C, 8)."""
    nx, ny, nz = n
    ox, oy, oz = origin
    X = ox + spacing * np.arange(nx)
    Y = oy + spacing * np.arange(ny)
    Z = oz + spacing * np.arange(nz)
    zz, yy, xx = np.meshgrid(Z, Y, X, indexing="ij")
    C = len(coef)
    nodes = np.zeros((nz, ny, nx, C), np.float64)
    for c in range(C):
        a, b, cc, d, e, f, g, hh = coef[c]
        nodes[..., c] = (a + b * xx + cc * yy + d * zz + e * xx * yy +
                         f * xx * zz + g * yy * zz + hh * xx * yy * zz)
    return Grid(tuple(n), tuple(origin), spacing, (0,) * C,
                nodes.astype(np.float32))


def toy_ligand(x, bonds, bond_K, T, lam, q=0.3, mass=1.0, dt=2.0, d0=2.0,
               k_restraint=K_RESTRAINT, n_channels=3):
    """Bond-only ligand with equal masses and equal charges and zero LJ
    factors, the solvable toy whose free energies have a quadrature form.
    lam are the per-state electrostatic weights (LJ weights equal lam too but
    the LJ factors are zero)."""
    x = np.asarray(x, np.float64)
    n = len(x)
    bonds = np.asarray(bonds, np.int32).reshape(-1, 2)
    x32 = x.astype(np.float32)
    xd = x32.astype(np.float64)
    bond_par = np.array([[bond_K, np.linalg.norm(xd[i] - xd[j])]
                         for i, j in bonds], np.float64).reshape(-1, 2)
    scale = np.zeros((n, n_channels))
    scale[:, 2] = q
    T = np.asarray(T, np.float64)
    lam = np.asarray(lam, np.float64)
    K = len(T)
    w = np.repeat(lam[:, None], n_channels, axis=1)
    return Ligand(n_atoms=n, mass=np.full(n, float(mass)), scale=scale,
                  bonds=bonds, bond_par=bond_par,
                  angles=np.zeros((0, 3), np.int32),
                  angle_par=np.zeros((0, 2)),
                  tors=np.zeros((0, 4), np.int32), tors_par=np.zeros((0, 3)),
                  site_center=np.zeros(3), d0=float(d0),
                  k_restraint=float(k_restraint), T=T, w=w,
                  dt=np.full(K, float(dt)),
                  x0=np.repeat(x32[None], K, axis=0), frame_atoms=(0, 1, 2),
                  cond_tors=np.zeros(0, np.int32))


def pair_params(lig, seed=0):
    """Intramolecular nonbonded and implicit-solvent parameters of a
    synthetic ligand: its own per-atom LJ sigma, eps and charge (recovered
    from the grid factors s_rep = 2 sqrt(eps) sigma^6, s_att = -2 sqrt(eps)
    sigma^3, s_ele = q), GB intrinsic radii ~ U(1.3, 1.9) A and HCT scale
    factors ~ U(0.72, 0.9) (the span of common radius sets), exclusions of
    the 1-2 and 1-3 pairs, the torsions' end pairs as 1-4 pairs (LJ x 1/2,
    Coulomb x 1/1.2), water outside (78.5) and a dielectric of 1 inside,
    surface tension 0.0225936 kJ/mol/A^2 with a 1.4 A probe."""
    rng = np.random.default_rng([seed, 4242, lig.n_atoms])
    s_rep, s_att, q = lig.scale[:, 0], lig.scale[:, 1], lig.scale[:, 2]
    sig3 = s_rep / (-s_att)
    sigma = np.cbrt(sig3)
    eps = (s_att / (2.0 * sig3)) ** 2
    n = lig.n_atoms
    excl = set()
    for i, j in np.asarray(lig.bonds).reshape(-1, 2):
        excl.add((min(i, j), max(i, j)))
    for i, _, k in np.asarray(lig.angles).reshape(-1, 3):
        excl.add((min(i, k), max(i, k)))
    p14 = set()
    for i, _, _, l in np.asarray(lig.tors).reshape(-1, 4):
        key = (min(i, l), max(i, l))
        if key not in excl:
            p14.add(key)
    return dict(charge=np.asarray(q, np.float64), sigma=sigma, eps=eps,
                rho=rng.uniform(1.3, 1.9, n), S=rng.uniform(0.72, 0.9, n),
                exclusions=np.array(sorted(excl), np.int32).reshape(-1, 2),
                pairs14=np.array(sorted(p14), np.int32).reshape(-1, 2),
                lj14=0.5, el14=1.0 / 1.2, eps_solute=1.0, eps_solvent=78.5,
                gamma=0.0225936, probe=1.4)
