"""FP64 CPU oracle for the BPMF hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library:
the C part (`oracle.c`) is compiled with gcc into `liboracle.so`, the
estimators (MBAR, BAR, ESS, exact-toy quadrature) are plain NumPy/SciPy in
double precision.

Python wrappers here do argument marshalling only; the arithmetic lives in
oracle.c (energies, forces, HMC, exchange, u_kn) and in mbar.py / toy.py.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source
# (CPU checking only; loaded instead of LIB_PATH when BPMF_ORACLE_LIB names
# it, in a process that preloads the sanitizer runtime)
SAN_LIB_PATH = os.path.join(HERE, "liboracle_san.so")
CLANG = "/opt/rocm/llvm/bin/clang"
R_GAS = 8.314462618e-3  # kJ/(mol K)

P_MOMENTA, P_ACCEPT, P_EXCHANGE, P_POSE = 1, 2, 3, 4
P_EXTERNAL = 6


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O3, OpenMP, FP64, no fast-math)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-fno-fast-math", "-ffp-contract=off", src, "-o",
               tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_sanitized(out: str = SAN_LIB_PATH) -> str:
    """Compile oracle.c with clang's AddressSanitizer and
    UndefinedBehaviorSanitizer (the runtime shared, so that one preloaded
    runtime serves this library and the HIP library's sanitized host code
    in one process); every undefined-behaviour report is fatal."""
    src = os.path.join(HERE, "oracle.c")
    tmp = out + ".tmp"
    cmd = [CLANG, "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-shared-libsan", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-ffp-contract=off", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("nc", C.c_int), ("ox", C.c_double), ("oy", C.c_double),
                ("oz", C.c_double), ("h", C.c_double),
                ("transform", C.POINTER(C.c_int)),
                ("nodes", C.POINTER(C.c_float))]


class _Ligand(C.Structure):
    _fields_ = [("n", C.c_int), ("mass", C.POINTER(C.c_double)),
                ("scale", C.POINTER(C.c_double)),
                ("nb", C.c_int), ("bij", C.POINTER(C.c_int)),
                ("bpar", C.POINTER(C.c_double)),
                ("na", C.c_int), ("aijk", C.POINTER(C.c_int)),
                ("apar", C.POINTER(C.c_double)),
                ("nt", C.c_int), ("tijkl", C.POINTER(C.c_int)),
                ("tpar", C.POINTER(C.c_double)),
                ("c0", C.c_double * 3), ("d0", C.c_double),
                ("krest", C.c_double),
                ("pair_on", C.c_int), ("pq", C.POINTER(C.c_double)),
                ("psig", C.POINTER(C.c_double)),
                ("peps", C.POINTER(C.c_double)),
                ("prho", C.POINTER(C.c_double)),
                ("pS", C.POINTER(C.c_double)),
                ("pexcl", C.POINTER(C.c_ubyte)),
                ("p14", C.POINTER(C.c_ubyte)),
                ("lj14", C.c_double), ("el14", C.c_double),
                ("eps_in", C.c_double), ("eps_out", C.c_double),
                ("gamma", C.c_double), ("probe", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("BPMF_ORACLE_LIB", LIB_PATH)
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        vp = C.c_void_p
        L.ora_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                 C.POINTER(C.c_uint32)]
        L.ora_interp.argtypes = [vp, dp, dp, dp]
        L.ora_atom_grid.argtypes = [vp, dp, dp, dp, dp]
        L.ora_energy.argtypes = [vp, vp, dp, dp, dp, dp, dp]
        L.ora_verlet.argtypes = [vp, vp, dp, C.c_double, C.c_int, dp, dp, dp,
                                 dp]
        L.ora_momenta.argtypes = [vp, C.c_double, C.c_uint64, C.c_int,
                                  C.c_int, C.c_uint64, dp]
        L.ora_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int,
                                  C.c_uint64, C.c_uint32]
        L.ora_uniform.restype = C.c_double
        L.ora_hmc_sweep.argtypes = [vp, vp, C.c_int, dp, dp, dp, C.c_uint64,
                                    C.c_int, C.c_int, C.c_uint64, C.c_int,
                                    dp, ip, dp, ip, dp, dp]
        L.ora_exchange.argtypes = [C.c_int, C.c_int, dp, dp, C.c_uint64,
                                   C.c_int, C.c_uint64, C.c_int, C.c_int,
                                   C.c_int, dp,
                                   ip, ip, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]
        L.ora_ukn.argtypes = [vp, vp, C.c_int, dp, dp, C.c_int64, dp, dp]
        L.ora_components.argtypes = [vp, vp, C.c_int64, dp, dp, dp]
        L.ora_grid_points.argtypes = [vp, C.c_int64, dp, dp, dp, dp, dp]
        L.ora_energy_batch.argtypes = [vp, vp, C.c_int64, dp, dp, dp, dp, dp]
        L.ora_normals3.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int,
                                   C.c_uint64, C.c_uint32, dp]
        L.ora_uniform4.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int,
                                   C.c_uint64, C.c_uint32, dp]
        L.ora_dihedral.argtypes = [dp, dp, dp, dp]
        L.ora_dihedral.restype = C.c_double
        L.ora_angle.argtypes = [dp, dp, dp]
        L.ora_angle.restype = C.c_double
        L.ora_num_threads.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class OGrid:
    """Grid as the oracle sees it (keeps its arrays alive)."""

    def __init__(self, grid):
        self.nodes = np.ascontiguousarray(grid.nodes, dtype=np.float32)
        self.transform = _i(grid.transform)
        nz, ny, nx, nc = self.nodes.shape
        self.nc = nc
        self.s = _Grid(nx, ny, nz, nc, float(grid.origin[0]),
                       float(grid.origin[1]), float(grid.origin[2]),
                       float(grid.spacing), _p(self.transform, C.c_int),
                       _p(self.nodes, C.c_float))

    @property
    def ref(self):
        return C.byref(self.s)


class OLigand:
    """Ligand as the oracle sees it.  pairs: optional intramolecular
    nonbonded / OBC GB-SA parameters (the dict synth.pair_params gives);
    with them the pair terms are part of the ligand's energy."""

    def __init__(self, lig, pairs=None):
        self.n = lig.n_atoms
        self.mass = _d(lig.mass)
        self.scale = _d(lig.scale)
        self.bij = _i(lig.bonds).reshape(-1)
        self.bpar = _d(lig.bond_par).reshape(-1)
        self.aijk = _i(lig.angles).reshape(-1)
        self.apar = _d(lig.angle_par).reshape(-1)
        self.tijkl = _i(lig.tors).reshape(-1)
        self.tpar = _d(lig.tors_par).reshape(-1)
        self.T = _d(lig.T)
        self.w = _d(lig.w)
        self.dt = _d(lig.dt)
        c0 = (C.c_double * 3)(*[float(v) for v in lig.site_center])
        self.s = _Ligand(self.n, _p(self.mass, C.c_double),
                         _p(self.scale, C.c_double),
                         len(lig.bonds), _p(self.bij, C.c_int),
                         _p(self.bpar, C.c_double),
                         len(lig.angles), _p(self.aijk, C.c_int),
                         _p(self.apar, C.c_double),
                         len(lig.tors), _p(self.tijkl, C.c_int),
                         _p(self.tpar, C.c_double), c0, float(lig.d0),
                         float(lig.k_restraint))
        self.K = len(lig.T)
        self.pairs = pairs
        if pairs is not None:
            n = self.n
            self.pq = _d(pairs["charge"])
            self.psig = _d(pairs["sigma"])
            self.peps = _d(pairs["eps"])
            self.prho = _d(pairs["rho"])
            self.pS = _d(pairs["S"])
            ex = np.zeros((n, n), np.uint8)
            for i, j in np.asarray(pairs["exclusions"], int).reshape(-1, 2):
                ex[i, j] = ex[j, i] = 1
            o4 = np.zeros((n, n), np.uint8)
            for i, j in np.asarray(pairs["pairs14"], int).reshape(-1, 2):
                if not ex[i, j]:
                    o4[i, j] = o4[j, i] = 1
            self.pexcl, self.p14 = ex, o4
            s = self.s
            s.pair_on = 1
            s.pq = _p(self.pq, C.c_double)
            s.psig = _p(self.psig, C.c_double)
            s.peps = _p(self.peps, C.c_double)
            s.prho = _p(self.prho, C.c_double)
            s.pS = _p(self.pS, C.c_double)
            s.pexcl = _p(self.pexcl, C.c_ubyte)
            s.p14 = _p(self.p14, C.c_ubyte)
            s.lj14, s.el14 = float(pairs["lj14"]), float(pairs["el14"])
            s.eps_in = float(pairs["eps_solute"])
            s.eps_out = float(pairs["eps_solvent"])
            s.gamma, s.probe = float(pairs["gamma"]), float(pairs["probe"])

    @property
    def ref(self):
        return C.byref(self.s)


# --------------------------------------------------------------------------
# thin wrappers
# --------------------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().ora_philox(c, k, o)
    return tuple(o)


def uniform(seed, index, lig, rep, sweep, purpose):
    return lib().ora_uniform(seed, index, lig, rep, sweep, purpose)


def uniform4(seed, index, lig, rep, sweep, purpose):
    u = np.zeros(4)
    lib().ora_uniform4(seed, index, lig, rep, sweep, purpose,
                       _p(u, C.c_double))
    return u


def normals3(seed, index, lig, rep, sweep, purpose):
    z = np.zeros(3)
    lib().ora_normals3(seed, index, lig, rep, sweep, purpose,
                       _p(z, C.c_double))
    return z


def interp(og: OGrid, p):
    p = _d(p)
    v = np.zeros(og.nc)
    dv = np.zeros((og.nc, 3))
    lib().ora_interp(og.ref, _p(p, C.c_double), _p(v, C.c_double),
                     _p(dv, C.c_double))
    return v, dv


def atom_grid(og: OGrid, p, scale):
    p = _d(p)
    s = _d(scale)
    e = np.zeros(og.nc)
    de = np.zeros((og.nc, 3))
    lib().ora_atom_grid(og.ref, _p(p, C.c_double), _p(s, C.c_double),
                        _p(e, C.c_double), _p(de, C.c_double))
    return e, de


def energy(og: OGrid, ol: OLigand, w, x, forces=True):
    """Return (terms, mags, F): terms = [U_bond, U_angle, U_tors, U_restr,
    Psi_c...], F = -grad(U_b + U_r + sum_c w_c Psi_c)."""
    w = _d(w)
    x = _d(x).reshape(-1)
    nt = 4 + og.nc
    terms = np.zeros(nt)
    mags = np.zeros(nt)
    F = np.zeros(3 * ol.n) if forces else None
    lib().ora_energy(og.ref, ol.ref, _p(w, C.c_double), _p(x, C.c_double),
                     _p(terms, C.c_double), _p(mags, C.c_double),
                     _p(F, C.c_double) if forces else None)
    return terms, mags, (F.reshape(ol.n, 3) if forces else None)


def grid_points(og, pos, scale, w):
    """Per-point channel energies (n, C) and forces (n, 3)."""
    pos = _d(pos).reshape(-1, 3)
    scale = _d(scale).reshape(len(pos), og.nc)
    w = _d(w)
    e = np.zeros((len(pos), og.nc))
    F = np.zeros((len(pos), 3))
    lib().ora_grid_points(og.ref, len(pos), _p(pos, C.c_double),
                          _p(scale, C.c_double), _p(w, C.c_double),
                          _p(e, C.c_double), _p(F, C.c_double))
    return e, F


def energy_batch(og, ol, xs, w):
    """terms (N, 4+C), mags (N, 4+C), forces (N, n, 3) for configurations
    xs (N, n, 3) under per-configuration weights w (N, C)."""
    xs = _d(xs)
    N = xs.shape[0]
    w = _d(np.broadcast_to(w, (N, og.nc)))
    terms = np.zeros((N, 4 + og.nc))
    mags = np.zeros((N, 4 + og.nc))
    F = np.zeros((N, ol.n, 3))
    lib().ora_energy_batch(og.ref, ol.ref, N, _p(w, C.c_double),
                           _p(xs, C.c_double), _p(terms, C.c_double),
                           _p(mags, C.c_double), _p(F, C.c_double))
    return terms, mags, F


def verlet(og, ol, w, dt, nleap, x, v):
    x = _d(x).reshape(-1).copy()
    v = _d(v).reshape(-1).copy()
    H = np.zeros(2)
    terms = np.zeros(4 + og.nc)
    wd = _d(w)
    lib().ora_verlet(og.ref, ol.ref, _p(wd, C.c_double), float(dt), int(nleap),
                     _p(x, C.c_double), _p(v, C.c_double), _p(H, C.c_double),
                     _p(terms, C.c_double))
    return x.reshape(ol.n, 3), v.reshape(ol.n, 3), H, terms


def momenta(ol, T, seed, lig, rep, sweep):
    v = np.zeros(3 * ol.n)
    lib().ora_momenta(ol.ref, float(T), seed, lig, rep, sweep,
                      _p(v, C.c_double))
    return v.reshape(ol.n, 3)


def components(og, ol, xs):
    xs = _d(xs)
    N = xs.shape[0]
    comps = np.zeros((N, 1 + og.nc))
    mags = np.zeros((N, 1 + og.nc))
    lib().ora_components(og.ref, ol.ref, N, _p(xs, C.c_double),
                         _p(comps, C.c_double), _p(mags, C.c_double))
    return comps, mags


def ukn(og, ol, xs):
    xs = _d(xs)
    N = xs.shape[0]
    out = np.zeros((ol.K, N))
    lib().ora_ukn(og.ref, ol.ref, ol.K, _p(ol.T, C.c_double),
                  _p(ol.w, C.c_double), N, _p(xs, C.c_double),
                  _p(out, C.c_double))
    return out


class Sampler:
    """Replica-exchange HMC for one ligand, run entirely by the oracle.

    State: x (R, n, 3) float64, state_of_replica, replica_of_state, comps
    (R, 1+C), sweep counter.  One call of sweep() = one HMC move for every
    replica, then (if due) one exchange attempt sweep, then (if due) one
    recorded sample per state, then counter += 1.
    """

    def __init__(self, og, ol, seed, lig_id=0, x0=None):
        self.og, self.ol = og, ol
        self.seed, self.lig = int(seed), int(lig_id)
        K = ol.K
        self.R = K
        x0 = np.asarray(x0, np.float64)
        self.x = np.ascontiguousarray(x0.reshape(K, ol.n, 3).copy())
        self.state = np.arange(K, dtype=np.int32)
        self.rep_of_state = np.arange(K, dtype=np.int32)
        self.comps, _ = components(og, ol, self.x)
        self.sweep_count = 0
        self.hmc_acc = np.zeros(K, np.int64)
        self.hmc_try = np.zeros(K, np.int64)
        self.ex_acc = np.zeros(max(K - 1, 1), np.int64)
        self.ex_try = np.zeros(max(K - 1, 1), np.int64)
        self.samples_x = []
        self.samples_c = []
        self.samples_state = []

    def hmc(self, nleap):
        og, ol = self.og, self.ol
        acc = np.zeros(self.R, np.int32)
        dH = np.zeros(self.R)
        lnu = np.zeros(self.R)
        lib().ora_hmc_sweep(og.ref, ol.ref, ol.K, _p(ol.T, C.c_double),
                            _p(ol.w, C.c_double), _p(ol.dt, C.c_double),
                            self.seed, self.lig, self.R, self.sweep_count,
                            int(nleap), _p(self.x, C.c_double),
                            _p(self.state, C.c_int),
                            _p(self.comps, C.c_double), _p(acc, C.c_int),
                            _p(dH, C.c_double), _p(lnu, C.c_double))
        for r in range(self.R):
            self.hmc_try[self.state[r]] += 1
            self.hmc_acc[self.state[r]] += acc[r]
        return acc, dH, lnu

    def exchange(self, scheme=0, max_sep=1, n_sweeps=1):
        """n_sweeps exchange sweeps in a row at the current counter (the
        paper ends each iteration with 25); sweep j draws with replica
        field j."""
        ol = self.ol
        for j in range(int(n_sweeps)):
            lib().ora_exchange(ol.K, self.og.nc, _p(ol.T, C.c_double),
                               _p(ol.w, C.c_double), self.seed, self.lig,
                               self.sweep_count, scheme, max_sep, j,
                               _p(self.comps, C.c_double),
                               _p(self.state, C.c_int),
                               _p(self.rep_of_state, C.c_int),
                               _p(self.ex_acc, C.c_int64),
                               _p(self.ex_try, C.c_int64))

    def record(self):
        for k in range(self.ol.K):
            r = self.rep_of_state[k]
            self.samples_x.append(self.x[r].copy())
            self.samples_c.append(self.comps[r].copy())
            self.samples_state.append(k)

    def sweep(self, nleap, exchange_every=1, sample_every=0, scheme=0,
              max_sep=1, exchange_sweeps=1):
        out = self.hmc(nleap)
        s = self.sweep_count
        if exchange_every > 0 and s % exchange_every == 0:
            self.exchange(scheme, max_sep, max(int(exchange_sweeps), 1))
        if sample_every > 0 and (s + 1) % sample_every == 0:
            self.record()
        self.sweep_count += 1
        return out


def num_threads():
    return lib().ora_num_threads()


def set_num_threads(t):
    lib().ora_set_num_threads(int(t))
