"""ctypes binding of libbpmf (include/bpmf.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpmf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bpmf.h")

BPMF_OK = 0
_ERRORS = {-1: "BPMF_E_INVAL", -2: "BPMF_E_NOMEM", -3: "BPMF_E_HIP",
           -4: "BPMF_E_STATE", -5: "BPMF_E_UNIMPL"}


class BPMFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("n_channels", C.c_int), ("origin", C.c_double * 3),
                ("spacing", C.c_double), ("transform", C.POINTER(C.c_int))]


class _LigandDesc(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("mass", C.POINTER(C.c_double)),
                ("scale", C.POINTER(C.c_double)),
                ("n_bonds", C.c_int), ("bond_ij", C.POINTER(C.c_int)),
                ("bond_k_r0", C.POINTER(C.c_double)),
                ("n_angles", C.c_int), ("angle_ijk", C.POINTER(C.c_int)),
                ("angle_k_t0", C.POINTER(C.c_double)),
                ("n_tors", C.c_int), ("tors_ijkl", C.POINTER(C.c_int)),
                ("tors_v_n_g", C.POINTER(C.c_double)),
                ("site_center", C.c_double * 3), ("d0", C.c_double),
                ("k_restraint", C.c_double), ("n_states", C.c_int),
                ("T", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("dt_fs", C.POINTER(C.c_double)),
                ("x0", C.POINTER(C.c_float)), ("sample_capacity", C.c_int)]


class _SweepArgs(C.Structure):
    _fields_ = [("n_sweeps", C.c_int), ("n_leapfrog", C.c_int),
                ("exchange_every", C.c_int), ("exchange_scheme", C.c_int),
                ("max_sep", C.c_int), ("sample_every", C.c_int),
                ("pose_move_every", C.c_int), ("external_moves", C.c_int),
                ("external_k_max", C.c_int), ("external_sigma", C.c_double),
                ("exchange_sweeps", C.c_int)]


class _InitArgs(C.Structure):
    _fields_ = [("ligand_id", C.c_int), ("kind", C.c_int),
                ("T_hot", C.c_double), ("T_cold", C.c_double),
                ("speed", C.c_double), ("n_trials", C.c_int),
                ("n_leapfrog", C.c_int), ("dt_start", C.c_double),
                ("dt_min", C.c_double), ("max_dt_rounds", C.c_int),
                ("max_selections", C.c_int), ("n_conf", C.c_int),
                ("n_com", C.c_int), ("n_orient", C.c_int),
                ("max_states", C.c_int)]


class _InitResult(C.Structure):
    _fields_ = [("n_states", C.c_int), ("reached_target", C.c_int),
                ("n_selections", C.c_int), ("n_runs", C.c_int),
                ("n_removed", C.c_int), ("n_trace", C.c_int),
                ("alpha", C.POINTER(C.c_double)), ("T", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("dt", C.POINTER(C.c_double)),
                ("acc", C.POINTER(C.c_double)),
                ("pacc", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)),
                ("x", C.POINTER(C.c_float)),
                ("trace", C.POINTER(C.c_double)), ("trace_cap", C.c_int)]


class _PairDesc(C.Structure):
    _fields_ = [("charge", C.POINTER(C.c_double)),
                ("lj_sigma", C.POINTER(C.c_double)),
                ("lj_eps", C.POINTER(C.c_double)),
                ("gb_radius", C.POINTER(C.c_double)),
                ("gb_scale", C.POINTER(C.c_double)),
                ("n_exclusions", C.c_int), ("exclusions", C.POINTER(C.c_int)),
                ("n_pairs14", C.c_int), ("pairs14", C.POINTER(C.c_int)),
                ("lj14", C.c_double), ("el14", C.c_double),
                ("eps_solute", C.c_double), ("eps_solvent", C.c_double),
                ("sa_gamma", C.c_double), ("probe_radius", C.c_double)]


TRACE_FIELDS = 10
SCHEDULE_LINEAR, SCHEDULE_SOFT = 0, 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def exported_names():
    """Function names declared in include/bpmf.h."""
    with open(HEADER) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"BPMF_API\s+[\w\s\*]+?\b(bpmf_\w+)\s*\(",
                                 txt)))


EXPORTED = exported_names() if os.path.exists(HEADER) else []

_lib = None


def library():
    """Load libbpmf.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("BPMF_LIB", LIB_PATH)
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, "
            "gfx950).  There is no fallback implementation.")
    L = C.CDLL(path)
    vp, dp, fp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_void_p, \
        C.POINTER(C.c_int)
    i64p = C.POINTER(C.c_int64)
    sig = {
        "bpmf_create": [C.POINTER(C.c_void_p), C.c_int, C.c_uint64, vp,
                        ALLOC_FN, FREE_FN, vp],
        "bpmf_destroy": [vp],
        "bpmf_sync": [vp],
        "bpmf_grid_upload": [vp, C.POINTER(_GridDesc), C.POINTER(C.c_float)],
        "bpmf_ligand_setup": [vp, C.POINTER(_LigandDesc), ip],
        "bpmf_hmc_sweep": [vp, C.POINTER(_SweepArgs)],
        "bpmf_exchange": [vp, C.c_int, C.c_int, C.c_int, C.c_int],
        "bpmf_energy_matrix": [vp, C.c_int, vp, C.c_int64, vp, C.c_int64],
        "bpmf_energy_matrix_batch": [vp, C.c_int, ip, C.POINTER(C.c_void_p),
                                     i64p, C.POINTER(C.c_void_p), i64p],
        "bpmf_energy_matrix_batch_noalloc": [
            vp, C.c_int, ip, C.POINTER(C.c_void_p), i64p,
            C.POINTER(C.c_void_p), i64p],
        "bpmf_mbar": [vp, vp, C.c_int, C.c_int64, C.c_int64, i64p, C.c_double,
                      C.c_int, dp, dp, ip, C.c_int],
        "bpmf_mbar_batch": [vp, C.c_int, C.POINTER(C.c_void_p), ip, i64p, i64p,
                            i64p, C.c_double, C.c_int, dp, dp, ip, C.c_int],
        "bpmf_evaluate": [vp, C.c_int, vp, C.c_int64, vp, vp, vp],
        "bpmf_grid_eval": [vp, vp, vp, C.c_int64, dp, vp, vp],
        "bpmf_get_replicas": [vp, C.c_int, C.POINTER(C.c_float), ip, dp,
                              C.POINTER(C.c_uint64)],
        "bpmf_set_replicas": [vp, C.c_int, C.POINTER(C.c_float), ip, dp,
                              C.c_uint64],
        "bpmf_get_stats": [vp, C.c_int, i64p, i64p, i64p, i64p, i64p],
        "bpmf_get_samples": [vp, C.c_int, i64p, C.POINTER(C.c_float), dp],
        "bpmf_reset_samples": [vp, C.c_int],
        "bpmf_set_timing": [vp, C.c_int, C.c_int],
        "bpmf_set_waves": [vp, C.c_int],
        "bpmf_set_graph": [vp, C.c_int],
        "bpmf_autotune": [vp, C.c_int, C.c_int, dp, ip],
        "bpmf_get_round_trips": [vp, C.c_int, C.POINTER(C.c_int64)],
        "bpmf_set_ligand_waves": [vp, C.c_int, C.c_int],
        "bpmf_set_task_order": [vp, C.c_int],
        "bpmf_get_task_order": [vp, ip],
        "bpmf_proposal_setup": [vp, C.c_int, ip, C.c_int, ip,
                                C.POINTER(C.c_float)],
        "bpmf_proposal_params": [vp, C.c_int, C.POINTER(C.c_float),
                                 C.POINTER(C.c_float)],
        "bpmf_pose_features": [vp, C.c_int, vp, C.c_int64, vp, vp],
        "bpmf_proposal_forward": [vp, C.c_int, vp, C.c_int64, vp],
        "bpmf_proposal_grad": [vp, C.c_int, vp, vp, C.c_int64, vp, dp],
        "bpmf_proposal_train": [vp, C.c_int, vp, vp, C.c_int64, C.c_int,
                                C.c_int, C.c_double, dp],
        "bpmf_pose_move": [vp, C.c_int, C.c_int],
        "bpmf_get_pose_stats": [vp, C.c_int, i64p, i64p, dp],
        "bpmf_external_move": [vp, C.c_int, C.c_int, C.c_int, C.c_double],
        "bpmf_get_external_stats": [vp, C.c_int, i64p, i64p],
        "bpmf_get_waves": [vp, C.c_int, ip],
        "bpmf_get_timing": [vp, C.c_int, dp, i64p],
        "bpmf_ligand_info": [vp, C.c_int, ip, ip, ip, ip],
        "bpmf_set_states": [vp, C.c_int, dp, dp, dp],
        "bpmf_hmc_sweep_ligand": [vp, C.c_int, C.POINTER(_SweepArgs)],
        "bpmf_place_poses": [vp, C.c_int, vp, C.c_int, C.c_int, C.c_int,
                             C.c_int64, C.c_int64, vp],
        "bpmf_protocol_state": [C.c_double, C.c_int, C.c_int, C.c_double,
                                C.c_double, dp, dp],
        "bpmf_protocol_sigmas": [dp, C.c_int64, C.c_int, C.c_double, C.c_int,
                                 C.c_double, C.c_double, dp],
        "bpmf_protocol_next_alpha": [C.c_double, dp, C.c_int, C.c_double,
                                     C.c_double, C.c_double, dp],
        "bpmf_protocol_next_temperature": [C.c_double, C.c_double,
                                           C.c_double, C.c_double, dp],
        "bpmf_protocol_sir": [dp, C.c_int64, C.c_int, C.c_uint64, C.c_int,
                              C.c_int, i64p],
        "bpmf_protocol_adapt_dt": [C.c_double, C.c_double, C.c_double, dp, ip],
        "bpmf_protocol_mean_pacc": [dp, dp, dp, dp, C.c_int64, dp],
        "bpmf_protocol_insert": [dp, C.c_int, dp, C.c_double, C.c_int, dp, ip],
        "bpmf_detect_equilibration": [dp, C.c_int64, C.c_int, i64p, dp, dp],
        "bpmf_initialize_ladder": [vp, C.POINTER(_InitArgs),
                                   C.POINTER(_InitResult)],
        "bpmf_pair_setup": [vp, C.c_int, C.POINTER(_PairDesc)],
        "bpmf_pair_sample": [vp, C.c_int, C.c_int],
        "bpmf_pair_evaluate": [vp, C.c_int, vp, C.c_int64, vp, vp],
        "bpmf_version": [],
        "bpmf_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.bpmf_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != BPMF_OK:
        msg = library().bpmf_last_error().decode(errors="replace")
        raise BPMFError(rc, msg)


def _pd(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _pf(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


# -- ladder initialisation: host-side steps (no context, no device) ----------
def protocol_state(alpha, kind, n_channels, T_hot, T_cold):
    T = C.c_double(0.0)
    w = np.zeros(n_channels)
    _check(library().bpmf_protocol_state(float(alpha), int(kind),
                                         int(n_channels), float(T_hot),
                                         float(T_cold), C.byref(T), _pd(w)))
    return T.value, w


def protocol_sigmas(comps, alpha, kind, T_hot, T_cold):
    comps = np.ascontiguousarray(comps, np.float64)
    out = np.zeros(3)
    _check(library().bpmf_protocol_sigmas(_pd(comps), comps.shape[0],
                                          comps.shape[1] - 1, float(alpha),
                                          int(kind), float(T_hot),
                                          float(T_cold), _pd(out)))
    return out


def protocol_next_alpha(alpha, sigma, kind, speed, T_hot, T_cold):
    sg = np.ascontiguousarray(sigma, np.float64)
    out = C.c_double(0.0)
    _check(library().bpmf_protocol_next_alpha(float(alpha), _pd(sg), int(kind),
                                              float(speed), float(T_hot),
                                              float(T_cold), C.byref(out)))
    return out.value


def protocol_next_temperature(T, sigma_U, speed, T_target):
    out = C.c_double(0.0)
    _check(library().bpmf_protocol_next_temperature(
        float(T), float(sigma_U), float(speed), float(T_target),
        C.byref(out)))
    return out.value


def protocol_sir(log_w, n_draw, seed, ligand_id, state):
    lw = np.ascontiguousarray(log_w, np.float64)
    idx = np.zeros(int(n_draw), np.int64)
    _check(library().bpmf_protocol_sir(
        _pd(lw), lw.shape[0], int(n_draw), int(seed), int(ligand_id),
        int(state), idx.ctypes.data_as(C.POINTER(C.c_int64))))
    return idx


def protocol_adapt_dt(dt, acc, dt_min):
    nd = C.c_double(0.0)
    done = C.c_int(0)
    _check(library().bpmf_protocol_adapt_dt(float(dt), float(acc),
                                            float(dt_min), C.byref(nd),
                                            C.byref(done)))
    return nd.value, bool(done.value)


def protocol_mean_pacc(uk_x, uk1_x, uk_y, uk1_y):
    a = [np.ascontiguousarray(v, np.float64) for v in (uk_x, uk1_x, uk_y,
                                                       uk1_y)]
    out = C.c_double(0.0)
    _check(library().bpmf_protocol_mean_pacc(*[_pd(v) for v in a],
                                             a[0].shape[0], C.byref(out)))
    return out.value


def protocol_insert(alpha, pacc, threshold=0.4):
    al = np.ascontiguousarray(alpha, np.float64)
    pa = np.ascontiguousarray(pacc, np.float64)
    out = np.zeros(2 * len(al))
    K = C.c_int(0)
    _check(library().bpmf_protocol_insert(_pd(al), len(al), _pd(pa),
                                          float(threshold), len(out),
                                          _pd(out), C.byref(K)))
    return out[:K.value].copy()


def detect_equilibration(a, n_candidates=100):
    a = np.ascontiguousarray(a, np.float64)
    t0 = C.c_int64(0)
    g = C.c_double(0.0)
    ne = C.c_double(0.0)
    _check(library().bpmf_detect_equilibration(_pd(a), a.shape[0],
                                               int(n_candidates),
                                               C.byref(t0), C.byref(g),
                                               C.byref(ne)))
    return t0.value, g.value, ne.value


class Context:
    """One libbpmf context on a GPU, ordered on a torch stream and allocating
    through torch's caching allocator."""

    def __init__(self, seed: int, device: int = 0, stream=None,
                 torch_allocator: bool = True):
        import torch
        self._torch = torch
        self._lib = library()
        self.device = int(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(self.device)
        self._keep = []
        if torch_allocator:
            self._alloc = ALLOC_FN(self._alloc_cb)
            self._free = FREE_FN(self._free_cb)
        else:
            self._alloc = ALLOC_FN(0)
            self._free = FREE_FN(0)
        h = C.c_void_p()
        _check(self._lib.bpmf_create(C.byref(h), self.device, int(seed),
                                     C.c_void_p(self.stream.cuda_stream),
                                     self._alloc, self._free, None))
        self._h = h
        self.n_channels = None
        self.ligands = []

    # -- allocator callbacks -------------------------------------------------
    def _alloc_cb(self, size, user):
        try:
            return self._torch.cuda.caching_allocator_alloc(
                int(size), self.device, self.stream)
        except Exception:  # out of memory -> NULL -> BPMF_E_NOMEM
            return None

    def _free_cb(self, ptr, user):
        self._torch.cuda.caching_allocator_delete(ptr)

    # -- lifecycle ------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.bpmf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(self._lib.bpmf_sync(self._h))

    # -- grid -----------------------------------------------------------------
    def grid_upload(self, nodes, origin, spacing, transform):
        nodes = np.ascontiguousarray(nodes, np.float32)
        nz, ny, nx, nc = nodes.shape
        tr = np.ascontiguousarray(transform, np.int32)
        d = _GridDesc(nx, ny, nz, nc, (C.c_double * 3)(*map(float, origin)),
                      float(spacing), _pi(tr))
        _check(self._lib.bpmf_grid_upload(self._h, C.byref(d), _pf(nodes)))
        self.n_channels = nc

    # -- ligands --------------------------------------------------------------
    def ligand_setup(self, lig, sample_capacity: int = 0) -> int:
        """`lig` provides n_atoms, mass, scale, bonds, bond_par, angles,
        angle_par, tors, tors_par, site_center, d0, k_restraint, T, w, dt, x0
        (see include/bpmf.h for meaning and layout)."""
        arrs = dict(
            mass=np.ascontiguousarray(lig.mass, np.float64),
            scale=np.ascontiguousarray(lig.scale, np.float64),
            bij=np.ascontiguousarray(lig.bonds, np.int32).reshape(-1),
            bpar=np.ascontiguousarray(lig.bond_par, np.float64).reshape(-1),
            aijk=np.ascontiguousarray(lig.angles, np.int32).reshape(-1),
            apar=np.ascontiguousarray(lig.angle_par, np.float64).reshape(-1),
            tijkl=np.ascontiguousarray(lig.tors, np.int32).reshape(-1),
            tpar=np.ascontiguousarray(lig.tors_par, np.float64).reshape(-1),
            T=np.ascontiguousarray(lig.T, np.float64),
            w=np.ascontiguousarray(lig.w, np.float64),
            dt=np.ascontiguousarray(lig.dt, np.float64),
            x0=np.ascontiguousarray(lig.x0, np.float32))
        a = arrs
        d = _LigandDesc(int(lig.n_atoms), _pd(a["mass"]), _pd(a["scale"]),
                        len(a["bij"]) // 2, _pi(a["bij"]), _pd(a["bpar"]),
                        len(a["aijk"]) // 3, _pi(a["aijk"]), _pd(a["apar"]),
                        len(a["tijkl"]) // 4, _pi(a["tijkl"]), _pd(a["tpar"]),
                        (C.c_double * 3)(*map(float, lig.site_center)),
                        float(lig.d0), float(lig.k_restraint), len(a["T"]),
                        _pd(a["T"]), _pd(a["w"]), _pd(a["dt"]), _pf(a["x0"]),
                        int(sample_capacity))
        out = C.c_int(-1)
        _check(self._lib.bpmf_ligand_setup(self._h, C.byref(d),
                                           C.byref(out)))
        self.ligands.append(dict(n=int(lig.n_atoms), K=len(a["T"])))
        return out.value

    # -- sampling -------------------------------------------------------------
    def hmc_sweep(self, n_sweeps, n_leapfrog, exchange_every=1,
                  exchange_scheme=0, max_sep=1, sample_every=0,
                  pose_move_every=0, external_moves=0, external_k_max=0,
                  external_sigma=0.6, exchange_sweeps=1):
        a = _SweepArgs(int(n_sweeps), int(n_leapfrog), int(exchange_every),
                       int(exchange_scheme), int(max_sep), int(sample_every),
                       int(pose_move_every), int(external_moves),
                       int(external_k_max), float(external_sigma),
                       int(exchange_sweeps))
        _check(self._lib.bpmf_hmc_sweep(self._h, C.byref(a)))

    def exchange(self, ligand_id=-1, scheme=0, max_sep=1, n_sweeps=1):
        _check(self._lib.bpmf_exchange(self._h, int(ligand_id), int(scheme),
                                       int(max_sep), int(n_sweeps)))

    # -- u_kn, MBAR -----------------------------------------------------------
    def n_records(self, ligand_id):
        """Number of sample records so far (each holds one sample per
        state)."""
        nr = C.c_int64(0)
        _check(self._lib.bpmf_get_samples(self._h, int(ligand_id),
                                          C.byref(nr), None, None))
        return int(nr.value)

    def energy_matrix(self, ligand_id, samples=None, n_samples=None, out=None):
        """u_kn (K x N float64 CUDA tensor) for device samples (N, n, 3)
        float32, or for the recorded samples when samples is None (all of
        them, K x records, unless n_samples says otherwise)."""
        torch = self._torch
        K = self.ligands[ligand_id]["K"]
        if samples is not None:
            assert samples.is_cuda and samples.dtype == torch.float32 and \
                samples.is_contiguous()
            N = samples.shape[0]
            ptr = samples.data_ptr()
        else:
            N = (K * self.n_records(ligand_id) if n_samples is None
                 else int(n_samples))
            ptr = None
        if out is None:
            out = torch.empty((K, N), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        assert out.is_cuda and out.dtype == torch.float64 and out.stride(1) == 1
        _check(self._lib.bpmf_energy_matrix(self._h, int(ligand_id), ptr, N,
                                            out.data_ptr(), out.stride(0)))
        return out

    def energy_matrix_batch(self, ligand_ids, samples=None, n_samples=None,
                            outs=None, noalloc=False):
        """u_kn of several ligands in one call.  samples: None (recorded
        samples of every ligand, n_samples[i] each, or all of them when
        n_samples or its entry is None) or a list of device
        tensors (N_i, n_i, 3) float32 / None; outs: optional list of K_i x
        N_i float64 tensors.  noalloc: call the entry point that allocates
        nothing (bpmf_energy_matrix_batch_noalloc; give `outs` so that the
        binding allocates nothing either).  Returns the list of u_kn
        tensors."""
        torch = self._torch
        m = len(ligand_ids)
        ids = np.ascontiguousarray(ligand_ids, np.int32)
        ptrs = (C.c_void_p * max(m, 1))()
        uptrs = (C.c_void_p * max(m, 1))()
        ns = np.zeros(max(m, 1), np.int64)
        lds = np.zeros(max(m, 1), np.int64)
        res = []
        for i, lid in enumerate(ligand_ids):
            x = None if samples is None else samples[i]
            if x is not None:
                assert x.is_cuda and x.dtype == torch.float32 and \
                    x.is_contiguous()
                ns[i] = x.shape[0]
                ptrs[i] = x.data_ptr()
            K = self.ligands[lid]["K"]
            if x is None:
                ns[i] = (K * self.n_records(lid)
                         if n_samples is None or n_samples[i] is None
                         else int(n_samples[i]))
            u = outs[i] if outs is not None else torch.empty(
                (K, int(ns[i])), dtype=torch.float64,
                device=f"cuda:{self.device}")
            assert u.is_cuda and u.dtype == torch.float64 and \
                u.stride(1) == 1
            uptrs[i] = u.data_ptr()
            lds[i] = u.stride(0)
            res.append(u)
        fn = (self._lib.bpmf_energy_matrix_batch_noalloc if noalloc else
              self._lib.bpmf_energy_matrix_batch)
        _check(fn(
            self._h, m, _pi(ids), ptrs,
            ns.ctypes.data_as(C.POINTER(C.c_int64)), uptrs,
            lds.ctypes.data_as(C.POINTER(C.c_int64))))
        return res

    def mbar(self, ukn, N_k, tol=1e-10, max_iter=100, f_init=None):
        """Returns (f, var, n_iter): f[K] with f[0] = 0, var[k] = asymptotic
        variance of f_k - f_0.  f_init: optional initial guess (K)."""
        torch = self._torch
        assert ukn.is_cuda and ukn.dtype == torch.float64 and ukn.stride(1) == 1
        K, N = ukn.shape
        Nk = np.ascontiguousarray(N_k, np.int64)
        f = np.zeros(K) if f_init is None else \
            np.array(f_init, dtype=np.float64).reshape(K).copy()
        var = np.zeros(K)
        it = C.c_int(0)
        _check(self._lib.bpmf_mbar(self._h, ukn.data_ptr(), K, N,
                                   ukn.stride(0),
                                   Nk.ctypes.data_as(C.POINTER(C.c_int64)),
                                   float(tol), int(max_iter), _pd(f), _pd(var),
                                   C.byref(it), int(f_init is not None)))
        return f, var, it.value

    def mbar_batch(self, ukns, N_ks, tol=1e-10, max_iter=100, f_init=None):
        """MBAR for several independent problems in one call (each solved
        exactly as `mbar` solves it alone).  ukns: list of K_p x N_p float64
        device matrices; N_ks: list of sample counts; f_init: None, or a
        list with one initial guess (or None) per problem.  Returns a list
        of (f, var, n_iter)."""
        torch = self._torch
        P = len(ukns)
        assert len(N_ks) == P
        Ks = np.zeros(P, np.int32)
        Ns = np.zeros(P, np.int64)
        lds = np.zeros(P, np.int64)
        ptrs = (C.c_void_p * max(P, 1))()
        for p, u in enumerate(ukns):
            assert u.is_cuda and u.dtype == torch.float64 and u.stride(1) == 1
            Ks[p], Ns[p] = u.shape
            lds[p] = u.stride(0)
            ptrs[p] = u.data_ptr()
        Nk = np.concatenate([np.asarray(n, np.int64).reshape(-1)
                             for n in N_ks]) if P else np.zeros(0, np.int64)
        assert Nk.size == Ks.sum()
        off = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int64)
        f = np.zeros(int(Ks.sum()))
        warm = f_init is not None and any(x is not None for x in f_init)
        if warm:
            for p in range(P):
                # a problem without a guess starts from zero
                if f_init[p] is not None:
                    f[off[p]:off[p + 1]] = np.asarray(
                        f_init[p], np.float64).reshape(Ks[p])
        var = np.zeros_like(f)
        its = np.zeros(max(P, 1), np.int32)
        _check(self._lib.bpmf_mbar_batch(
            self._h, P, ptrs, Ks.ctypes.data_as(C.POINTER(C.c_int)),
            Ns.ctypes.data_as(C.POINTER(C.c_int64)),
            lds.ctypes.data_as(C.POINTER(C.c_int64)),
            np.ascontiguousarray(Nk).ctypes.data_as(C.POINTER(C.c_int64)),
            float(tol), int(max_iter), _pd(f), _pd(var),
            its.ctypes.data_as(C.POINTER(C.c_int)), int(warm)))
        return [(f[off[p]:off[p + 1]].copy(), var[off[p]:off[p + 1]].copy(),
                 int(its[p])) for p in range(P)]

    # -- direct evaluation ----------------------------------------------------
    def evaluate(self, ligand_id, x, w, forces=True):
        torch = self._torch
        n = self.ligands[ligand_id]["n"]
        nc = self.n_channels
        N = x.shape[0]
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        assert w.is_cuda and w.dtype == torch.float64 and w.is_contiguous()
        dev = f"cuda:{self.device}"
        terms = torch.empty((N, 4 + nc), dtype=torch.float64, device=dev)
        F = torch.empty((N, n, 3), dtype=torch.float32, device=dev) \
            if forces else None
        _check(self._lib.bpmf_evaluate(self._h, int(ligand_id), x.data_ptr(),
                                       N, w.data_ptr(), terms.data_ptr(),
                                       F.data_ptr() if forces else None))
        return terms, F

    def grid_eval(self, pos, scale, w, energy=None, force=None):
        torch = self._torch
        nc = self.n_channels
        N = pos.shape[0]
        dev = f"cuda:{self.device}"
        if energy is None:
            energy = torch.empty((N, nc), dtype=torch.float32, device=dev)
        if force is None:
            force = torch.empty((N, 3), dtype=torch.float32, device=dev)
        wd = np.ascontiguousarray(w, np.float64)
        _check(self._lib.bpmf_grid_eval(self._h, pos.data_ptr(),
                                        scale.data_ptr(), N, _pd(wd),
                                        energy.data_ptr(), force.data_ptr()))
        return energy, force

    # -- replica state ----------------------------------------------------------
    def get_replicas(self, ligand_id):
        L = self.ligands[ligand_id]
        K, n, nc = L["K"], L["n"], self.n_channels
        x = np.zeros((K, n, 3), np.float32)
        sor = np.zeros(K, np.int32)
        comps = np.zeros((K, 1 + nc))
        cnt = C.c_uint64(0)
        _check(self._lib.bpmf_get_replicas(self._h, int(ligand_id), _pf(x),
                                           _pi(sor), _pd(comps),
                                           C.byref(cnt)))
        return dict(x=x, state_of_replica=sor, comps=comps, counter=cnt.value)

    def set_replicas(self, ligand_id, x, state_of_replica, comps=None,
                     counter=0):
        x = np.ascontiguousarray(x, np.float32)
        sor = np.ascontiguousarray(state_of_replica, np.int32)
        cp = None if comps is None else np.ascontiguousarray(comps, np.float64)
        _check(self._lib.bpmf_set_replicas(self._h, int(ligand_id), _pf(x),
                                           _pi(sor),
                                           _pd(cp) if cp is not None else None,
                                           int(counter)))

    def get_stats(self, ligand_id):
        K = self.ligands[ligand_id]["K"]
        ha = np.zeros(K, np.int64)
        ht = np.zeros(K, np.int64)
        ea = np.zeros(max(K - 1, 1), np.int64)
        et = np.zeros(max(K - 1, 1), np.int64)
        nf = C.c_int64(0)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))  # noqa: E731
        _check(self._lib.bpmf_get_stats(self._h, int(ligand_id), p(ha), p(ht),
                                        p(ea), p(et), C.byref(nf)))
        return dict(hmc_acc=ha, hmc_try=ht, ex_acc=ea[:K - 1],
                    ex_try=et[:K - 1], nonfinite=nf.value)

    def get_round_trips(self, ligand_id):
        """Replica round trips 0 -> K-1 -> 0 since setup."""
        out = C.c_int64(0)
        _check(self._lib.bpmf_get_round_trips(self._h, int(ligand_id),
                                              C.byref(out)))
        return out.value

    def get_samples(self, ligand_id):
        L = self.ligands[ligand_id]
        K, n, nc = L["K"], L["n"], self.n_channels
        nr = C.c_int64(0)
        _check(self._lib.bpmf_get_samples(self._h, int(ligand_id),
                                          C.byref(nr), None, None))
        x = np.zeros((nr.value, K, n, 3), np.float32)
        comps = np.zeros((nr.value, K, 1 + nc))
        _check(self._lib.bpmf_get_samples(self._h, int(ligand_id),
                                          C.byref(nr), _pf(x), _pd(comps)))
        return x, comps

    # -- learned pose proposal ------------------------------------------------
    N_PARAMS, N_OUT, N_FEAT = 96872, 104, 16

    def proposal_setup(self, ligand_id, frame_atoms, cond_ijkl, params):
        fa = np.ascontiguousarray(frame_atoms, np.int32)
        cd = np.ascontiguousarray(cond_ijkl, np.int32).reshape(-1, 4)
        pr = np.ascontiguousarray(params, np.float32).reshape(-1)
        assert pr.size == self.N_PARAMS
        _check(self._lib.bpmf_proposal_setup(
            self._h, int(ligand_id), _pi(fa), len(cd),
            _pi(cd) if len(cd) else None, _pf(pr)))

    def proposal_params(self, ligand_id, new=None):
        out = np.zeros(self.N_PARAMS, np.float32)
        inp = None if new is None else np.ascontiguousarray(new, np.float32)
        _check(self._lib.bpmf_proposal_params(
            self._h, int(ligand_id), _pf(out),
            _pf(inp) if inp is not None else None))
        return out if new is None else None

    def pose_features(self, ligand_id, x):
        torch = self._torch
        N = x.shape[0]
        dev = f"cuda:{self.device}"
        f = torch.empty((N, self.N_FEAT), dtype=torch.float32, device=dev)
        p = torch.empty((N, 6), dtype=torch.float32, device=dev)
        _check(self._lib.bpmf_pose_features(self._h, int(ligand_id),
                                            x.data_ptr(), N, f.data_ptr(),
                                            p.data_ptr()))
        return f, p

    def proposal_forward(self, ligand_id, feats):
        torch = self._torch
        N = feats.shape[0]
        out = torch.empty((N, self.N_OUT), dtype=torch.float32,
                          device=f"cuda:{self.device}")
        _check(self._lib.bpmf_proposal_forward(self._h, int(ligand_id),
                                               feats.data_ptr(), N,
                                               out.data_ptr()))
        return out

    def proposal_grad(self, ligand_id, feats, poses):
        torch = self._torch
        g = torch.empty(self.N_PARAMS, dtype=torch.float32,
                        device=f"cuda:{self.device}")
        loss = C.c_double(0.0)
        _check(self._lib.bpmf_proposal_grad(self._h, int(ligand_id),
                                            feats.data_ptr(), poses.data_ptr(),
                                            feats.shape[0], g.data_ptr(),
                                            C.byref(loss)))
        return g, loss.value

    def proposal_train(self, ligand_id, feats, poses, batch, steps, lr,
                       losses=False):
        out = np.zeros(max(int(steps), 1))
        _check(self._lib.bpmf_proposal_train(
            self._h, int(ligand_id), feats.data_ptr(), poses.data_ptr(),
            feats.shape[0], int(batch), int(steps), float(lr),
            _pd(out) if losses else None))
        return out[:steps] if losses else None

    def pose_move(self, ligand_id=-1, rounds=1):
        _check(self._lib.bpmf_pose_move(self._h, int(ligand_id), int(rounds)))

    def external_move(self, ligand_id=-1, n_moves=1, k_max=1, sigma=0.6):
        """n_moves external moves of every replica in states < k_max."""
        _check(self._lib.bpmf_external_move(self._h, int(ligand_id),
                                            int(n_moves), int(k_max),
                                            float(sigma)))

    def get_external_stats(self, ligand_id):
        K = self.ligands[ligand_id]["K"]
        a = np.zeros(K, np.int64)
        t = np.zeros(K, np.int64)
        p = lambda v: v.ctypes.data_as(C.POINTER(C.c_int64))  # noqa: E731
        _check(self._lib.bpmf_get_external_stats(self._h, int(ligand_id),
                                                 p(a), p(t)))
        return dict(acc=a, tries=t)

    def get_pose_stats(self, ligand_id):
        K = self.ligands[ligand_id]["K"]
        a = np.zeros(K, np.int64)
        t = np.zeros(K, np.int64)
        la = np.zeros(K)
        p = lambda v: v.ctypes.data_as(C.POINTER(C.c_int64))  # noqa: E731
        _check(self._lib.bpmf_get_pose_stats(self._h, int(ligand_id), p(a),
                                             p(t), _pd(la)))
        return dict(acc=a, tries=t, last_ln_alpha=la)

    def autotune(self, n_sweeps=20, n_leapfrog=10, cache_path=None,
                 signature=None):
        """Pick the wavefronts per replica of the HMC sweep by timing every
        candidate on the ligands set up, then refine them per atom-count
        class and choose the workgroup order (state restored afterwards).
        With cache_path, the choice (the context-wide one, every ligand's
        and the order) is stored in / reused from a
        JSON file keyed by GPU architecture and `signature` (a string
        describing the workload).  Returns (chosen, {candidate: ms}) for
        the context-wide candidates."""
        import json
        import os
        arch = self._torch.cuda.get_device_properties(
            self.device).gcnArchName
        key = f"{arch}|{signature}"
        ids = range(len(self.ligands))
        if cache_path and signature and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
            hit = cache.get(key)
            if (hit and len(hit.get("waves", [])) == len(ids)
                    and "task_order" in hit):
                self.set_waves(hit["chosen"])
                for i, w in zip(ids, hit["waves"]):
                    self.set_ligand_waves(i, w)
                self.set_task_order(hit["task_order"])
                return hit["chosen"], hit["ms"]
        ms = np.zeros(5)
        ch = C.c_int(0)
        _check(self._lib.bpmf_autotune(self._h, int(n_sweeps),
                                       int(n_leapfrog), _pd(ms), C.byref(ch)))
        table = {str(w): float(m) for w, m in zip(("auto", 1, 2, 4, 8), ms)}
        if cache_path and signature:
            cache = {}
            if os.path.exists(cache_path):
                with open(cache_path) as fh:
                    cache = json.load(fh)
            cache[key] = {"chosen": ch.value, "ms": table,
                          "waves": [self.get_waves(i) for i in ids],
                          "task_order": self.get_task_order()}
            with open(cache_path, "w") as fh:
                json.dump(cache, fh, indent=1)
        return ch.value, table

    def set_graph(self, chunk):
        """Replay sweeps as hipGraphs of `chunk` sweeps (0 = plain)."""
        _check(self._lib.bpmf_set_graph(self._h, int(chunk)))

    def set_waves(self, waves):
        """Wavefronts per replica (1, 2, 4; 0 = automatic)."""
        _check(self._lib.bpmf_set_waves(self._h, int(waves)))

    def set_ligand_waves(self, ligand_id, waves):
        """A ligand's own wavefronts per replica (0 = the context-wide
        choice)."""
        _check(self._lib.bpmf_set_ligand_waves(self._h, int(ligand_id),
                                               int(waves)))

    def set_task_order(self, order):
        """Workgroup order of the sweep: 1 (default) heaviest ligands
        first, 0 ligand by ligand."""
        _check(self._lib.bpmf_set_task_order(self._h, int(order)))

    def get_task_order(self):
        v = C.c_int(0)
        _check(self._lib.bpmf_get_task_order(self._h, C.byref(v)))
        return v.value

    def get_waves(self, ligand_id):
        out = C.c_int(0)
        _check(self._lib.bpmf_get_waves(self._h, int(ligand_id),
                                        C.byref(out)))
        return out.value

    TIMER_HMC, TIMER_COMPONENTS, TIMER_TAIL, TIMER_GRID_EVAL = 0, 1, 2, 3

    def set_timing(self, enable=True, every=1):
        _check(self._lib.bpmf_set_timing(self._h, int(bool(enable)),
                                         int(every)))

    def get_timing(self, kernel):
        """(mean ms per bracketed launch, number of launches timed)."""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        _check(self._lib.bpmf_get_timing(self._h, int(kernel), C.byref(ms),
                                         C.byref(n)))
        return ms.value, n.value

    def reset_samples(self, ligand_id=-1):
        _check(self._lib.bpmf_reset_samples(self._h, int(ligand_id)))

    # -- intramolecular nonbonded / implicit solvent ----------------------------
    def pair_setup(self, ligand_id, p):
        """p: dict with charge, sigma, eps, rho, S (per atom), exclusions and
        pairs14 (k x 2), lj14, el14, eps_solute, eps_solvent, gamma,
        probe."""
        arr = {k: np.ascontiguousarray(p[k], np.float64)
               for k in ("charge", "sigma", "eps", "rho", "S")}
        ex = np.ascontiguousarray(p["exclusions"], np.int32).reshape(-1, 2)
        o4 = np.ascontiguousarray(p["pairs14"], np.int32).reshape(-1, 2)
        d = _PairDesc(_pd(arr["charge"]), _pd(arr["sigma"]), _pd(arr["eps"]),
                      _pd(arr["rho"]), _pd(arr["S"]), len(ex), _pi(ex),
                      len(o4), _pi(o4), float(p["lj14"]), float(p["el14"]),
                      float(p["eps_solute"]), float(p["eps_solvent"]),
                      float(p["gamma"]), float(p["probe"]))
        _check(self._lib.bpmf_pair_setup(self._h, int(ligand_id),
                                         C.byref(d)))

    def pair_evaluate(self, ligand_id, x, forces=True):
        torch = self._torch
        n = self.ligands[ligand_id]["n"]
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        N = x.shape[0]
        dev = f"cuda:{self.device}"
        terms = torch.empty((N, 4), dtype=torch.float64, device=dev)
        F = torch.empty((N, n, 3), dtype=torch.float32, device=dev) \
            if forces else None
        _check(self._lib.bpmf_pair_evaluate(
            self._h, int(ligand_id), x.data_ptr(), N, terms.data_ptr(),
            F.data_ptr() if forces else None))
        return terms, F

    # -- single-ligand control, ladder initialisation --------------------------
    def pair_sample(self, ligand_id, on=True):
        """Put the ligand's pair terms into its sampled energy (or take them
        out); pair_setup must have been called."""
        _check(self._lib.bpmf_pair_sample(self._h, int(ligand_id),
                                          1 if on else 0))

    def ligand_info(self, ligand_id):
        v = [C.c_int(0) for _ in range(4)]
        _check(self._lib.bpmf_ligand_info(self._h, int(ligand_id),
                                          *[C.byref(x) for x in v]))
        return dict(n_atoms=v[0].value, n_states=v[1].value,
                    n_channels=v[2].value, sample_capacity=v[3].value)

    def set_states(self, ligand_id, T, w, dt):
        T = np.ascontiguousarray(T, np.float64)
        w = np.ascontiguousarray(w, np.float64)
        dt = np.ascontiguousarray(dt, np.float64)
        _check(self._lib.bpmf_set_states(self._h, int(ligand_id), _pd(T),
                                         _pd(w), _pd(dt)))

    def hmc_sweep_ligand(self, ligand_id, n_sweeps, n_leapfrog,
                         exchange_every=1, exchange_scheme=0, max_sep=1,
                         sample_every=0, pose_move_every=0, external_moves=0,
                         external_k_max=0, external_sigma=0.6,
                         exchange_sweeps=1):
        a = _SweepArgs(int(n_sweeps), int(n_leapfrog), int(exchange_every),
                       int(exchange_scheme), int(max_sep), int(sample_every),
                       int(pose_move_every), int(external_moves),
                       int(external_k_max), float(external_sigma),
                       int(exchange_sweeps))
        _check(self._lib.bpmf_hmc_sweep_ligand(self._h, int(ligand_id),
                                               C.byref(a)))

    def place_poses(self, ligand_id, confs, n_com, n_orient, first=0,
                    count=None, out=None):
        torch = self._torch
        assert confs.is_cuda and confs.dtype == torch.float32 \
            and confs.is_contiguous()
        n_conf, n = confs.shape[0], confs.shape[1]
        total = n_conf * int(n_com) * int(n_orient)
        if count is None:
            count = total - int(first)
        if out is None:
            out = torch.empty((int(count), n, 3), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        _check(self._lib.bpmf_place_poses(
            self._h, int(ligand_id), confs.data_ptr(), int(n_conf),
            int(n_com), int(n_orient), int(first), int(count),
            out.data_ptr()))
        return out

    def initialize_ladder(self, ligand_id, kind, T_hot, T_cold, speed=0.2,
                          n_trials=200, n_leapfrog=10, dt_start=1.0,
                          dt_min=0.125, max_dt_rounds=8, max_selections=6,
                          n_conf=0, n_com=0, n_orient=0, max_states=256,
                          trace_cap=1024, want_x=True):
        info = self.ligand_info(ligand_id)
        K, n, nc = info["n_states"], info["n_atoms"], info["n_channels"]
        M = int(max_states)
        a = _InitArgs(int(ligand_id), int(kind), float(T_hot), float(T_cold),
                      float(speed), int(n_trials), int(n_leapfrog),
                      float(dt_start), float(dt_min), int(max_dt_rounds),
                      int(max_selections), int(n_conf), int(n_com),
                      int(n_orient), M)
        arr = dict(alpha=np.zeros(M), T=np.zeros(M), w=np.zeros((M, nc)),
                   dt=np.zeros(M), acc=np.zeros(M), pacc=np.zeros(M),
                   sigma=np.zeros((M, 3)),
                   trace=np.zeros((int(trace_cap), TRACE_FIELDS)))
        x = np.zeros((M, K, n, 3), np.float32) if want_x else None
        r = _InitResult()
        for k in ("alpha", "T", "w", "dt", "acc", "pacc", "sigma", "trace"):
            setattr(r, k, _pd(arr[k]))
        r.x = _pf(x) if want_x else None
        r.trace_cap = int(trace_cap)
        _check(self._lib.bpmf_initialize_ladder(self._h, C.byref(a),
                                                C.byref(r)))
        m = r.n_states
        out = {k: arr[k][:m].copy() for k in ("alpha", "T", "w", "dt", "acc",
                                              "pacc", "sigma")}
        out["trace"] = arr["trace"][:r.n_trace].copy()
        out["x"] = x[:m].copy() if want_x else None
        out.update(n_states=m, reached_target=bool(r.reached_target),
                   n_selections=r.n_selections, n_runs=r.n_runs,
                   n_removed=r.n_removed)
        return out
