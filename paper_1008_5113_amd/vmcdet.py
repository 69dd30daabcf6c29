"""ctypes binding of libvmcdet.so (argument marshalling only).

Every step of the determinant-ratio path runs in the HIP library; this module
only converts numpy / torch arguments to the C-ABI declared in
``include/vmcdet.h``.  There is no CPU fallback: importing the binding without
the built library raises ``ImportError``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VMCDET_LIB") or os.path.join(_HERE, "libvmcdet.so")

VMC_OK = 0
VMC_EINVAL = -1
VMC_ENOMEM = -2
VMC_EHIP = -3
VMC_ENOCONV = -4
VMC_ESINGULAR = -5
VMC_ECAPACITY = -6
VMC_ESTATE = -7

PREC_FP64 = 0
PREC_MIXED = 1

FLAG_ACCEPTED = 1
FLAG_REORDERED = 2
FLAG_REFACTORED = 4
FLAG_CONVERGED = 8
FLAG_SINGULAR = 16
FLAG_CAPACITY = 32
FLAG_TRIG_N = 64
FLAG_TRIG_NOCONV = 128
FLAG_TRIG_ITERS = 256
FLAG_TRIG_FORCED = 512
FLAG_NOCONV = 1024

TEST_ZERO_RATIO = 1
TEST_FIRST_SOLVE_ONE_ITER = 2
TEST_ILU_FAST_SMALL = 4

PHASE_NAMES = ["prepare", "lsolve", "usolve", "updates", "spmv", "ortho", "solution", "resid64",
               "accept", "refactor", "reorder", "launch"]
WALL_CLOCK_HZ = 100e6  # device wall clock (s_memrealtime) on CDNA3/CDNA4

EXPORTED = [
    "vmc_default_params", "vmc_create", "vmc_build_slater", "vmc_ilutp", "vmc_det_ratio",
    "vmc_accept", "vmc_run_steps", "vmc_run_sweeps", "vmc_sync", "vmc_get_dims",
    "vmc_get_state", "vmc_get_stats", "vmc_last_error", "vmc_destroy", "vmc_phase_bench",
    "vmc_run_steps_graph", "vmc_autotune", "vmc_kinetic_energy", "vmc_run_steps_energy",
    "vmc_sm_prepare", "vmc_sm_prepare_static", "vmc_sm_run_steps", "vmc_sm_get_inverse",
]
PHASE_BENCH = {"spmv": 0, "lsolve": 1, "usolve": 2, "updates": 3, "resid64": 4, "ilutp": 5}


class VmcParams(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("gmres_maxit", ctypes.c_int32),
        ("gmres_rtol", ctypes.c_double),
        ("droptol", ctypes.c_double),
        ("permtol", ctypes.c_double),
        ("lfil", ctypes.c_int32),
        ("m_max", ctypes.c_int32),
        ("n_thresh", ctypes.c_double),
        ("iter_factor", ctypes.c_double),
        ("iter_min_solves", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double),
        ("refine_tol", ctypes.c_double),
        ("refine_maxit", ctypes.c_int32),
        ("step", ctypes.c_double),
        ("row_cap", ctypes.c_int32),
        ("force_reorder_every", ctypes.c_int32),
        ("plain_stop", ctypes.c_int32),
        ("refactor_cost", ctypes.c_double),
        ("ilu_work_cap", ctypes.c_int32),
        ("ilu_drop_norm", ctypes.c_int32),
        ("energy_tol", ctypes.c_double),
        ("device_ptrs", ctypes.c_int32),
        ("test_knobs", ctypes.c_int32),
    ]


class VmcWalkerInit(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("lattice", ctypes.c_int32 * 3),
        ("a", ctypes.c_double),
        ("site_margin", ctypes.c_double),
        ("sites", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
        ("orbital_kind", ctypes.c_int32),
        ("p_scale", ctypes.c_double),
        ("p_sigma", ctypes.c_double),
        ("cutoff", ctypes.c_double),
        ("pos0", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("n_basis", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("basis", (ctypes.c_double * 3) * 4),
    ]


class VmcStepRecord(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("walker", ctypes.c_int32),
        ("particle", ctypes.c_int32),
        ("new_pos", ctypes.c_double * 3),
        ("ratio", ctypes.c_double),
        ("log_abs_ratio", ctypes.c_double),
        ("u_acc", ctypes.c_double),
        ("N", ctypes.c_double),
        ("resid", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("inner_solves", ctypes.c_int32),
    ]


STEP_RECORD_DTYPE = np.dtype([
    ("step", np.int64), ("walker", np.int32), ("particle", np.int32), ("new_pos", np.float64, (3,)),
    ("ratio", np.float64), ("log_abs_ratio", np.float64), ("u_acc", np.float64), ("N", np.float64),
    ("resid", np.float64), ("iters", np.int32), ("flags", np.int32), ("refinements", np.int32),
    ("inner_solves", np.int32),
])
assert STEP_RECORD_DTYPE.itemsize == ctypes.sizeof(VmcStepRecord) == 96


class VmcStateView(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in [
        "pos", "row_particle", "col_site", "reorder_row", "reorder_col", "a_len", "a_col", "a_val",
        "l_len", "l_col", "l_val", "u_len", "u_col", "u_val", "u_diag", "ilu_perm", "step",
        "n_updates"]]


class VmcStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("accepted", ctypes.c_int64), ("solves", ctypes.c_int64),
        ("iters", ctypes.c_int64), ("reorders", ctypes.c_int64), ("refactors", ctypes.c_int64),
        ("nonconverged", ctypes.c_int64), ("inner_solves", ctypes.c_int64),
        ("refine_passes", ctypes.c_int64), ("update_sum", ctypes.c_int64),
        ("phase_ticks", ctypes.c_int64 * 12),
        ("max_N", ctypes.c_double), ("sum_N", ctypes.c_double),
        ("update_entries", ctypes.c_double), ("refactor_cost", ctypes.c_double),
        ("status", ctypes.c_int32), ("ilu_retries", ctypes.c_int32),
    ]


class VmcTuneInfo(ctypes.Structure):
    _fields_ = [
        ("ilutp_us_mean", ctypes.c_double), ("update_ns_per_entry", ctypes.c_double),
        ("refactor_cost_mean", ctypes.c_double), ("step_us_min", ctypes.c_double),
        ("step_us_max", ctypes.c_double), ("from_cache", ctypes.c_int32),
        ("trial_steps", ctypes.c_int32),
    ]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libvmcdet.so not built at {path}; run paper_1008_5113_amd/build.py")
    # torch (which provides the device buffers of the logging calls) ships its
    # own HIP runtime under the same soname.  Loading torch first makes the
    # library bind to that one runtime; loaded the other way round, the process
    # ends up with two runtimes and whichever initialises second finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.vmc_default_params.argtypes = [ctypes.POINTER(VmcParams)]
    lib.vmc_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(VmcParams), i32,
                               ctypes.POINTER(VmcWalkerInit), P]
    lib.vmc_build_slater.argtypes = [P, P, i32]
    lib.vmc_ilutp.argtypes = [P, P, i32, i32]
    lib.vmc_det_ratio.argtypes = [P, P, i32, P, P, P, P]
    lib.vmc_accept.argtypes = [P, P, i32, P, P]
    lib.vmc_run_steps.argtypes = [P, i32, P, ctypes.c_int64]
    lib.vmc_run_sweeps.argtypes = [P, i32, P, ctypes.c_int64]
    lib.vmc_sync.argtypes = [P]
    lib.vmc_get_dims.argtypes = [P, i32, P, P, P]
    lib.vmc_get_state.argtypes = [P, i32, ctypes.POINTER(VmcStateView)]
    lib.vmc_get_stats.argtypes = [P, P]
    lib.vmc_last_error.argtypes = [P]
    lib.vmc_last_error.restype = ctypes.c_char_p
    lib.vmc_destroy.argtypes = [P]
    lib.vmc_phase_bench.argtypes = [P, i32, i32]
    lib.vmc_run_steps_graph.argtypes = [P, i32, P, ctypes.c_int64]
    lib.vmc_autotune.argtypes = [P, ctypes.c_char_p, i32, ctypes.POINTER(VmcTuneInfo)]
    lib.vmc_kinetic_energy.argtypes = [P, P, i32, i32, i32, P, P]
    lib.vmc_run_steps_energy.argtypes = [P, i32, P, ctypes.c_int64, P, i32]
    lib.vmc_sm_prepare.argtypes = [P, ctypes.c_double]
    lib.vmc_sm_prepare_static.argtypes = [P, ctypes.c_double]
    lib.vmc_sm_run_steps.argtypes = [P, i32, P, ctypes.c_int64]
    lib.vmc_sm_get_inverse.argtypes = [P, i32, P]
    for name in EXPORTED:
        if name != "vmc_last_error":
            getattr(lib, name).restype = i32
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class VmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vmcdet status {status}: {msg}")
        self.status = status


def default_params(**kw) -> VmcParams:
    p = VmcParams()
    lib().vmc_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def params_from_workload(wp, **kw) -> VmcParams:
    """VmcParams from a ``workloads.Params``."""
    base = dict(precision=PREC_MIXED if wp.mixed else PREC_FP64, gmres_maxit=wp.gmres_maxit,
                gmres_rtol=wp.gmres_rtol, droptol=wp.droptol, permtol=wp.permtol, lfil=wp.lfil,
                m_max=wp.m_max, n_thresh=wp.n_thresh, iter_factor=wp.iter_factor,
                iter_min_solves=wp.iter_min_solves, inner_rtol=wp.inner_rtol,
                refine_tol=wp.refine_tol, refine_maxit=wp.refine_maxit, step=wp.step,
                ilu_work_cap=getattr(wp, "ilu_work_cap", 0),
                ilu_drop_norm=getattr(wp, "ilu_drop_norm", 0),
                plain_stop=int(getattr(wp, "plain_stop", False)))
    base.update(kw)
    return default_params(**base)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """A set of walkers on one GPU stream (owns the library context)."""

    def __init__(self, systems, walkers, params: VmcParams, stream=None):
        """systems: list of objects with lattice, a, sites, sigma, kind, p_scale, p_sigma,
        cutoff, site_margin() and optionally basis (fractional site offsets per cell);
        walkers: list of (system index, pos0, seed)."""
        self._keep = []
        n_w = len(walkers)
        inits = (VmcWalkerInit * n_w)()
        margins = {}
        for k, (si, pos0, seed) in enumerate(walkers):
            s = systems[si]
            if si not in margins:
                margins[si] = s.site_margin()
            sites = np.ascontiguousarray(s.sites, dtype=np.float64)
            sigma = np.ascontiguousarray(s.sigma, dtype=np.float64)
            pos = np.ascontiguousarray(pos0, dtype=np.float64)
            # the library copies n*3, n and n*3 doubles from these arrays
            n = sites.shape[0] if sites.ndim == 2 else -1
            if sites.shape != (n, 3) or sigma.shape != (n,) or pos.shape != (n, 3):
                raise ValueError(f"walker {k}: sites {sites.shape}, sigma {sigma.shape} and positions "
                                 f"{pos.shape} must be (n, 3), (n,) and (n, 3)")
            self._keep += [sites, sigma, pos]
            w = inits[k]
            w.n = sites.shape[0]
            w.lattice[0], w.lattice[1], w.lattice[2] = s.lattice
            w.a = s.a
            w.site_margin = margins[si]
            w.sites = sites.ctypes.data
            w.sigma = sigma.ctypes.data
            w.orbital_kind = s.kind
            w.p_scale = s.p_scale
            w.p_sigma = s.p_sigma
            w.cutoff = s.cutoff
            w.pos0 = pos.ctypes.data
            w.seed = int(seed)
            basis = getattr(s, "basis", None)
            if basis is not None:
                if not 1 <= len(basis) <= 4:
                    raise ValueError("a lattice cell holds 1 to 4 sites")
                w.n_basis = len(basis)
                for b, off in enumerate(basis):
                    for c in range(3):
                        w.basis[b][c] = float(off[c])
        self.params = params
        self.n_walkers = n_w
        self.ns = [inits[k].n for k in range(n_w)]
        self._stream = stream
        h = ctypes.c_void_p()
        st = lib().vmc_create(ctypes.byref(h), ctypes.byref(params), n_w, inits,
                              ctypes.c_void_p(stream) if stream else None)
        self._keep = []
        if st != VMC_OK:
            raise VmcError(st, lib().vmc_last_error(None).decode())
        self.h = h

    @classmethod
    def from_instance(cls, inst, params: Optional[VmcParams] = None, walkers=None, stream=None, **kw):
        ws = inst.walkers if walkers is None else [inst.walkers[k] for k in walkers]
        p = params if params is not None else params_from_workload(inst.params, **kw)
        return cls(inst.systems, [(w.system, w.pos0, w.seed) for w in ws], p, stream)

    def _check(self, st: int):
        if st != VMC_OK:
            raise VmcError(st, lib().vmc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().vmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _wl(walkers):
        if walkers is None:
            return None, None
        w = np.ascontiguousarray(walkers, dtype=np.int32)
        return w, len(w)

    def build_slater(self, walkers=None):
        w, cnt = self._wl(walkers)
        self._check(lib().vmc_build_slater(self.h, _ptr(w), cnt or 0))

    def ilutp(self, reorder: bool = True, walkers=None):
        w, cnt = self._wl(walkers)
        self._check(lib().vmc_ilutp(self.h, _ptr(w), cnt or 0, 1 if reorder else 0))

    def det_ratio(self, walkers=None, particles=None, new_pos=None, check=True):
        w, cnt = self._wl(walkers)
        count = cnt if w is not None else self.n_walkers
        ratio = np.zeros(count, dtype=np.float64)
        info = np.zeros(count, dtype=STEP_RECORD_DTYPE)
        part = None if particles is None else np.ascontiguousarray(particles, dtype=np.int32).reshape(-1)
        pos = None if new_pos is None else np.ascontiguousarray(new_pos, dtype=np.float64).reshape(-1)
        # the library reads count particles and 3*count coordinates
        if (part is not None and part.size != count) or (pos is not None and pos.size != 3 * count):
            raise ValueError(f"{count} walkers need {count} particles and {3 * count} coordinates")
        st = lib().vmc_det_ratio(self.h, _ptr(w), count, _ptr(part), _ptr(pos), _ptr(ratio),
                                 info.ctypes.data_as(ctypes.c_void_p))
        if check:
            self._check(st)
        return ratio, info

    def det_ratio_device(self, ratio_ptr: int, info_ptr: Optional[int] = None,
                         particle_ptr: Optional[int] = None, new_pos_ptr: Optional[int] = None):
        """vmc_det_ratio in device-pointer mode (vmc_params.device_ptrs set at
        creation): every walker, device arrays given by address, no
        synchronisation (errors surface at sync())."""
        vp = lambda x: ctypes.c_void_p(x) if x else None  # noqa: E731
        self._check(lib().vmc_det_ratio(self.h, None, 0, vp(particle_ptr), vp(new_pos_ptr), vp(ratio_ptr),
                                         vp(info_ptr)))

    def accept_device(self, decisions_ptr: Optional[int] = None, accepted_ptr: Optional[int] = None):
        """vmc_accept in device-pointer mode: every walker, device arrays by
        address (uint8 decisions, or None for the Metropolis rule), no
        synchronisation."""
        vp = lambda x: ctypes.c_void_p(x) if x else None  # noqa: E731
        self._check(lib().vmc_accept(self.h, None, 0, vp(decisions_ptr), vp(accepted_ptr)))

    def accept(self, walkers=None, decisions=None):
        w, cnt = self._wl(walkers)
        count = cnt if w is not None else self.n_walkers
        dec = None if decisions is None else np.ascontiguousarray(decisions, dtype=np.uint8).reshape(-1)
        if dec is not None and dec.size != count:
            raise ValueError(f"{count} walkers need {count} decisions")
        out = np.zeros(count, dtype=np.uint8)
        self._check(lib().vmc_accept(self.h, _ptr(w), count, _ptr(dec), _ptr(out)))
        return out.astype(bool)

    def run_steps(self, steps: int, log_device_ptr: Optional[int] = None, log_cap: int = 0,
                  graph: bool = False):
        fn = lib().vmc_run_steps_graph if graph else lib().vmc_run_steps
        self._check(fn(self.h, int(steps), ctypes.c_void_p(log_device_ptr) if log_device_ptr else None,
                       int(log_cap)))

    def run_steps_logged(self, steps: int, graph: bool = False, log_walkers: Optional[int] = None):
        """Run and return the step log as a numpy structured array [walker, step]
        of the first log_walkers walkers (all by default)."""
        import torch
        nlog = self.n_walkers if log_walkers is None else max(1, min(int(log_walkers), self.n_walkers))
        cap = nlog * steps
        buf = torch.empty(cap * STEP_RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self.run_steps(steps, buf.data_ptr(), cap, graph=graph)
        self.sync()
        arr = buf.cpu().numpy().view(STEP_RECORD_DTYPE)
        return arr.reshape(nlog, steps)

    def kinetic_energy(self, walkers=None, p_begin: int = 0, p_end: Optional[int] = None,
                       terms: bool = False):
        """Kinetic energy per particle of the listed walkers (see vmc_kinetic_energy).
        Returns the energies, and with terms=True also the list of per-particle
        term arrays (particle ids p_begin..p_end-1 of each walker)."""
        ws = list(range(self.n_walkers)) if walkers is None else [int(w) for w in walkers]
        hi = (1 << 30) if p_end is None else int(p_end)
        wl_arr = np.asarray(ws, dtype=np.int32)
        e = np.zeros(len(ws))
        lens = [max(0, min(hi, self.ns[w]) - min(int(p_begin), min(hi, self.ns[w]))) for w in ws]
        t = np.zeros(max(1, sum(lens))) if terms else None
        self._check(lib().vmc_kinetic_energy(self.h, _ptr(wl_arr), len(ws), int(p_begin), hi,
                                             _ptr(e), _ptr(t)))
        if not terms:
            return e
        out, o = [], 0
        for L in lens:
            out.append(t[o:o + L].copy())
            o += L
        return e, out

    def run_steps_energy(self, steps: int, energy_cap: int, log: bool = False,
                         log_walkers: Optional[int] = None):
        """Run `steps` persistent steps, sampling the kinetic energy at every sweep
        end.  Returns the energies [walker, energy_cap] (NaN where no sample was
        taken) and, with log=True, the step log [walker, step] of the first
        log_walkers walkers (all by default)."""
        import torch
        en = torch.full((self.n_walkers * energy_cap,), float("nan"), dtype=torch.float64, device="cuda")
        # the fill runs on torch's stream; the library's kernels on the context's
        torch.cuda.synchronize()
        buf, cap = None, 0
        nlog = self.n_walkers if log_walkers is None else min(int(log_walkers), self.n_walkers)
        if log:
            cap = nlog * steps
            buf = torch.empty(max(1, cap) * STEP_RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self._check(lib().vmc_run_steps_energy(self.h, int(steps), buf.data_ptr() if log else None, cap,
                                               en.data_ptr(), int(energy_cap)))
        self.sync()
        energies = en.cpu().numpy().reshape(self.n_walkers, energy_cap)
        if not log:
            return energies
        recs = buf.cpu().numpy().view(STEP_RECORD_DTYPE)[:cap]
        return energies, recs.reshape(nlog, steps)

    def sm_prepare(self, tol: float = 1e-13):
        """Explicit inverses for the standard algorithm (see vmc_sm_prepare)."""
        self._check(lib().vmc_sm_prepare(self.h, float(tol)))

    def sm_prepare_static(self, tol: float = 1e-13):
        """vmc_sm_prepare into the library's static device scratch (no device
        allocation; see vmc_sm_prepare_static)."""
        self._check(lib().vmc_sm_prepare_static(self.h, float(tol)))

    def sm_run_steps(self, steps: int, log: bool = False):
        """Steps by the standard algorithm; with log=True returns the step log
        [walker, step]."""
        import torch
        if not log:
            self._check(lib().vmc_sm_run_steps(self.h, int(steps), None, 0))
            return None
        cap = self.n_walkers * steps
        buf = torch.empty(cap * STEP_RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self._check(lib().vmc_sm_run_steps(self.h, int(steps), buf.data_ptr(), cap))
        self.sync()
        return buf.cpu().numpy().view(STEP_RECORD_DTYPE).reshape(self.n_walkers, steps)

    def sm_inverse(self, walker: int) -> np.ndarray:
        """Walker's stored inverse as B[j, p] = (A^{-1})_{jp} (site j, particle p)."""
        n = self.ns[walker]
        out = np.zeros((n, n))
        self._check(lib().vmc_sm_get_inverse(self.h, int(walker), _ptr(out)))
        return out.T.copy()

    def autotune(self, trial_steps: int = 100, cache_path: Optional[str] = None) -> dict:
        """Cost-balance thresholds and launch order (see vmc_autotune)."""
        info = VmcTuneInfo()
        self._check(lib().vmc_autotune(self.h, cache_path.encode() if cache_path else None,
                                       int(trial_steps), ctypes.byref(info)))
        return {f[0]: getattr(info, f[0]) for f in VmcTuneInfo._fields_}

    def phase_bench(self, phase: str, reps: int):
        self._check(lib().vmc_phase_bench(self.h, PHASE_BENCH[phase], int(reps)))

    def sync(self):
        self._check(lib().vmc_sync(self.h))

    def dims(self, walker: int):
        n, W, F = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().vmc_get_dims(self.h, walker, ctypes.byref(n), ctypes.byref(W), ctypes.byref(F)))
        return n.value, W.value, F.value

    def state(self, walker: int, factors: bool = False) -> dict:
        n, W, F = self.dims(walker)
        out = dict(
            pos=np.zeros((n, 3)), row_particle=np.zeros(n, np.int32), col_site=np.zeros(n, np.int32),
            reorder_row=np.zeros(n, np.int32), reorder_col=np.zeros(n, np.int32),
            a_len=np.zeros(n, np.int32), a_col=np.zeros((n, W), np.int32), a_val=np.zeros((n, W)),
            ilu_perm=np.zeros(n, np.int32), step=np.zeros(1, np.int64), n_updates=np.zeros(1, np.int32))
        if factors:
            out.update(l_len=np.zeros(n, np.int32), l_col=np.zeros((n, F), np.int32),
                       l_val=np.zeros((n, F)), u_len=np.zeros(n, np.int32),
                       u_col=np.zeros((n, F), np.int32), u_val=np.zeros((n, F)), u_diag=np.zeros(n))
        v = VmcStateView()
        for k, arr in out.items():
            setattr(v, k, arr.ctypes.data)
        self._check(lib().vmc_get_state(self.h, walker, ctypes.byref(v)))
        out["step"] = int(out["step"][0])
        out["n_updates"] = int(out["n_updates"][0])
        return out

    def stats(self):
        arr = (VmcStats * self.n_walkers)()
        self._check(lib().vmc_get_stats(self.h, ctypes.cast(arr, ctypes.c_void_p)))
        keys = [f[0] for f in VmcStats._fields_ if f[0] not in ("pad", "phase_ticks")]
        out = []
        for i in range(self.n_walkers):
            d = {k: getattr(arr[i], k) for k in keys}
            d["phase_ticks"] = list(arr[i].phase_ticks)
            out.append(d)
        return out
