"""Python binding of libsmcgw.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch supplies device memory
(tensors' data pointers) and the current HIP stream.  The functions mirror
the C ABI in include/smcgw.h.  Importing this module on a machine without
the built library raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import synth

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libsmcgw.so")

OK, WARN_FALLBACK = 0, 1
ERR_INVALID, ERR_SHAPE, ERR_HIP, ERR_OOM, ERR_NOT_INIT, ERR_STALL = -1, -2, -3, -4, -5, -6
MAX_BINS = 1 << 24   # frequency bins of one event (SMCGW_MAX_BINS)
NOALLOC_MAX_P = 16384   # particles of smcgw_loglike_grad_noalloc (SMCGW_NOALLOC_MAX_P)
PLAIN_FP64, MIXED = 0, 1
KERNEL_BINS, KERNEL_PREP, KERNEL_FINISH, KERNEL_NUTS, KERNEL_SMC, KERNEL_METRIC = 0, 1, 2, 3, 4, 5
OPT_NUTS_WAVES = 0
OPT_NUTS_PRIORITY = 1
OPT_NUTS_SLOTS_PER_CU = 2


class SmcgwError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {code} ({status_string(code)})")
        self.code = code


class EventDesc(C.Structure):
    _fields_ = [("f_low", C.c_double), ("df", C.c_double), ("n_bins", C.c_int32), ("n_det", C.c_int32),
                ("gmst", C.c_double), ("t_sun", C.c_double), ("mpc_m", C.c_double), ("c_light", C.c_double),
                ("pn_order", C.c_int32), ("reserved", C.c_int32)]


class Detector(C.Structure):
    _fields_ = [("lat", C.c_double), ("lon", C.c_double), ("az_x", C.c_double), ("az_y", C.c_double),
                ("radius", C.c_double)]


class Bounds(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("bnd", C.c_int32), ("prior", C.c_int32)]


class NutsParams(C.Structure):
    _fields_ = [("step", C.c_double), ("beta", C.c_double), ("max_delta_h", C.c_double),
                ("max_depth", C.c_int32), ("uturn", C.c_int32), ("seed", C.c_uint64), ("iteration", C.c_uint64),
                ("chol_per_particle", C.c_int32), ("reserved", C.c_int32), ("beta_device", C.c_void_p),
                ("state_device", C.c_void_p), ("run_size", C.c_int32), ("reserved2", C.c_int32)]


# Device run state and per-iteration record (smcgw_smc_iteration): entries of one run's state and of one
# record row.
STATE_SIZE = 8
ST_BETA, ST_LOGZ, ST_DLOGZ, ST_ITER, ST_NEXT, ST_DONE, ST_STALL = range(7)
HIST_SIZE = 8
H_BETA, H_LOGZ, H_DLOGZ, H_LEAPFROG, H_DEPTH, H_DIVERGENT, H_MM_FALLBACK, H_METRIC_FALLBACKS = range(8)
MAX_RUNS = 64


class SmcIterDesc(C.Structure):
    _fields_ = [("n_runs", C.c_int32), ("P", C.c_int32), ("D", C.c_int32), ("precision", C.c_int32),
                ("theta", C.c_void_p), ("logl", C.c_void_p), ("grad", C.c_void_p), ("ancestors", C.c_void_p),
                ("n_leapfrog", C.c_void_p), ("depth", C.c_void_p), ("divergent", C.c_void_p),
                ("accept_stat", C.c_void_p), ("inv_mass", C.c_void_p), ("chol", C.c_void_p),
                ("mm_status", C.c_void_p), ("chol_pp", C.c_void_p), ("metric_status", C.c_void_p),
                ("state", C.c_void_p), ("history", C.c_void_p), ("history_cap", C.c_int32),
                ("max_depth", C.c_int32), ("alpha", C.c_double), ("shrink", C.c_double), ("step", C.c_double),
                ("max_delta_h", C.c_double), ("seed", C.c_uint64), ("uturn", C.c_int32), ("nuts_form", C.c_int32)]
NUTS_PERSISTENT, NUTS_SWEEPS = 0, 1


_lib = None


def rb_edges(f_low: float, df: float, n_bins: int, eps: float) -> np.ndarray:
    """Grid indices of the relative-binning edges (host computation, no device needed)."""
    out = np.zeros(n_bins + 1, dtype=np.int32)
    m = lib().smcgw_rb_edges(f_low, df, n_bins, eps, out.ctypes.data_as(C.c_void_p), len(out))
    if m < 0:
        raise RuntimeError(f"smcgw_rb_edges: {lib().smcgw_status_string(m).decode()}")
    return out[:m].copy()


def _chol_mode(chol: torch.Tensor, P: int, D: int, n_runs: int = 0) -> int:
    """0 for one shared [D][D] factor (or, with n_runs independent runs, one [D][D] factor per run),
    1 for per-particle [P][D][D] factors."""
    _dev(chol, torch.float64, "chol")
    if tuple(chol.shape) == (D, D):
        return 0
    if tuple(chol.shape) == (P, D, D):
        return 1
    if n_runs > 0 and tuple(chol.shape) == (n_runs, D, D):
        return 0
    raise ValueError(f"chol must be [{D}][{D}] or [{P}][{D}][{D}], got {tuple(chol.shape)}")


def lib():
    """Load libsmcgw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: run `python -m paper_2601_02336_amd.build` "
                               "(or __graft_entry__.build()) first; there is no fallback path")
        L = C.CDLL(_LIB_PATH)
        vp, i, d, u64 = C.c_void_p, C.c_int, C.c_double, C.c_uint64
        L.smcgw_status_string.restype = C.c_char_p
        L.smcgw_status_string.argtypes = [i]
        L.smcgw_create.argtypes = [C.POINTER(vp), i, vp]
        L.smcgw_destroy.argtypes = [vp]
        L.smcgw_set_stream.argtypes = [vp, vp]
        L.smcgw_add_event.argtypes = [vp, C.POINTER(EventDesc), vp, vp, C.POINTER(Detector), C.POINTER(i)]
        L.smcgw_set_param_map.argtypes = [vp, i, vp, vp]
        L.smcgw_set_event_map.argtypes = [vp, vp]
        L.smcgw_set_prior.argtypes = [vp, i, C.POINTER(Bounds)]
        L.smcgw_set_target.argtypes = [vp, i, i, vp, i]
        L.smcgw_loglike_grad.argtypes = [vp, i, vp, vp, vp, vp, i]
        L.smcgw_waveform.argtypes = [vp, i, vp, vp]
        L.smcgw_target_loglike_grad.argtypes = [vp, i, vp, vp, vp, i]
        L.smcgw_mass_matrix.argtypes = [vp, i, i, vp, d, vp, vp, vp]
        L.smcgw_local_metric.argtypes = [vp, i, i, vp, d, vp, vp, vp, vp, vp]
        L.smcgw_ps_reweight_resample.argtypes = [vp, i, i, i, vp, vp, vp, vp, vp, d, u64, u64, vp, vp, vp, vp,
                                                 C.POINTER(d), C.POINTER(d)]
        L.smcgw_smc_reweight_resample_async.argtypes = [vp, i, i, d, d, u64, u64, vp, vp, vp, vp, vp, vp]
        L.smcgw_add_event_rb.argtypes = [vp, C.POINTER(EventDesc), vp, vp, C.POINTER(Detector), vp, d,
                                         C.POINTER(i), C.POINTER(i)]
        L.smcgw_rb_edges.argtypes = [d, d, i, d, vp, i]
        L.smcgw_recycle.argtypes = [vp, i, i, vp, vp, vp, u64, vp, vp, C.POINTER(C.c_int64), C.POINTER(d)]
        L.smcgw_nuts_step.argtypes = [vp, i, i, vp, vp, vp, vp, C.POINTER(NutsParams), vp, vp, i, vp, vp, vp, vp]
        L.smcgw_timing_enable.argtypes = [vp, i]
        L.smcgw_autotune_nuts.argtypes = [vp, i, i, vp, vp, vp, vp, C.POINTER(NutsParams), i, i, C.POINTER(i),
                                          C.POINTER(d)]
        L.smcgw_set_option.argtypes = [vp, i, C.c_int64]
        L.smcgw_timing_read.argtypes = [vp, i, C.POINTER(d), C.POINTER(C.c_int64)]
        L.smcgw_timing_intervals.argtypes = [vp, i, vp, vp, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.smcgw_smc_reweight_resample.argtypes = [vp, i, i, d, d, u64, u64, vp, vp, vp, vp, vp,
                                                  C.POINTER(d), C.POINTER(d)]
        L.smcgw_loglike_grad_noalloc.argtypes = [vp, i, vp, vp, vp, vp, i]
        L.smcgw_loglike_grad_tangent.argtypes = [vp, i, vp, vp, vp, vp]
        L.smcgw_nuts_step_sweeps.argtypes = [vp, i, i, vp, vp, vp, vp, C.POINTER(NutsParams), vp, vp, vp, vp, vp, i,
                                             C.POINTER(i)]
        L.smcgw_smc_iteration.argtypes = [vp, C.POINTER(SmcIterDesc)]
        L.smcgw_smc_graph_create.argtypes = [vp, C.POINTER(SmcIterDesc), C.POINTER(vp)]
        L.smcgw_graph_launch.argtypes = [vp, i]
        L.smcgw_graph_destroy.argtypes = [vp]
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().smcgw_status_string(code).decode()


def _check(fn: str, rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        raise SmcgwError(fn, rc)
    return rc


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")
    return t


class Context:
    """One library context on one device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = device
        self._h = C.c_void_p()
        with torch.cuda.device(device):
            s = torch.cuda.current_stream(device).cuda_stream
        _check("smcgw_create", lib().smcgw_create(C.byref(self._h), device, C.c_void_p(s)))
        self.events = []

    def close(self):
        if self._h:
            lib().smcgw_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        lib().smcgw_set_stream(self._h, C.c_void_p(s))

    def set_option(self, option: int, value: int):
        _check("smcgw_set_option", lib().smcgw_set_option(self._h, option, value))

    # ------------------------------------------------------------ timing
    def timing(self, *kernel_classes: int):
        """Record events around launches of the given kernel classes (none: off)."""
        mask = 0
        for k in kernel_classes:
            mask |= 1 << k
        _check("smcgw_timing_enable", lib().smcgw_timing_enable(self._h, mask))

    def timing_read(self, kernel_class: int):
        """(summed milliseconds, launches) of one kernel class since the last read."""
        ms = C.c_double()
        n = C.c_int64()
        _check("smcgw_timing_read", lib().smcgw_timing_read(self._h, kernel_class, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def timing_intervals(self, kernel_class: int, ref: "torch.cuda.Event", cap: int = 65536):
        """(start_ms, end_ms) arrays of one kernel class's launches since the last read, in ms after the
        recorded timing event ref (which may be shared by contexts on other streams of the device)."""
        start = np.zeros(cap)
        end = np.zeros(cap)
        n = C.c_int64()
        _check("smcgw_timing_intervals", lib().smcgw_timing_intervals(
            self._h, kernel_class, C.c_void_p(ref.cuda_event), start.ctypes.data, end.ctypes.data, cap,
            C.byref(n)))
        return start[:n.value], end[:n.value]

    # ------------------------------------------------------------ set-up
    def add_event(self, ev: "synth.Event") -> int:
        desc = EventDesc(ev.f_low, ev.df, ev.n, ev.n_det, ev.gmst, ev.t_sun, ev.mpc_m, ev.c_light, ev.pn_order, 0)
        dets = (Detector * ev.n_det)(*[Detector(*s.as_tuple()) for s in ev.sites])
        data = np.ascontiguousarray(ev.data_reim(), dtype=np.float64)
        psd = np.ascontiguousarray(ev.psd, dtype=np.float64)
        eid = C.c_int()
        self._stream()
        _check("smcgw_add_event", lib().smcgw_add_event(self._h, C.byref(desc), data.ctypes.data_as(C.c_void_p),
                                                        psd.ctypes.data_as(C.c_void_p), dets, C.byref(eid)))
        self.events.append(ev)
        return eid.value

    def add_event_rb(self, ev: "synth.Event", theta0: Sequence[float], eps: float = 0.1):
        """Relative-binning event around the fiducial point theta0 (11); returns (event id, edge count)."""
        desc = EventDesc(ev.f_low, ev.df, ev.n, ev.n_det, ev.gmst, ev.t_sun, ev.mpc_m, ev.c_light, ev.pn_order, 0)
        dets = (Detector * ev.n_det)(*[Detector(*s.as_tuple()) for s in ev.sites])
        data = np.ascontiguousarray(ev.data_reim(), dtype=np.float64)
        psd = np.ascontiguousarray(ev.psd, dtype=np.float64)
        th0 = np.ascontiguousarray(theta0, dtype=np.float64)
        if th0.shape != (11,):
            raise ValueError("theta0 holds the 11 source parameters")
        eid = C.c_int()
        ne = C.c_int()
        self._stream()
        _check("smcgw_add_event_rb", lib().smcgw_add_event_rb(
            self._h, C.byref(desc), data.ctypes.data_as(C.c_void_p), psd.ctypes.data_as(C.c_void_p), dets,
            th0.ctypes.data_as(C.c_void_p), eps, C.byref(eid), C.byref(ne)))
        self.events.append(ev)
        return eid.value, ne.value

    def set_event_map(self, event_of_particle: Optional[torch.Tensor]):
        """Device int32 [P] event index per particle for the sampler calls (kept alive here)."""
        if event_of_particle is not None:
            _dev(event_of_particle, torch.int32, "event_of_particle")
        self._event_map = event_of_particle
        _check("smcgw_set_event_map", lib().smcgw_set_event_map(self._h, _ptr(event_of_particle)))

    def set_param_map(self, param_index: Sequence[int], fixed11: Optional[Sequence[float]] = None):
        idx = np.ascontiguousarray(param_index, dtype=np.int32)
        fx = None if fixed11 is None else np.ascontiguousarray(fixed11, dtype=np.float64)
        _check("smcgw_set_param_map", lib().smcgw_set_param_map(
            self._h, len(idx), idx.ctypes.data_as(C.c_void_p), None if fx is None else fx.ctypes.data_as(C.c_void_p)))

    def set_prior(self, bounds):
        arr = (Bounds * len(bounds))(*[Bounds(b.lo, b.hi, b.bnd, b.prior) for b in bounds])
        _check("smcgw_set_prior", lib().smcgw_set_prior(self._h, len(bounds), arr))

    def set_target(self, kind: int, dim: int, params: Optional[Sequence[float]] = None):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        self._stream()
        _check("smcgw_set_target", lib().smcgw_set_target(
            self._h, kind, dim, None if p is None else p.ctypes.data_as(C.c_void_p), 0 if p is None else p.size))

    # ------------------------------------------------------------ hot path
    def loglike_grad(self, theta: torch.Tensor, logl: Optional[torch.Tensor] = None,
                     grad: Optional[torch.Tensor] = None, want_grad: bool = True,
                     event_of_particle: Optional[torch.Tensor] = None, precision: int = MIXED):
        theta = _dev(theta, torch.float64, "theta")
        P = theta.shape[0]
        if logl is None:
            logl = torch.empty(P, dtype=torch.float64, device=theta.device)
        if want_grad and grad is None:
            grad = torch.empty_like(theta)
        if event_of_particle is not None:
            _dev(event_of_particle, torch.int32, "event_of_particle")
        self._stream()
        _check("smcgw_loglike_grad", lib().smcgw_loglike_grad(
            self._h, P, _ptr(event_of_particle), _ptr(theta), _ptr(logl), _ptr(grad) if want_grad else None,
            precision))
        return (logl, grad) if want_grad else logl

    def loglike_grad_noalloc(self, theta: torch.Tensor, logl: torch.Tensor, grad: Optional[torch.Tensor],
                             event_of_particle: Optional[torch.Tensor] = None, precision: int = MIXED):
        """smcgw_loglike_grad_noalloc into caller-provided logl [P] and grad [P][D] (grad may be None):
        the library allocates nothing (at most NOALLOC_MAX_P particles)."""
        theta = _dev(theta, torch.float64, "theta")
        _dev(logl, torch.float64, "logl")
        if grad is not None:
            _dev(grad, torch.float64, "grad")
        if event_of_particle is not None:
            _dev(event_of_particle, torch.int32, "event_of_particle")
        self._stream()
        return lib().smcgw_loglike_grad_noalloc(self._h, theta.shape[0], _ptr(event_of_particle), _ptr(theta),
                                                _ptr(logl), _ptr(grad), precision)

    def loglike_grad_tangent(self, theta: torch.Tensor, logl: Optional[torch.Tensor] = None,
                             grad: Optional[torch.Tensor] = None, want_grad: bool = True,
                             event_of_particle: Optional[torch.Tensor] = None):
        """The plain comparison form (smcgw_loglike_grad_tangent): FP64 per-bin terms, gradient by forward-mode
        tangents."""
        theta = _dev(theta, torch.float64, "theta")
        P = theta.shape[0]
        if logl is None:
            logl = torch.empty(P, dtype=torch.float64, device=theta.device)
        if want_grad and grad is None:
            grad = torch.empty_like(theta)
        if event_of_particle is not None:
            _dev(event_of_particle, torch.int32, "event_of_particle")
        self._stream()
        _check("smcgw_loglike_grad_tangent", lib().smcgw_loglike_grad_tangent(
            self._h, P, _ptr(event_of_particle), _ptr(theta), _ptr(logl), _ptr(grad) if want_grad else None))
        return (logl, grad) if want_grad else logl

    def nuts_step_sweeps(self, theta: torch.Tensor, logl: torch.Tensor, grad: torch.Tensor, chol: torch.Tensor,
                         step: float, beta: float, seed: int, iteration: int, max_depth: int = 10,
                         uturn: bool = True, max_delta_h: float = 1000.0,
                         max_depth_per_particle: Optional[torch.Tensor] = None, sweeps_per_group: int = 8,
                         beta_device: Optional[torch.Tensor] = None, state: Optional[torch.Tensor] = None,
                         run_size: int = 0):
        """The plain comparison form of nuts_step (smcgw_nuts_step_sweeps): lockstep sweeps with the
        forward-mode plain likelihood, groups of sweeps replayed from a HIP graph.  Synchronises; returns the
        diagnostics dict with n_sweeps added."""
        theta = _dev(theta, torch.float64, "theta")
        P, D = theta.shape
        if beta_device is not None:
            _dev(beta_device, torch.float64, "beta_device")
        if state is not None:
            _dev(state, torch.float64, "state")
        n_runs = P // run_size if (state is not None and run_size > 0) else 0
        prm = NutsParams(step, 0.0 if (beta_device is not None or state is not None) else beta, max_delta_h,
                         max_depth, 1 if uturn else 0, seed, iteration, _chol_mode(chol, P, D, n_runs), 0,
                         _ptr(beta_device), _ptr(state), run_size if state is not None else 0, 0)
        dev = theta.device
        out = dict(depth=torch.empty(P, dtype=torch.int32, device=dev),
                   n_leapfrog=torch.empty(P, dtype=torch.int32, device=dev),
                   divergent=torch.empty(P, dtype=torch.uint8, device=dev),
                   accept_stat=torch.empty(P, dtype=torch.float64, device=dev))
        if max_depth_per_particle is not None:
            _dev(max_depth_per_particle, torch.int32, "max_depth_per_particle")
        n = C.c_int(0)
        self._stream()
        _check("smcgw_nuts_step_sweeps", lib().smcgw_nuts_step_sweeps(
            self._h, P, D, _ptr(theta), _ptr(logl), _ptr(grad), _ptr(chol), C.byref(prm),
            _ptr(max_depth_per_particle), _ptr(out["depth"]), _ptr(out["n_leapfrog"]), _ptr(out["divergent"]),
            _ptr(out["accept_stat"]), sweeps_per_group, C.byref(n)))
        out["n_sweeps"] = n.value
        return out

    def target_loglike_grad(self, theta: torch.Tensor, logl: Optional[torch.Tensor] = None,
                            grad: Optional[torch.Tensor] = None, precision: int = MIXED):
        """logL and gradient of the context's current target (GW or analytic)."""
        theta = _dev(theta, torch.float64, "theta")
        P = theta.shape[0]
        if logl is None:
            logl = torch.empty(P, dtype=torch.float64, device=theta.device)
        if grad is None:
            grad = torch.empty_like(theta)
        self._stream()
        _check("smcgw_target_loglike_grad", lib().smcgw_target_loglike_grad(
            self._h, P, _ptr(theta), _ptr(logl), _ptr(grad), precision))
        return logl, grad

    def waveform(self, event_id: int, theta11) -> torch.Tensor:
        ev = self.events[event_id]
        th = np.ascontiguousarray(theta11, dtype=np.float64)
        h = torch.empty((ev.n_det, ev.n, 2), dtype=torch.float64, device=f"cuda:{self.device}")
        self._stream()
        _check("smcgw_waveform", lib().smcgw_waveform(self._h, event_id, th.ctypes.data_as(C.c_void_p), _ptr(h)))
        return h

    def mass_matrix(self, theta: torch.Tensor, shrink: float = 0.0, status: Optional[torch.Tensor] = None):
        """(inv_mass, chol, rc).  With a device int32 `status` tensor the call does not synchronise:
        the fallback flag lands in status[0] and rc is OK."""
        theta = _dev(theta, torch.float64, "theta")
        P, D = theta.shape
        inv = torch.empty((D, D), dtype=torch.float64, device=theta.device)
        L = torch.empty_like(inv)
        if status is not None:
            _dev(status, torch.int32, "status")
        self._stream()
        rc = _check("smcgw_mass_matrix", lib().smcgw_mass_matrix(self._h, P, D, _ptr(theta), shrink, _ptr(inv),
                                                                 _ptr(L), _ptr(status)), allow=(OK, WARN_FALLBACK))
        return inv, L, rc

    def local_metric(self, theta: torch.Tensor, beta: float, fallback: Optional[torch.Tensor] = None,
                     fisher: bool = False, status: bool = True, beta_device: Optional[torch.Tensor] = None):
        """Per-particle metric factors chol [P][D][D] (lower Cholesky factor of (beta F + prior precision)^-1).
        beta_device (a one-element device float64 tensor) supplies beta from device memory instead.
        Returns (chol, fisher or None, status or None); asynchronous."""
        if beta_device is not None:
            _dev(beta_device, torch.float64, "beta_device")
            beta = 0.0
        theta = _dev(theta, torch.float64, "theta")
        P, D = theta.shape
        dev = theta.device
        L = torch.empty((P, D, D), dtype=torch.float64, device=dev)
        F = torch.empty((P, D, D), dtype=torch.float64, device=dev) if fisher else None
        st = torch.empty(P, dtype=torch.int32, device=dev) if status else None
        if fallback is not None:
            fallback = _dev(fallback, torch.float64, "fallback")
            if tuple(fallback.shape) != (D, D):
                raise ValueError("fallback must be [D][D]")
        self._stream()
        _check("smcgw_local_metric", lib().smcgw_local_metric(self._h, P, D, _ptr(theta), beta, _ptr(beta_device),
                                                              _ptr(fallback), _ptr(L), _ptr(F), _ptr(st)))
        return L, F, st

    def recycle(self, logl_pool: torch.Tensor, betas: Sequence[float], logz: Sequence[float], seed: int):
        """Sample recycling over the pool logl_pool [T][N] (device): returns (log weights [T*N], kept pool
        indices (device int32, increasing), Kish ESS).  Synchronises."""
        logl_pool = _dev(logl_pool, torch.float64, "logl_pool")
        T, N = logl_pool.shape
        b = np.ascontiguousarray(betas, dtype=np.float64)
        z = np.ascontiguousarray(logz, dtype=np.float64)
        if b.shape != (T,) or z.shape != (T,):
            raise ValueError("betas and logz need one entry per pooled iteration")
        logw = torch.empty(T * N, dtype=torch.float64, device=logl_pool.device)
        kept = torch.empty(T * N, dtype=torch.int32, device=logl_pool.device)
        nk = C.c_int64()
        ess = C.c_double()
        self._stream()
        _check("smcgw_recycle", lib().smcgw_recycle(self._h, T, N, _ptr(logl_pool), b.ctypes.data_as(C.c_void_p),
                                                    z.ctypes.data_as(C.c_void_p), seed, _ptr(logw), _ptr(kept),
                                                    C.byref(nk), C.byref(ess)))
        return logw, kept[:nk.value], ess.value

    def nuts_step(self, theta: torch.Tensor, logl: torch.Tensor, grad: torch.Tensor, chol: torch.Tensor,
                  step: float, beta: float, seed: int, iteration: int, max_depth: int = 10, uturn: bool = True,
                  max_delta_h: float = 1000.0, max_depth_per_particle: Optional[torch.Tensor] = None,
                  precision: int = MIXED, diagnostics: bool = True, work_hint: Optional[torch.Tensor] = None,
                  beta_device: Optional[torch.Tensor] = None):
        """One NUTS transition per particle; chol is one [D][D] factor of M^-1 or [P][D][D], one per particle.
        beta_device (a one-element device float64 tensor) supplies beta from device memory instead."""
        theta = _dev(theta, torch.float64, "theta")
        P, D = theta.shape
        if beta_device is not None:
            _dev(beta_device, torch.float64, "beta_device")
        prm = NutsParams(step, 0.0 if beta_device is not None else beta, max_delta_h, max_depth, 1 if uturn else 0,
                         seed, iteration, _chol_mode(chol, P, D), 0, _ptr(beta_device), None, 0, 0)
        dev = theta.device
        out = {}
        if diagnostics:
            # the kernel writes every particle's entry
            out = dict(depth=torch.empty(P, dtype=torch.int32, device=dev),
                       n_leapfrog=torch.empty(P, dtype=torch.int32, device=dev),
                       divergent=torch.empty(P, dtype=torch.uint8, device=dev),
                       accept_stat=torch.empty(P, dtype=torch.float64, device=dev))
        if max_depth_per_particle is not None:
            _dev(max_depth_per_particle, torch.int32, "max_depth_per_particle")
        if work_hint is not None:
            _dev(work_hint, torch.int32, "work_hint")
        self._stream()
        _check("smcgw_nuts_step", lib().smcgw_nuts_step(
            self._h, P, D, _ptr(theta), _ptr(logl), _ptr(grad), _ptr(chol), C.byref(prm),
            _ptr(max_depth_per_particle), _ptr(work_hint), precision, _ptr(out.get("depth")), _ptr(out.get("n_leapfrog")),
            _ptr(out.get("divergent")), _ptr(out.get("accept_stat"))))
        return out

    def autotune_nuts(self, theta: torch.Tensor, logl: torch.Tensor, grad: torch.Tensor, chol: torch.Tensor,
                      step: float, beta: float, seed: int, iteration: int, max_depth: int = 10, uturn: bool = True,
                      max_delta_h: float = 1000.0, precision: int = MIXED, trials: int = 3):
        """Pick the NUTS slot width by timing transitions of this batch (inputs untouched).
        Returns (best width, {width: median ms})."""
        theta = _dev(theta, torch.float64, "theta")
        P, D = theta.shape
        prm = NutsParams(step, beta, max_delta_h, max_depth, 1 if uturn else 0, seed, iteration,
                         _chol_mode(chol, P, D), 0, None, None, 0, 0)
        best = C.c_int(0)
        times = (C.c_double * 4)()
        self._stream()
        _check("smcgw_autotune_nuts", lib().smcgw_autotune_nuts(
            self._h, P, D, _ptr(theta), _ptr(logl), _ptr(grad), _ptr(chol), C.byref(prm), precision, trials,
            C.byref(best), times))
        return best.value, dict(zip((2, 4, 6, 8), list(times)))

    def smc_reweight_resample(self, theta: torch.Tensor, logl: torch.Tensor, grad: Optional[torch.Tensor],
                              beta_prev: float, alpha: float, seed: int, iteration: int,
                              ancestors: Optional[torch.Tensor] = None, carry: Optional[torch.Tensor] = None):
        theta = _dev(theta, torch.float64, "theta")
        P, D = theta.shape
        if ancestors is None:
            ancestors = torch.empty(P, dtype=torch.int32, device=theta.device)
        b = C.c_double()
        dz = C.c_double()
        self._stream()
        if carry is not None:
            _dev(carry, torch.int32, "carry")
        rc = lib().smcgw_smc_reweight_resample(self._h, P, D, beta_prev, alpha, seed, iteration, _ptr(theta),
                                               _ptr(logl), _ptr(grad), _ptr(carry), _ptr(ancestors), C.byref(b),
                                               C.byref(dz))
        _check("smcgw_smc_reweight_resample", rc)
        return b.value, dz.value, ancestors

    def ps_reweight_resample(self, theta_pool: torch.Tensor, logl_pool: torch.Tensor,
                             grad_pool: Optional[torch.Tensor], betas: Sequence[float], logz: Sequence[float],
                             alpha: float, seed: int, iteration: int, theta: torch.Tensor, logl: torch.Tensor,
                             grad: Optional[torch.Tensor], ancestors: Optional[torch.Tensor] = None):
        """Persistent-sampling step over a pool of T populations of N points: theta_pool [T*N][D], logl_pool [T*N]
        (device), betas/logz of the T populations.  Draws N points into theta/logl/grad; returns
        (beta_next, log Z(beta_next), ancestors).  Synchronises."""
        theta_pool = _dev(theta_pool, torch.float64, "theta_pool")
        _dev(logl_pool, torch.float64, "logl_pool")
        theta = _dev(theta, torch.float64, "theta")
        N, D = theta.shape
        T = len(betas)
        if len(logz) != T or logl_pool.numel() != T * N or theta_pool.shape != (T * N, D):
            raise ValueError("pool shapes do not match T populations of the population's size")
        b = np.ascontiguousarray(betas, dtype=np.float64)
        z = np.ascontiguousarray(logz, dtype=np.float64)
        if ancestors is None:
            ancestors = torch.empty(N, dtype=torch.int32, device=theta.device)
        bn = C.c_double()
        lz = C.c_double()
        self._stream()
        _check("smcgw_ps_reweight_resample", lib().smcgw_ps_reweight_resample(
            self._h, T, N, D, _ptr(theta_pool), _ptr(logl_pool), _ptr(grad_pool), b.ctypes.data_as(C.c_void_p),
            z.ctypes.data_as(C.c_void_p), alpha, seed, iteration, _ptr(theta), _ptr(logl), _ptr(grad),
            _ptr(ancestors), C.byref(bn), C.byref(lz)))
        return bn.value, lz.value, ancestors

    def smc_reweight_resample_async(self, theta: torch.Tensor, logl: torch.Tensor, grad: Optional[torch.Tensor],
                                    beta_prev: float, alpha: float, seed: int, iteration: int, out: torch.Tensor,
                                    ancestors: Optional[torch.Tensor] = None, carry: Optional[torch.Tensor] = None):
        """As smc_reweight_resample without synchronising: out (device float64 [2]) receives beta_next and the
        evidence increment when the queued work has run."""
        theta = _dev(theta, torch.float64, "theta")
        _dev(out, torch.float64, "out")
        if out.numel() < 2:
            raise ValueError("out needs two entries")
        P, D = theta.shape
        if ancestors is None:
            ancestors = torch.empty(P, dtype=torch.int32, device=theta.device)
        if carry is not None:
            _dev(carry, torch.int32, "carry")
        self._stream()
        _check("smcgw_smc_reweight_resample_async", lib().smcgw_smc_reweight_resample_async(
            self._h, P, D, beta_prev, alpha, seed, iteration, _ptr(theta), _ptr(logl), _ptr(grad), _ptr(carry),
            _ptr(ancestors), _ptr(out)))
        return ancestors


class Graph:
    """A captured SMC iteration (smcgw_smc_graph_create), replayed on the context's current stream."""

    def __init__(self, ctx: "Context", desc: SmcIterDesc):
        self._ctx = ctx
        self._h = C.c_void_p()
        ctx._stream()
        _check("smcgw_smc_graph_create", lib().smcgw_smc_graph_create(ctx._h, C.byref(desc), C.byref(self._h)))

    def launch(self, count: int = 1):
        self._ctx._stream()
        _check("smcgw_graph_launch", lib().smcgw_graph_launch(self._h, count))

    def close(self):
        if self._h:
            lib().smcgw_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SmcRuns:
    """Device buffers of n_runs independent SMC runs of P particles each (run r: rows [r P, (r+1) P)) and the
    whole-iteration call over them (smcgw_smc_iteration).  Run r draws with Philox key seed + r.  The runs'
    states (temperature, running log evidence, iteration index, done flag) and per-iteration records stay on
    the device; state() and history() copy them out."""

    def __init__(self, ctx: "Context", theta0: torch.Tensor, n_runs: int, *, alpha: float, step: float,
                 max_depth: int, shrink: float, seed: int, precision: int, metric: str = "population",
                 uturn: bool = True, max_delta_h: float = 1000.0, history_cap: int = 512,
                 nuts_form: int = NUTS_PERSISTENT):
        theta0 = _dev(theta0, torch.float64, "theta0")
        n, D = theta0.shape
        if n_runs < 1 or n_runs > MAX_RUNS or n % n_runs != 0:
            raise ValueError("theta0 must hold n_runs equal runs")
        if metric not in ("population", "local"):
            raise ValueError(f"unknown metric {metric!r}")
        dev = theta0.device
        P = n // n_runs
        self.ctx, self.n_runs, self.P, self.D = ctx, n_runs, P, D
        self.theta = theta0.clone()
        if nuts_form == NUTS_SWEEPS:   # the plain comparison form evaluates with its own likelihood
            self.logl, self.grad = ctx.loglike_grad_tangent(self.theta)
        else:
            self.logl, self.grad = ctx.target_loglike_grad(self.theta, precision=precision)
        i32 = dict(dtype=torch.int32, device=dev)
        f64 = dict(dtype=torch.float64, device=dev)
        self.ancestors = torch.zeros(n, **i32)
        self.n_leapfrog = torch.zeros(n, **i32)
        self.depth = torch.zeros(n, **i32)
        self.divergent = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.accept_stat = torch.zeros(n, **f64)
        self.inv_mass = torch.zeros((n_runs, D, D), **f64)
        self.chol = torch.zeros((n_runs, D, D), **f64)
        self.mm_status = torch.zeros(n_runs, **i32)
        self.chol_pp = torch.zeros((n, D, D), **f64) if metric == "local" else None
        self.metric_status = torch.zeros(n, **i32) if metric == "local" else None
        self.state_dev = torch.zeros((n_runs, STATE_SIZE), **f64)
        self.history_cap = history_cap
        self.history_dev = torch.zeros((n_runs, history_cap, HIST_SIZE), **f64)
        self.desc = SmcIterDesc(n_runs, P, D, precision, _ptr(self.theta), _ptr(self.logl), _ptr(self.grad),
                                _ptr(self.ancestors), _ptr(self.n_leapfrog), _ptr(self.depth), _ptr(self.divergent),
                                _ptr(self.accept_stat), _ptr(self.inv_mass), _ptr(self.chol), _ptr(self.mm_status),
                                _ptr(self.chol_pp), _ptr(self.metric_status), _ptr(self.state_dev),
                                _ptr(self.history_dev), history_cap, max_depth, alpha, shrink, step, max_delta_h,
                                seed, 1 if uturn else 0, nuts_form)

    def step(self):
        """Queue one iteration of every run (asynchronous)."""
        self.ctx._stream()
        _check("smcgw_smc_iteration", lib().smcgw_smc_iteration(self.ctx._h, C.byref(self.desc)))

    def graph(self) -> Graph:
        """A HIP graph of one iteration over these buffers."""
        return Graph(self.ctx, self.desc)

    def state(self) -> np.ndarray:
        """[n_runs][STATE_SIZE] copy of the run states (synchronises)."""
        return self.state_dev.cpu().numpy()

    def history(self) -> np.ndarray:
        """[n_runs][history_cap][HIST_SIZE] copy of the records (synchronises)."""
        return self.history_dev.cpu().numpy()

    def run_slice(self, r: int) -> slice:
        return slice(r * self.P, (r + 1) * self.P)


def runs_finished(state: np.ndarray) -> np.ndarray:
    """Per run: True once its last iteration mutated at beta = 1, or the run has stopped."""
    return (state[:, ST_DONE] != 0) | ((state[:, ST_BETA] >= 1.0) & (state[:, ST_NEXT] > 0))


class LogLikelihood(torch.autograd.Function):
    """logL(theta) with the hand-written adjoint as its backward pass."""

    @staticmethod
    def forward(ctx_, theta: torch.Tensor, context: Context, precision: int = MIXED):
        logl, grad = context.loglike_grad(theta.detach().contiguous(), precision=precision)
        ctx_.save_for_backward(grad)
        return logl

    @staticmethod
    def backward(ctx_, grad_out):
        (grad,) = ctx_.saved_tensors
        return grad_out[:, None] * grad, None, None
