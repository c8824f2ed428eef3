"""Thin ctypes binding of ``libehdbim.so`` (declared in include/ehdbim.h).

Argument marshalling only: device tensors are passed by pointer, every step
of the computation runs in the library's HIP kernels.  There is no fallback:
if the library is missing or fails to load, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libehdbim.so")

EHD_OK, EHD_E_ARG, EHD_E_SHAPE, EHD_E_STATE, EHD_E_NOMEM, EHD_E_HIP = range(6)
STOKES_SL, STOKES_DL, LAP_SL, LAP_DL, LAP_DLADJ = 1, 2, 4, 8, 16
ALL_KINDS = 31
METRIC_KINDS = STOKES_SL | STOKES_DL | LAP_SL | LAP_DL
FAR_FP64, FAR_FP32C = 0, 1
GRID_PAPER, GRID_2P = 0, 1
EOS_CLEAN, EOS_LINEAR, EOS_LANGMUIR = 0, 1, 2
MAX_P = 48
MAX_Q = 160
MAX_Q_CHECK = 400

COMPONENTS = ("Sx", "Sy", "Sz", "Dx", "Dy", "Dz", "SL", "L", "Kstar")
_KIND_OF_COMP = (STOKES_SL,) * 3 + (STOKES_DL,) * 3 + (LAP_SL, LAP_DL, LAP_DLADJ)

EXPORTED = ("ehd_create", "ehd_destroy", "ehd_last_error", "ehd_grid_dims", "ehd_set_drops",
            "ehd_num_targets", "ehd_layer_potentials", "ehd_synthesize", "ehd_analyze",
            "ehd_target_geometry", "ehd_sync", "ehd_wigner_d", "ehd_set_timing",
            "ehd_stage_times", "ehd_self_class_times", "ehd_set_graph", "ehd_set_far_config",
            "ehd_get_far_config", "ehd_time_far", "ehd_num_coefs", "ehd_solve_En",
            "ehd_solve_velocity", "ehd_surface", "ehd_drop_coefs", "ehd_explicit_step",
            "ehd_solve_surfactant", "ehd_mlp_create", "ehd_mlp_destroy", "ehd_mlp_last_error",
            "ehd_mlp_num_params", "ehd_mlp_get_params", "ehd_mlp_set_params", "ehd_mlp_get_grads",
            "ehd_mlp_forward", "ehd_mlp_backward", "ehd_mlp_mse", "ehd_mlp_adam", "ehd_area_weights",
            "ehd_update_shape", "ehd_surfactant_terms", "ehd_evolve_step", "ehd_evolve", "ehd_set_near",
            "ehd_near_pairs", "ehd_set_overlap", "ehd_overlap_plan", "ehd_self_config_candidates", "ehd_set_self_config", "ehd_get_self_config", "ehd_time_self", "ehd_solve_En_noalloc", "ehd_surfactant_guess",
            "ehd_learned_features")
STAGES = ("densities", "self", "far", "combine")
DEGREE_CLASSES = (16, 24, 32, 48)   # largest p of each self-interaction kernel class

_lib = None


class StepParams(C.Structure):
    """ehd_step_params (include/ehdbim.h)."""
    _fields_ = [("lam", C.c_double), ("R", C.c_double), ("Q", C.c_double), ("CaE", C.c_double),
                ("Eu", C.c_double), ("Eq", C.c_double), ("eos", C.c_int), ("beta", C.c_double),
                ("xs", C.c_double), ("dt", C.c_double), ("far_prec", C.c_int), ("restart", C.c_int),
                ("maxit", C.c_int), ("tol", C.c_double)]


class StepReport(C.Structure):
    """ehd_step_report (include/ehdbim.h)."""
    _fields_ = [("err_drop", C.c_double), ("err_surf", C.c_double), ("iters", C.c_int * 4),
                ("iters_gamma", C.c_int)]


class EvolveStats(C.Structure):
    """ehd_evolve_stats (include/ehdbim.h)."""
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("max_err", C.c_double), ("accepted", C.c_int),
                ("rejected", C.c_int), ("matvecs", C.c_longlong)]


class EhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ehdbim error {code}: {msg}")
        self.code = code


def self_config_candidates(cls: int):
    """Prefetch batches built for self-interaction class cls, the default
    first (host only)."""
    lib = load()
    pf, n = (C.c_int * 3)(), C.c_int()
    if lib.ehd_self_config_candidates(cls, pf, C.byref(n)) != 0:
        raise ValueError(f"invalid degree class {cls}")
    return [pf[i] for i in range(n.value)]


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no non-HIP fallback)")
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    lib.ehd_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, vp]
    lib.ehd_destroy.argtypes = [vp]
    lib.ehd_destroy.restype = None
    lib.ehd_last_error.argtypes = [vp]
    lib.ehd_last_error.restype = C.c_char_p
    lib.ehd_grid_dims.argtypes = [C.c_int, C.c_int, ip, ip]
    lib.ehd_set_drops.argtypes = [vp, C.c_int, ip, ip, ip, C.c_int, vp]
    lib.ehd_num_targets.argtypes = [vp, C.POINTER(C.c_longlong)]
    lib.ehd_layer_potentials.argtypes = [vp, vp, vp, vp, C.c_uint, C.c_int, vp, vp]
    lib.ehd_synthesize.argtypes = [vp, C.c_int, vp, vp]
    lib.ehd_analyze.argtypes = [vp, C.c_int, vp, vp]
    lib.ehd_target_geometry.argtypes = [vp, vp, vp]
    lib.ehd_sync.argtypes = [vp]
    lib.ehd_wigner_d.argtypes = [C.c_int, C.c_double, dp]
    lib.ehd_set_timing.argtypes = [vp, C.c_int]
    lib.ehd_stage_times.argtypes = [vp, C.c_int, dp]
    lib.ehd_self_class_times.argtypes = [vp, C.c_int, dp]
    lib.ehd_set_graph.argtypes = [vp, C.c_int]
    lib.ehd_set_far_config.argtypes = [vp, C.c_int, C.c_int]
    lib.ehd_get_far_config.argtypes = [vp, ip, ip]
    lib.ehd_time_far.argtypes = [vp, C.c_int, C.c_uint, C.c_int, C.c_int, C.c_int, dp]
    lib.ehd_num_coefs.argtypes = [vp, C.POINTER(C.c_longlong)]
    lib.ehd_surface.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    lib.ehd_drop_coefs.argtypes = [vp, vp]
    fp = C.POINTER(C.c_float)
    lib.ehd_mlp_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, vp, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_ulonglong]
    lib.ehd_mlp_destroy.argtypes = [vp]
    lib.ehd_mlp_destroy.restype = None
    lib.ehd_mlp_last_error.argtypes = [vp]
    lib.ehd_mlp_last_error.restype = C.c_char_p
    lib.ehd_mlp_num_params.argtypes = [vp, C.POINTER(C.c_longlong)]
    lib.ehd_mlp_get_params.argtypes = [vp, fp]
    lib.ehd_mlp_set_params.argtypes = [vp, fp]
    lib.ehd_mlp_get_grads.argtypes = [vp, fp]
    lib.ehd_mlp_forward.argtypes = [vp, C.c_int, vp, vp]
    lib.ehd_mlp_backward.argtypes = [vp, C.c_int, vp]
    lib.ehd_mlp_mse.argtypes = [vp, C.c_int, vp, vp, vp, dp]
    lib.ehd_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
    lib.ehd_solve_surfactant.argtypes = [vp, dp, vp, C.c_int, C.c_int, C.c_int, C.c_double, vp, ip, dp]
    lib.ehd_explicit_step.argtypes = [vp, C.POINTER(StepParams), vp, vp, vp, vp, ip]
    lib.ehd_area_weights.argtypes = [vp, vp]
    lib.ehd_set_overlap.argtypes = [vp, C.c_int]
    lib.ehd_overlap_plan.argtypes = [vp, C.c_uint, C.c_int, C.c_int, C.POINTER(C.c_uint), C.POINTER(C.c_longlong)]
    lib.ehd_self_config_candidates.argtypes = [C.c_int, ip, ip]
    lib.ehd_set_self_config.argtypes = [vp, C.c_int, C.c_int]
    lib.ehd_get_self_config.argtypes = [vp, C.c_int, ip]
    lib.ehd_time_self.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_int, dp]
    lib.ehd_set_near.argtypes = [vp, C.c_double, C.c_double, C.c_int, C.c_int]
    lib.ehd_near_pairs.argtypes = [vp, C.POINTER(C.c_longlong)]
    lib.ehd_update_shape.argtypes = [vp, vp]
    lib.ehd_surfactant_terms.argtypes = [vp, vp, vp, C.c_double, vp, vp]
    lib.ehd_evolve_step.argtypes = [vp, C.POINTER(StepParams), C.c_double, C.c_double, vp, vp, vp,
                                    C.POINTER(StepReport)]
    lib.ehd_evolve.argtypes = [vp, C.POINTER(StepParams), C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                               vp, C.POINTER(EvolveStats)]
    lib.ehd_solve_En.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                 C.c_double, vp, ip, dp]
    lib.ehd_solve_En_noalloc.argtypes = lib.ehd_solve_En.argtypes
    lib.ehd_surfactant_guess.argtypes = [vp, dp, vp, vp, C.c_int, vp, vp, vp, vp]
    lib.ehd_learned_features.argtypes = [vp, dp, vp, vp, vp, vp]
    lib.ehd_solve_velocity.argtypes = [vp, C.c_double, vp, C.c_int, C.c_int, C.c_int, C.c_double, vp,
                                       ip, dp]
    _lib = lib
    return lib


def _fptr(t):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device tensors (torch, on the GPU) are required")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("contiguous float32 tensors are required")
    return C.c_void_p(t.data_ptr())


class MLP:
    """The library's perceptron (ehd_mlp_*): forward/backward/loss/Adam kernels."""

    def __init__(self, nin: int, nhidden: int, nlayers: int, nout: int, seed: int = 1, device: int = 0,
                 stream=None):
        import numpy as np
        lib = load()
        self._lib = lib
        self._np = np
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        rc = lib.ehd_mlp_create(C.byref(h), device, C.c_void_p(stream.cuda_stream), nin, nhidden, nlayers, nout,
                                seed)
        if rc:
            raise EhdError(rc, "ehd_mlp_create failed")
        self._h = h
        self.nin, self.nout = nin, nout
        n = C.c_longlong()
        lib.ehd_mlp_num_params(h, C.byref(n))
        self.nparams = n.value

    def _check(self, rc):
        if rc:
            raise EhdError(rc, self._lib.ehd_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ehd_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = self._np.zeros(self.nparams, self._np.float32)
        self._check(self._lib.ehd_mlp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p):
        p = self._np.ascontiguousarray(p, self._np.float32)
        self._check(self._lib.ehd_mlp_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))))

    def grads(self):
        out = self._np.zeros(self.nparams, self._np.float32)
        self._check(self._lib.ehd_mlp_get_grads(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def forward(self, x: torch.Tensor, y: torch.Tensor | None = None):
        self._check(self._lib.ehd_mlp_forward(self._h, x.shape[0], _fptr(x), _fptr(y) if y is not None else None))

    def backward(self, dy: torch.Tensor):
        self._check(self._lib.ehd_mlp_backward(self._h, dy.shape[0], _fptr(dy)))

    def mse(self, y: torch.Tensor, t: torch.Tensor, dy: torch.Tensor, want_loss: bool = True):
        loss = C.c_double()
        self._check(self._lib.ehd_mlp_mse(self._h, y.shape[0], _fptr(y), _fptr(t), _fptr(dy),
                                          C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._check(self._lib.ehd_mlp_adam(self._h, lr, beta1, beta2, eps))


def rows_for_kinds(kinds: int) -> list[int]:
    """Component indices (into COMPONENTS) of the output rows for `kinds`."""
    return [c for c in range(9) if kinds & _KIND_OF_COMP[c]]


def grid_dims(P: int, grid_mode: int = GRID_PAPER) -> tuple[int, int]:
    lib = load()
    a, b = C.c_int(), C.c_int()
    rc = lib.ehd_grid_dims(P, grid_mode, C.byref(a), C.byref(b))
    if rc:
        raise EhdError(rc, "invalid grid")
    return a.value, b.value


def wigner_d(n: int, beta: float):
    import numpy as np
    out = np.zeros((2 * n + 1) ** 2)
    rc = load().ehd_wigner_d(n, float(beta), out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc:
        raise EhdError(rc, "invalid Wigner request")
    return out.reshape(2 * n + 1, 2 * n + 1)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device tensors (torch, on the GPU) are required")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("contiguous float64 tensors are required")
    return C.c_void_p(t.data_ptr())


class Context:
    """One library context bound to a device and a HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        lib = load()
        self._lib = lib
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        rc = lib.ehd_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if rc:
            raise EhdError(rc, lib.ehd_last_error(None).decode())
        self._h = h
        self.device = device
        self.ntargets = 0

    def _check(self, rc: int):
        if rc:
            raise EhdError(rc, self._lib.ehd_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ehd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_drops(self, p, q_self, q_far, grid_mode: int, xcoef: torch.Tensor):
        import numpy as np
        p = np.ascontiguousarray(p, np.int32)
        qs = np.ascontiguousarray(q_self, np.int32)
        qf = np.ascontiguousarray(q_far, np.int32)
        ip = C.POINTER(C.c_int)
        self._check(self._lib.ehd_set_drops(self._h, len(p), p.ctypes.data_as(ip),
                                            qs.ctypes.data_as(ip), qf.ctypes.data_as(ip),
                                            grid_mode, _ptr(xcoef)))
        n = C.c_longlong()
        self._check(self._lib.ehd_num_targets(self._h, C.byref(n)))
        self.ntargets = n.value
        self.p = p

    def layer_potentials(self, fcoef, ucoef, sigcoef, kinds: int, far_prec: int,
                         self_out: torch.Tensor, far_out: torch.Tensor | None = None):
        self._check(self._lib.ehd_layer_potentials(self._h, _ptr(fcoef), _ptr(ucoef),
                                                   _ptr(sigcoef), kinds, far_prec,
                                                   _ptr(self_out), _ptr(far_out)))

    def synthesize(self, nfields: int, coef: torch.Tensor, grid: torch.Tensor):
        self._check(self._lib.ehd_synthesize(self._h, nfields, _ptr(coef), _ptr(grid)))

    def analyze(self, nfields: int, grid: torch.Tensor, coef: torch.Tensor):
        self._check(self._lib.ehd_analyze(self._h, nfields, _ptr(grid), _ptr(coef)))

    def target_geometry(self, x: torch.Tensor, n: torch.Tensor):
        self._check(self._lib.ehd_target_geometry(self._h, _ptr(x), _ptr(n)))

    def sync(self):
        self._check(self._lib.ehd_sync(self._h))

    def set_timing(self, nslots: int):
        self._check(self._lib.ehd_set_timing(self._h, nslots))

    def set_overlap(self, enable: bool):
        """Far field on a second stream, concurrent with the self-interaction (ehd_set_overlap)."""
        self._check(self._lib.ehd_set_overlap(self._h, 1 if enable else 0))

    def set_self_config(self, cls: int, pf: int):
        """Legendre prefetch batch of degree class cls (0: the default; see
        self_config_candidates)."""
        self._check(self._lib.ehd_set_self_config(self._h, cls, pf))

    def self_config(self, cls: int) -> int:
        pf = C.c_int()
        self._check(self._lib.ehd_get_self_config(self._h, cls, C.byref(pf)))
        return pf.value

    def time_self(self, cls: int, pf: int, fcoef, sigcoef, reps: int = 3) -> float:
        """Milliseconds of one launch of class cls with prefetch batch pf
        (kinds S, D, S_L, L from fcoef and sigcoef)."""
        ms = C.c_double()
        self._check(self._lib.ehd_time_self(self._h, cls, pf, _ptr(fcoef), _ptr(sigcoef), reps, C.byref(ms)))
        return ms.value

    def overlap_plan(self, kinds: int, far_prec: int, with_u: bool = False):
        """(classes beside the forked far-field share as a bit mask, forked
        far-field work items) of an evaluation now (ehd_overlap_plan)."""
        m, n = C.c_uint(0), C.c_longlong(0)
        self._check(self._lib.ehd_overlap_plan(self._h, kinds, far_prec, 1 if with_u else 0, C.byref(m), C.byref(n)))
        return int(m.value), int(n.value)

    def set_graph(self, enable: bool):
        self._check(self._lib.ehd_set_graph(self._h, 1 if enable else 0))

    def set_far_config(self, targets_per_thread: int, nchunk: int):
        self._check(self._lib.ehd_set_far_config(self._h, targets_per_thread, nchunk))

    def far_config(self):
        a, b = C.c_int(), C.c_int()
        self._check(self._lib.ehd_get_far_config(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def time_far(self, far_prec: int, targets_per_thread: int, nchunk: int, reps: int = 3,
                 kinds: int = ALL_KINDS) -> float:
        ms = C.c_double()
        self._check(self._lib.ehd_time_far(self._h, far_prec, kinds, targets_per_thread, nchunk, reps,
                                           C.byref(ms)))
        return ms.value

    def self_class_times(self, slot: int):
        """Milliseconds of the self-interaction kernel of each degree class
        (DEGREE_CLASSES) in a recorded call; 0 for a class without drops."""
        ms = (C.c_double * 4)()
        self._check(self._lib.ehd_self_class_times(self._h, slot, ms))
        return list(ms)

    def surface(self, H: torch.Tensor, gcoef: torch.Tensor | None = None, grad: torch.Tensor | None = None,
                ng: int = 0, lap: torch.Tensor | None = None):
        """Mean curvature H[T], surface gradients grad[ng][3][T] and, if given,
        Laplace-Beltrami values lap[ng][T] of ng packed scalar fields at the
        target nodes."""
        self._check(self._lib.ehd_surface(self._h, ng, _ptr(gcoef), _ptr(H), _ptr(grad), _ptr(lap)))

    def solve_surfactant(self, kappa, rhs: torch.Tensor, gamma: torch.Tensor, precond: bool = True,
                         restart: int = 30, maxit: int = 200, tol: float = 1e-10):
        """GMRES solve of (I - kappa Lap_S) Gamma = rhs in Galerkin form; kappa
        is one value or one per drop; gamma holds the initial guess and
        receives the solution.  Returns (iters, relres)."""
        import numpy as np
        k = np.broadcast_to(np.asarray(kappa, np.float64), (len(self.p),)).copy()
        it, rr = C.c_int(), C.c_double()
        self._check(self._lib.ehd_solve_surfactant(self._h, k.ctypes.data_as(C.POINTER(C.c_double)), _ptr(rhs),
                                                   1 if precond else 0, restart, maxit, float(tol), _ptr(gamma),
                                                   C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def drop_coefs(self, x: torch.Tensor):
        """Copy of the current drops' surface coefficients (3 packed fields)."""
        self._check(self._lib.ehd_drop_coefs(self._h, _ptr(x)))

    def explicit_step(self, lam: float, R: float, Q: float, CaE: float, Eu: float, Eq: float, dt: float,
                      en: torch.Tensor, u: torch.Tensor, xnew: torch.Tensor, gamma: torch.Tensor | None = None,
                      eos: int = EOS_CLEAN, beta: float = 0.0, xs: float = 0.0, far_prec: int = FAR_FP64,
                      restart: int = 30, maxit: int = 200, tol: float = 1e-12):
        """One explicit step (ehd_explicit_step).  en (1 field) and u (3 fields)
        hold initial guesses and receive E_n and the velocity; xnew receives
        x + dt u.  Returns the GMRES iterations (E_n, velocity)."""
        prm = StepParams(lam, R, Q, CaE, Eu, Eq, eos, beta, xs, dt, far_prec, restart, maxit, tol)
        its = (C.c_int * 2)()
        self._check(self._lib.ehd_explicit_step(self._h, C.byref(prm), _ptr(gamma), _ptr(en), _ptr(u),
                                                _ptr(xnew), its))
        return its[0], its[1]

    def set_near(self, delta: float, s_check: float | None = None, m: int = 8, q_check: int | None = None):
        """Nearly singular correction for targets closer than delta to another
        drop (ehd_set_near); delta = 0 switches it off.  q_check defaults to
        10 times the largest p (at most MAX_Q_CHECK), s_check to three
        check-grid spacings of a unit drop, 3 pi / (q_check + 1)."""
        if q_check is None:
            q_check = min(MAX_Q_CHECK, 10 * int(max(self.p)))
        if s_check is None:
            s_check = 3.0 * math.pi / (q_check + 1)
        self._check(self._lib.ehd_set_near(self._h, float(delta), float(s_check), int(m), int(q_check)))

    def near_pairs(self) -> int:
        n = C.c_longlong()
        self._check(self._lib.ehd_near_pairs(self._h, C.byref(n)))
        return n.value

    def area_weights(self, w: torch.Tensor):
        """Area quadrature weights at the target nodes (ehd_area_weights)."""
        self._check(self._lib.ehd_area_weights(self._h, _ptr(w)))

    def update_shape(self, x: torch.Tensor):
        """New surface coefficients for the same drops (ehd_update_shape)."""
        self._check(self._lib.ehd_update_shape(self._h, _ptr(x)))

    def surfactant_terms(self, u: torch.Tensor | None, gamma: torch.Tensor, inv_pe: float,
                         gE: torch.Tensor | None, gI: torch.Tensor | None):
        """g_E = P[-Gamma div_S u] and g_I = P[inv_pe Lap_S Gamma] (ehd_surfactant_terms)."""
        self._check(self._lib.ehd_surfactant_terms(self._h, _ptr(u), _ptr(gamma), float(inv_pe), _ptr(gE),
                                                   _ptr(gI)))

    @staticmethod
    def step_params(lam, R, Q, CaE, Eu, Eq, eos=EOS_CLEAN, beta=0.0, xs=0.0, far_prec=FAR_FP64, restart=30,
                    maxit=200, tol=1e-12) -> StepParams:
        return StepParams(lam, R, Q, CaE, Eu, Eq, eos, beta, xs, 0.0, far_prec, restart, maxit, tol)

    def evolve_step(self, prm: StepParams, inv_pe: float, dt: float, gamma: torch.Tensor, xnew: torch.Tensor,
                    gnew: torch.Tensor) -> dict:
        """One step of Algorithm 1 (ehd_evolve_step); the context stays at x^n."""
        rep = StepReport()
        self._check(self._lib.ehd_evolve_step(self._h, C.byref(prm), float(inv_pe), float(dt), _ptr(gamma),
                                              _ptr(xnew), _ptr(gnew), C.byref(rep)))
        return {"err_drop": rep.err_drop, "err_surf": rep.err_surf, "iters": list(rep.iters),
                "iters_gamma": rep.iters_gamma}

    def evolve(self, prm: StepParams, inv_pe: float, t_end: float, dt0: float, tol: float, max_steps: int,
               gamma: torch.Tensor) -> dict:
        """Adaptive time stepping to t_end (ehd_evolve); drops and gamma advance in place."""
        st = EvolveStats()
        self._check(self._lib.ehd_evolve(self._h, C.byref(prm), float(inv_pe), float(t_end), float(dt0),
                                         float(tol), int(max_steps), _ptr(gamma), C.byref(st)))
        return {"t": st.t, "dt": st.dt, "max_err": st.max_err, "accepted": st.accepted, "rejected": st.rejected,
                "matvecs": st.matvecs}

    def num_coefs(self) -> int:
        """Doubles of one packed field of the current drops."""
        n = C.c_longlong()
        self._check(self._lib.ehd_num_coefs(self._h, C.byref(n)))
        return n.value

    def solve_En(self, R: float, Eu: float, Eq: float, en: torch.Tensor, far_prec: int = FAR_FP64,
                 restart: int = 30, maxit: int = 200, tol: float = 1e-12):
        """GMRES solve of the E_n Galerkin system; `en` (1 packed field) holds
        the initial guess and receives the solution.  Returns (iters, relres)."""
        it, rr = C.c_int(), C.c_double()
        self._check(self._lib.ehd_solve_En(self._h, float(R), float(Eu), float(Eq), far_prec, restart,
                                           maxit, float(tol), _ptr(en), C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def solve_En_noalloc(self, R: float, Eu: float, Eq: float, en: torch.Tensor, far_prec: int = FAR_FP64,
                         restart: int = 30, maxit: int = 200, tol: float = 1e-12):
        """As solve_En, through the allocation-free entry point (workspace in
        the library's static device array)."""
        it, rr = C.c_int(), C.c_double()
        self._check(self._lib.ehd_solve_En_noalloc(self._h, float(R), float(Eu), float(Eq), far_prec, restart,
                                                   maxit, float(tol), _ptr(en), C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def surfactant_guess(self, kappa, rhs: torch.Tensor, guess: torch.Tensor, y: torch.Tensor | None = None,
                         ymean: torch.Tensor | None = None, ystd: torch.Tensor | None = None,
                         gain: torch.Tensor | None = None):
        """guess = M^{-1} rhs (+ kappa |rhs| gain (y ystd + ymean) per drop when
        y, the network's FP32 outputs [ndrops][ny], is given)."""
        import numpy as np
        k = np.broadcast_to(np.asarray(kappa, np.float64), (len(self.p),)).copy()
        ny = int(y.shape[1]) if y is not None else 0
        self._check(self._lib.ehd_surfactant_guess(
            self._h, k.ctypes.data_as(C.POINTER(C.c_double)), _ptr(rhs),
            _fptr(y) if y is not None else None, ny,
            _ptr(ymean) if y is not None else None, _ptr(ystd) if y is not None else None,
            _ptr(gain) if y is not None else None, _ptr(guess)))

    def learned_features(self, kappa, rhs: torch.Tensor, mean: torch.Tensor, std: torch.Tensor,
                         feat: torch.Tensor):
        """FP32 network inputs [ndrops][4 nc + 1], standardised with mean, std."""
        import numpy as np
        k = np.broadcast_to(np.asarray(kappa, np.float64), (len(self.p),)).copy()
        self._check(self._lib.ehd_learned_features(self._h, k.ctypes.data_as(C.POINTER(C.c_double)), _ptr(rhs),
                                                   _ptr(mean), _ptr(std), _fptr(feat)))

    def solve_velocity(self, lam: float, fcoef: torch.Tensor, u: torch.Tensor, far_prec: int = FAR_FP64,
                       restart: int = 30, maxit: int = 200, tol: float = 1e-12):
        """GMRES solve of the velocity Galerkin system for the force density
        `fcoef`; `u` (3 packed fields) holds the initial guess and receives
        the solution.  Returns (iters, relres)."""
        it, rr = C.c_int(), C.c_double()
        self._check(self._lib.ehd_solve_velocity(self._h, float(lam), _ptr(fcoef), far_prec, restart,
                                                 maxit, float(tol), _ptr(u), C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def stage_times(self, slot: int):
        """Milliseconds of (densities, self, far, combine) of a recorded call."""
        ms = (C.c_double * 4)()
        self._check(self._lib.ehd_stage_times(self._h, slot, ms))
        return list(ms)


def evaluate(susp, kinds: int = ALL_KINDS, far_prec: int = FAR_FP64, split: bool = True,
             device: int = 0, overlap: bool = False, autotune: bool = False):
    """Convenience: one evaluation of a workloads.Suspension on `device`
    (optionally in overlap mode, with the far-field tile shape from the
    autotuner, as the benchmark runs it).  Returns (self_out, far_out) as
    CPU float64 tensors [rows][ntargets]."""
    dev = torch.device("cuda", device)
    ctx = Context(device)
    x = torch.from_numpy(susp.xcoef).to(dev)
    ctx.set_drops(susp.p, susp.q_self, susp.q_far, susp.grid_mode, x)
    if autotune:
        from . import autotune as _tune
        _tune.autotune_far(ctx, susp.p, susp.q_far, susp.grid_mode, far_prec, kinds=kinds, use_cache=False)
    if overlap:
        ctx.set_overlap(True)
    f = torch.from_numpy(susp.fcoef).to(dev)
    s = torch.from_numpy(susp.sigcoef).to(dev)
    u = torch.from_numpy(susp.ucoef).to(dev) if susp.ucoef is not None else None
    rows = len(rows_for_kinds(kinds))
    so = torch.zeros(rows, ctx.ntargets, dtype=torch.float64, device=dev)
    fo = torch.zeros_like(so) if split else None
    ctx.layer_potentials(f, u, s, kinds, far_prec, so, fo)
    ctx.sync()
    out = (so.cpu(), fo.cpu() if fo is not None else None)
    ctx.close()
    return out
