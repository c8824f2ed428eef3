"""ctypes wrapper around the plain FP64 CPU oracle (``ehd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  The
oracle shares no code with the HIP path; both read the same seeded inputs.

Output component order everywhere: S_x S_y S_z D_x D_y D_z S_L L K*.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libehd_oracle.so")
_lib = None

COMPONENTS = ("Sx", "Sy", "Sz", "Dx", "Dy", "Dz", "SL", "L", "Kstar")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.ora_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
    lib.ora_surface_point.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_double, C.c_double, _dp]
    lib.ora_surface_point.restype = None
    lib.ora_pbar.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
    lib.ora_pbar.restype = None
    lib.ora_synth_grid.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.c_int, _dp]
    lib.ora_analyze_grid.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.c_int, _dp]
    lib.ora_targets.argtypes = [C.c_int, _ip, C.c_int, _dp, C.c_int, _ip, _ip, _dp, _dp]
    lib.ora_far.argtypes = [C.c_int, _ip, _ip, C.c_int, _dp, _dp, _dp, _dp, C.c_int, _dp, _dp,
                            _ip, _dp]
    lib.ora_self.argtypes = [C.c_int, _ip, _ip, C.c_int, _dp, _dp, _dp, _dp, C.c_int, _ip, _ip,
                             _dp]
    lib.ora_surface_integrals.argtypes = [C.c_int, _dp, C.c_int, _dp, C.c_int, C.c_int, _dp, _dp,
                                          _dp]
    lib.ora_sh_point.argtypes = [C.c_int, C.c_int, _dp, C.c_double, C.c_double, C.c_double,
                                 C.c_double, _dp, _dp, _dp]
    lib.ora_sh_point.restype = None
    lib.ora_geom_point.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                   _dp, _dp, _dp]
    lib.ora_geom_point.restype = None
    lib.ora_num_threads.restype = C.c_int
    lib.ora_set_threads.argtypes = [C.c_int]
    lib.ora_set_threads.restype = None
    lib.ora_far_sources.argtypes = [C.c_int, _ip, _ip, C.c_int, _dp, _dp, _dp, _dp]
    lib.ora_far_sources.restype = C.c_void_p
    lib.ora_far_eval.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _ip, _dp]
    lib.ora_far_free.argtypes = [C.c_void_p]
    lib.ora_far_free.restype = None
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def nlon_of(P: int, grid_mode: int) -> int:
    return 2 * P + 2 if grid_mode == 0 else 2 * P


def num_threads() -> int:
    return int(_load().ora_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of later oracle calls."""
    _load().ora_set_threads(int(n))


def gauss_legendre(n: int):
    t = np.zeros(n)
    w = np.zeros(n)
    _load().ora_gauss_legendre(n, _d(t), _d(w))
    return t, w


def pbar(p: int, theta: float):
    """Pbar_n^m(cos theta), dPbar/dtheta and Pbar/sin(theta), indexed n(n+1)/2+m."""
    nc = (p + 1) * (p + 2) // 2
    out, dth, ovs = np.zeros(nc), np.zeros(nc), np.zeros(nc)
    _load().ora_pbar(p, float(np.cos(theta)), float(np.sin(theta)), _d(out), _d(dth), _d(ovs))
    return out, dth, ovs


def sh_point(p: int, coef: np.ndarray, theta: float, phi: float, nf: int = 1):
    coef = _f64(coef)
    v, dt, dp = np.zeros(nf), np.zeros(nf), np.zeros(nf)
    _load().ora_sh_point(p, nf, _d(coef), float(np.cos(theta)), float(np.sin(theta)),
                         float(np.cos(phi)), float(np.sin(phi)), _d(v), _d(dt), _d(dp))
    return v, dt, dp


def geom_point(p: int, xcoef: np.ndarray, theta: float, phi: float):
    xcoef = _f64(xcoef)
    x, n, J = np.zeros(3), np.zeros(3), np.zeros(1)
    _load().ora_geom_point(p, _d(xcoef), float(np.cos(theta)), float(np.sin(theta)),
                           float(np.cos(phi)), float(np.sin(phi)), _d(x), _d(n), _d(J))
    return x, n, float(J[0])


def surface_point(p: int, xcoef: np.ndarray, theta: float, phi: float, gcoef=None, ng: int = 0,
                  lap: bool = False):
    """x(3), outward normal n(3), mean curvature H = (1/2) div_S n and the
    surface gradients (3 each) of ng scalar fields, at one parameter point.
    With lap=True also their Laplace-Beltrami values (a fifth result)."""
    xcoef = _f64(xcoef)
    gc = _f64(gcoef) if ng else np.zeros(2)
    out = np.zeros(7 + 4 * ng)
    _load().ora_surface_point(p, _d(xcoef), ng, _d(gc), float(theta), float(phi), _d(out))
    g = out[7:].reshape(ng, 4)
    if lap:
        return out[0:3], out[3:6], float(out[6]), g[:, :3].copy(), g[:, 3].copy()
    return out[0:3], out[3:6], float(out[6]), g[:, :3].copy()


def synth_grid(p: int, coef: np.ndarray, Q: int, grid_mode: int = 0, nf: int = 1):
    coef = _f64(coef)
    nlat, nlon = Q + 1, nlon_of(Q, grid_mode)
    out = np.zeros(nf * nlat * nlon)
    _load().ora_synth_grid(p, nf, _d(coef), Q, grid_mode, _d(out))
    return out.reshape(nf, nlat, nlon)


def analyze_grid(p: int, grid: np.ndarray, Q: int, grid_mode: int = 0, nf: int = 1):
    grid = _f64(grid)
    coef = np.zeros(nf * (p + 1) * (p + 2))
    _load().ora_analyze_grid(p, nf, _d(grid), Q, grid_mode, _d(coef))
    return coef


def surface_integrals(p: int, xcoef, Q: int, grid_mode: int = 0, pg: int = 0, gcoef=None):
    xcoef = _f64(xcoef)
    a, v, g = np.zeros(1), np.zeros(1), np.zeros(1)
    gc = _f64(gcoef) if gcoef is not None else None
    _load().ora_surface_integrals(p, _d(xcoef), pg, _d(gc) if gc is not None else None, Q,
                                  grid_mode, _d(a), _d(v), _d(g))
    return float(a[0]), float(v[0]), float(g[0])


def _susp_args(s):
    p = _i32(s.p)
    x = _f64(s.xcoef)
    f = _f64(s.fcoef)
    sg = _f64(s.sigcoef)
    u = _f64(s.ucoef) if s.ucoef is not None else None
    return p, x, f, u, sg


def targets(s, tgt_drop, tgt_node):
    p, x, f, u, sg = _susp_args(s)
    td, tn = _i32(tgt_drop), _i32(tgt_node)
    nt = len(td)
    x0, n0 = np.zeros(3 * nt), np.zeros(3 * nt)
    _load().ora_targets(s.ndrops, _i(p), s.grid_mode, _d(x), nt, _i(td), _i(tn), _d(x0), _d(n0))
    return x0.reshape(3, nt), n0.reshape(3, nt)


def far_points(s, x0: np.ndarray, n0: np.ndarray, exclude=None):
    """Far-field sums (regular quadrature on each drop's q_far grid) at
    arbitrary points x0[3][nt] with target normals n0[3][nt]."""
    p, x, f, u, sg = _susp_args(s)
    qf = _i32(s.q_far)
    x0 = _f64(x0)
    n0 = _f64(n0)
    nt = x0.shape[1]
    ex = _i32(exclude if exclude is not None else -np.ones(nt))
    out = np.zeros(9 * nt)
    _load().ora_far(s.ndrops, _i(p), _i(qf), s.grid_mode, _d(x), _d(f),
                    _d(u) if u is not None else None, _d(sg), nt, _d(x0), _d(n0), _i(ex),
                    _d(out))
    return out.reshape(9, nt)


class FarSources:
    """The regular-rule source records of every drop, built once
    (``ora_far_sources``) and summed at points by ``eval``; ``far_points``
    does both in one call."""

    def __init__(self, s):
        p, x, f, u, sg = _susp_args(s)
        qf = _i32(s.q_far)
        self._keep = (p, qf, x, f, u, sg)
        self.h = _load().ora_far_sources(s.ndrops, _i(p), _i(qf), s.grid_mode, _d(x), _d(f),
                                         _d(u) if u is not None else None, _d(sg))

    def eval(self, x0, n0, exclude=None):
        x0 = _f64(x0)
        n0 = _f64(n0)
        nt = x0.shape[1]
        ex = _i32(exclude if exclude is not None else -np.ones(nt))
        out = np.zeros(9 * nt)
        _load().ora_far_eval(self.h, nt, _d(x0), _d(n0), _i(ex), _d(out))
        return out.reshape(9, nt)

    def close(self):
        if self.h:
            _load().ora_far_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


def far(s, tgt_drop, tgt_node):
    """Far field at drop grid nodes, own drop excluded."""
    x0, n0 = targets(s, tgt_drop, tgt_node)
    return far_points(s, x0, n0, exclude=tgt_drop)


def self_(s, tgt_drop, tgt_node):
    """Singular self-interaction at drop grid nodes (rotated-pole rule)."""
    p, x, f, u, sg = _susp_args(s)
    qs = _i32(s.q_self)
    td, tn = _i32(tgt_drop), _i32(tgt_node)
    nt = len(td)
    out = np.zeros(9 * nt)
    _load().ora_self(s.ndrops, _i(p), _i(qs), s.grid_mode, _d(x), _d(f),
                     _d(u) if u is not None else None, _d(sg), nt, _i(td), _i(tn), _d(out))
    return out.reshape(9, nt)


def all_targets(s):
    """(tgt_drop, tgt_node) for every grid node of every drop, in the global
    target order (drop-major, node = j*nlon + k)."""
    td, tn = [], []
    for d, pp in enumerate(s.p):
        n = (int(pp) + 1) * nlon_of(int(pp), s.grid_mode)
        td.append(np.full(n, d, np.int32))
        tn.append(np.arange(n, dtype=np.int32))
    return np.concatenate(td), np.concatenate(tn)
