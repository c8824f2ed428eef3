"""Galerkin systems of the paper (Sec. 2, eq. galerkin_En and
eq. BIM_galerkin), assembled as dense matrices column by column from the
oracle's layer potentials and solved with a library LU factorisation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain FP64, no code
shared with the HIP path.

Unknowns are packed SH coefficient vectors of real fields (the layout of
``include/ehdbim.h``); the imaginary slots of the m = 0 coefficients are
not unknowns and stay zero.  The projection (y, Y_nm) of values at a drop's
grid nodes is the oracle's Gaussian-grid analysis on that grid.

E_n system (eq. galerkin_En, with the adjoint double layer K*: eq. E_n is
eq. BIE01 dotted with the target normal n(x0)):
    (1/2) E_n - (R-1)/(R+1) P[K*[E_n]] = R/(R+1) P[E_inf . n],
E_inf = -grad phi_inf with phi_inf = -(E_u z + E_q (z^2 - (x^2 + y^2)/2)),
the uniform and quadrupole parts of the applied potential (Sec. 1).

Velocity system (eq. BIM_galerkin):
    (lambda+1) u - (lambda-1) P[D[u]] = P[S[f]].
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import all_targets, analyze_grid, far, nlon_of, self_, targets

ROW_S, ROW_D, ROW_SL, ROW_L, ROW_KSTAR = 0, 3, 6, 7, 8


def project(s, vals: np.ndarray, nf: int) -> np.ndarray:
    """(values at all targets [nf][T]) -> packed coefficients, nf fields per drop."""
    out, off = [], 0
    for p in (int(x) for x in s.p):
        nl = nlon_of(p, s.grid_mode)
        n = (p + 1) * nl
        out.append(analyze_grid(p, vals[:, off:off + n].reshape(nf, p + 1, nl), p, s.grid_mode, nf))
        off += n
    return np.concatenate(out)


def potentials(s) -> np.ndarray:
    """All nine components, self (singular rule) + far, at every target."""
    td, tn = all_targets(s)
    return self_(s, td, tn) + far(s, td, tn)


def unknown_mask(s, nf: int) -> np.ndarray:
    """True at the packed entries that are unknowns (all but Im of m = 0)."""
    mask = []
    for p in (int(x) for x in s.p):
        blk = np.ones((nf, (p + 1) * (p + 2) // 2, 2), bool)
        for n in range(p + 1):
            blk[:, n * (n + 1) // 2, 1] = False
        mask.append(blk.ravel())
    return np.concatenate(mask)


def einf_dot_n(s, Eu: float, Eq: float) -> np.ndarray:
    x0, n0 = targets(s, *all_targets(s))
    x, y, z = x0
    return -Eq * x * n0[0] - Eq * y * n0[1] + (Eu + 2.0 * Eq * z) * n0[2]


def En_rhs(s, R: float, Eu: float, Eq: float) -> np.ndarray:
    return R / (R + 1.0) * project(s, einf_dot_n(s, Eu, Eq)[None, :], 1)


def En_apply(s, R: float, en: np.ndarray) -> np.ndarray:
    ks = potentials(dataclasses.replace(s, sigcoef=np.asarray(en, float)))[ROW_KSTAR]
    return 0.5 * en - (R - 1.0) / (R + 1.0) * project(s, ks[None, :], 1)


def velocity_rhs(s, f: np.ndarray) -> np.ndarray:
    sf = potentials(dataclasses.replace(s, fcoef=np.asarray(f, float)))[ROW_S:ROW_S + 3]
    return project(s, sf, 3)


def velocity_apply(s, lam: float, u: np.ndarray) -> np.ndarray:
    z = np.zeros_like(np.asarray(u, float))
    du = potentials(dataclasses.replace(s, fcoef=z, ucoef=np.asarray(u, float)))[ROW_D:ROW_D + 3]
    return (lam + 1.0) * u - (lam - 1.0) * project(s, du, 3)


def _dense_solve(apply, rhs: np.ndarray, mask: np.ndarray) -> np.ndarray:
    idx = np.flatnonzero(mask)
    A = np.zeros((len(idx), len(idx)))
    e = np.zeros(len(mask))
    for j, k in enumerate(idx):
        e[:] = 0.0
        e[k] = 1.0
        A[:, j] = apply(e)[idx]
    x = np.zeros(len(mask))
    x[idx] = np.linalg.solve(A, rhs[idx])
    return x


def solve_En_dense(s, R: float, Eu: float, Eq: float) -> np.ndarray:
    return _dense_solve(lambda v: En_apply(s, R, v), En_rhs(s, R, Eu, Eq), unknown_mask(s, 1))


def solve_velocity_dense(s, lam: float, f: np.ndarray) -> np.ndarray:
    return _dense_solve(lambda v: velocity_apply(s, lam, v), velocity_rhs(s, f), unknown_mask(s, 3))
