"""Nearly singular evaluation by line interpolation (Sec. 2.1: the on-surface
value from the singular rule, regular-rule values at points aligned with the
target farther out, and a 1D Lagrange interpolation at the target).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain FP64, no code
shared with the HIP path.

For a target x0 outside drop j (closer than a threshold to its surface):
  1. y = x(theta*, phi*) the closest point of drop j's surface (least
     squares in the surface parameters), s_t = |x0 - y|, nu = (x0 - y) / s_t;
  2. the limit at y, from the exterior, of drop j's layer potentials: the
     on-surface values of the singular rule at drop j's grid nodes, projected
     to degree p and evaluated at y, plus the jump to the exterior side
     (S, S_L continuous; D: -u(y); L: +sigma(y)/2; K* with the target normal
     n0: -n0 . grad_S S_L(y) + (K*(y) + sigma(y)/2)(n0 . n_y), since K* is
     -n0 . grad S_L and the normal derivative of S_L jumps by -sigma/2);
  3. drop j's regular-rule sums at y + s_k nu, s_k = s_check (1 + (k - 1)/2),
     k = 1..m (the target's normal n0 for K*), on an upsampled grid;
  4. the Lagrange polynomial through (0, limit) and (s_k, values), at s_t.
Returns drop j's corrected contribution at x0 and its plain regular-rule
value there (9 rows: S_x S_y S_z D_x D_y D_z S_L L K*).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.optimize import least_squares

from . import all_targets, analyze_grid, far_points, gauss_legendre, nlon_of, self_, sh_point, surface_point


def drop_only(s, j: int):
    """The suspension reduced to drop j."""
    off = np.concatenate([[0], np.cumsum([(int(p) + 1) * (int(p) + 2) for p in s.p])])
    a, b = off[j], off[j + 1]
    return dataclasses.replace(
        s, p=s.p[j:j + 1], q_self=s.q_self[j:j + 1], q_far=s.q_far[j:j + 1], xcoef=s.xcoef[3 * a:3 * b],
        fcoef=s.fcoef[3 * a:3 * b], sigcoef=s.sigcoef[a:b],
        ucoef=None if s.ucoef is None else s.ucoef[3 * a:3 * b])


def closest_point(p: int, xc: np.ndarray, x0: np.ndarray):
    """(theta, phi) of the point of the surface x(theta, phi) closest to x0,
    from the nearest grid node of the degree-p grid."""
    t, _ = gauss_legendre(p + 1)
    nl = 2 * p + 2
    best = None
    for th in np.arccos(t):
        for k in range(nl):
            ph = 2 * np.pi * k / nl
            d = np.linalg.norm(sh_point(p, xc, th, ph, nf=3)[0] - x0)
            if best is None or d < best[0]:
                best = (d, th, ph)

    def res(v):
        return sh_point(p, xc, v[0], v[1], nf=3)[0] - x0

    def jac(v):
        _, dt, dp = sh_point(p, xc, v[0], v[1], nf=3)
        return np.stack([dt, np.sin(v[0]) * dp], axis=1)

    r = least_squares(res, np.array([best[1], best[2]]), jac=jac, xtol=1e-15, ftol=1e-15, gtol=1e-15)
    return float(r.x[0]), float(r.x[1])


def lagrange(nodes: np.ndarray, vals: np.ndarray, s: float) -> np.ndarray:
    """Value at s of the polynomial through (nodes[k], vals[k]) (vals [k][...])."""
    out = np.zeros(vals.shape[1:])
    for k in range(len(nodes)):
        w = 1.0
        for i in range(len(nodes)):
            if i != k:
                w *= (s - nodes[i]) / (nodes[k] - nodes[i])
        out += w * vals[k]
    return out


def surface_limit(s, j: int, th: float, ph: float, n0: np.ndarray) -> np.ndarray:
    """Exterior limit at x(th, ph) on drop j of its nine layer-potential rows."""
    sj = drop_only(s, j)
    p = int(sj.p[0])
    td, tn = all_targets(sj)
    vals = self_(sj, td, tn)                                   # on-surface, singular rule
    nl = nlon_of(p, sj.grid_mode)
    coef = analyze_grid(p, vals.reshape(9, p + 1, nl), p, sj.grid_mode, 9)
    v = sh_point(p, coef, th, ph, nf=9)[0]
    nc2 = (p + 1) * (p + 2)
    _, ny, _, g = surface_point(p, sj.xcoef, th, ph, gcoef=coef[6 * nc2:7 * nc2], ng=1)
    u = sh_point(p, sj.ucoef if sj.ucoef is not None else sj.fcoef, th, ph, nf=3)[0]
    sig = sh_point(p, sj.sigcoef, th, ph)[0][0]
    out = v.copy()
    out[3:6] -= u
    out[7] += 0.5 * sig
    out[8] = -float(n0 @ g[0]) + (v[8] + 0.5 * sig) * float(n0 @ ny)
    return out


def near_value(s, j: int, x0: np.ndarray, n0: np.ndarray, s_check: float, m: int = 4, q_check: int | None = None):
    """(corrected, plain) contribution of drop j at the target x0 (normal n0);
    the check points use drop j's regular rule on a degree-q_check grid
    (default its q_far)."""
    sj = drop_only(s, j)
    sc = sj if q_check is None else dataclasses.replace(sj, q_far=np.array([q_check], np.int32))
    p = int(sj.p[0])
    th, ph = closest_point(p, sj.xcoef, x0)
    y = sh_point(p, sj.xcoef, th, ph, nf=3)[0]
    st = float(np.linalg.norm(x0 - y))
    nu = (x0 - y) / st
    sk = s_check * (1.0 + 0.5 * np.arange(m))
    pts = y[:, None] + nu[:, None] * sk[None, :]
    chk = far_points(sc, pts, np.repeat(n0[:, None], m, axis=1))
    nodes = np.concatenate([[0.0], sk])
    vals = np.concatenate([surface_limit(s, j, th, ph, n0)[None, :], chk.T], axis=0)
    plain = far_points(sj, x0[:, None], n0[:, None])[:, 0]
    return lagrange(nodes, vals, st), plain, {"theta": th, "phi": ph, "y": y, "dist": st}
