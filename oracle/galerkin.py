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

from . import all_targets, analyze_grid, far, gauss_legendre, nlon_of, self_, targets

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


# ---------------------------------------------------------------------------
# One explicit step (Sec. 1, steps i-vii): E_n, tangential field, electric
# and interfacial forces, velocity, position update.
# ---------------------------------------------------------------------------
def node_angles(s):
    """(drop, theta, phi) of every target node in the global order."""
    out = []
    for d, p in enumerate(int(x) for x in s.p):
        nl = nlon_of(p, s.grid_mode)
        t, _ = gauss_legendre(p + 1)
        for j in range(p + 1):
            for k in range(nl):
                out.append((d, float(np.arccos(t[j])), 2.0 * np.pi * k / nl))
    return out


def _drop_block(s, vec: np.ndarray, d: int, nf: int) -> np.ndarray:
    off = np.concatenate([[0], np.cumsum([(int(p) + 1) * (int(p) + 2) for p in s.p])])
    return vec[nf * off[d]:nf * off[d + 1]]


def gamma_eos(G: float, eos: int, beta: float, xs: float):
    """gamma and dgamma/dGamma (eq. langmuir, eq. lin_eq_state), gamma(1) = 1."""
    if eos == 1:
        return 1.0 + beta * (1.0 - G), -beta
    if eos == 2:
        nrm = 1.0 + beta * np.log(1.0 - xs)
        return (1.0 + beta * np.log(1.0 - xs * G)) / nrm, -beta * xs / (1.0 - xs * G) / nrm
    return 1.0, 0.0


def forces(s, R, Q, CaE, Eu, Eq, en, gamma=None, eos=0, beta=0.0, xs=0.0):
    """Force density -(f / Ca_E - f^E) and the tangential field E_t at the
    target nodes ([3][T] each).  E_t = (I - n n) E_inf - grad_S S_L[q] with
    q = (1 - 1/R) E_n (the potential phi_inf + S_L[q] of eq. BIE01);
    f^E of eq. el_force with eps~ eps_0 = 1; f = 2 gamma H n - grad_S gamma."""
    from . import sh_point, surface_point
    q = (1.0 - 1.0 / R) * np.asarray(en, float)
    slq = potentials(dataclasses.replace(s, sigcoef=q))[ROW_SL]
    phq = project(s, slq[None, :], 1)
    nodes = node_angles(s)
    T = len(nodes)
    ftot, Et = np.zeros((3, T)), np.zeros((3, T))
    for i, (d, th, ph) in enumerate(nodes):
        p = int(s.p[d])
        xd = _drop_block(s, s.xcoef, d, 3)
        x, n, H, gq = surface_point(p, xd, th, ph, gcoef=_drop_block(s, phq, d, 1), ng=1)
        e = sh_point(p, _drop_block(s, en, d, 1), th, ph)[0][0]
        einf = np.array([-Eq * x[0], -Eq * x[1], Eu + 2.0 * Eq * x[2]])
        et = einf - (einf @ n) * n - gq[0]
        fE = 0.5 * ((1.0 - Q / R**2) * e * e - (1.0 - Q) * (et @ et)) * n + (1.0 - Q / R) * e * et
        G, gG = 1.0, np.zeros(3)
        if gamma is not None and eos != 0:
            gd = _drop_block(s, gamma, d, 1)
            G = sh_point(p, gd, th, ph)[0][0]
            gG = surface_point(p, xd, th, ph, gcoef=gd, ng=1)[3][0]
        g, dg = gamma_eos(G, eos, beta, xs)
        f = 2.0 * g * H * n - dg * gG
        ftot[:, i] = fE - f / CaE
        Et[:, i] = et
    return ftot, Et


def explicit_step(s, lam, R, Q, CaE, Eu, Eq, dt, gamma=None, eos=0, beta=0.0, xs=0.0):
    """(E_n, u, x + dt u) as packed coefficient vectors."""
    en = solve_En_dense(s, R, Eu, Eq)
    ftot, _ = forces(s, R, Q, CaE, Eu, Eq, en, gamma, eos, beta, xs)
    fc = project(s, ftot, 3)
    u = solve_velocity_dense(s, lam, fc)
    return en, u, s.xcoef + dt * u


# ---------------------------------------------------------------------------
# Implicit surfactant diffusion (Sec. 2.2, Algorithm 1): (I - kappa Lap_S) Gamma = b
# in Galerkin form, kappa = dt / (2 Pe).
# ---------------------------------------------------------------------------
def lap_values(s, c: np.ndarray) -> np.ndarray:
    """Laplace-Beltrami of the packed field c at every target node."""
    from . import surface_point
    out = []
    for d, th, ph in node_angles(s):
        p = int(s.p[d])
        out.append(surface_point(p, _drop_block(s, s.xcoef, d, 3), th, ph,
                                 gcoef=_drop_block(s, c, d, 1), ng=1, lap=True)[4][0])
    return np.array(out)


def surfactant_apply(s, kappa: float, c: np.ndarray) -> np.ndarray:
    return c - kappa * project(s, lap_values(s, c)[None, :], 1)


def solve_surfactant_dense(s, kappa: float, b: np.ndarray) -> np.ndarray:
    return _dense_solve(lambda v: surfactant_apply(s, kappa, v), np.asarray(b, float), unknown_mask(s, 1))


# ---------------------------------------------------------------------------
# Time stepping (Sec. 2.2, Algorithm 1).  Surface points move with the full
# velocity u; following them, eq. surfactant0 becomes
#   dGamma/dt = -Gamma div_S u + Pe^-1 Lap_S Gamma
# (its convective terms plus the frame term u_t . grad_S Gamma).
# ---------------------------------------------------------------------------
def area_weights(s) -> np.ndarray:
    """(2 pi / nlon) w_j J at every target node (eq. reg_quadrature)."""
    from . import geom_point
    out = []
    for d, th, ph in node_angles(s):
        p = int(s.p[d])
        t, w = gauss_legendre(p + 1)
        j = int(np.argmin(np.abs(np.arccos(t) - th)))
        _, _, J = geom_point(p, _drop_block(s, s.xcoef, d, 3), th, ph)
        out.append(2.0 * np.pi / nlon_of(p, s.grid_mode) * w[j] * J)
    return np.array(out)


def surfactant_terms(s, u: np.ndarray, gamma: np.ndarray, inv_pe: float):
    """g_E = P[-Gamma div_S u] and g_I = P[inv_pe Lap_S Gamma], div_S u the
    trace of the surface gradients of the three velocity components."""
    from . import sh_point, surface_point
    gE, gI = [], []
    for d, th, ph in node_angles(s):
        p = int(s.p[d])
        xd = _drop_block(s, s.xcoef, d, 3)
        gd = _drop_block(s, gamma, d, 1)
        gu = surface_point(p, xd, th, ph, gcoef=_drop_block(s, u, d, 3), ng=3)[3]
        G = sh_point(p, gd, th, ph)[0][0]
        lapG = surface_point(p, xd, th, ph, gcoef=gd, ng=1, lap=True)[4][0]
        gE.append(-G * (gu[0][0] + gu[1][1] + gu[2][2]))
        gI.append(inv_pe * lapG)
    return project(s, np.array(gE)[None, :], 1), project(s, np.array(gI)[None, :], 1)


def _node_values(s, c: np.ndarray, nf: int) -> np.ndarray:
    from . import sh_point
    return np.array([sh_point(int(s.p[d]), _drop_block(s, c, d, nf), th, ph, nf=nf)[0]
                     for d, th, ph in node_angles(s)])


def evolve_step(s, lam, R, Q, CaE, Eu, Eq, inv_pe, dt, gamma, eos=0, beta=0.0, xs=0.0):
    """One step of Algorithm 1: the midpoint rule for x and the second-order
    IMEX Runge-Kutta scheme for Gamma (implicit stage at the half step):
        u0 = u(x, Gamma);  xh = x + dt/2 u0
        (I - dt/(2 Pe) Lap_S(xh)) Gh = Gamma + dt/2 g_E(x, u0, Gamma)
        uh = u(xh, Gh);  x' = x + dt uh;  Gamma' = Gamma + dt (g_E + g_I)(xh, uh, Gh)
    Returns (x', Gamma', err_drop, err_surf) with the errors the largest node
    values of x' - (x + dt u0) and Gamma' - (Gamma + dt (g_E + g_I)(x, u0, Gamma))."""
    gamma = np.asarray(gamma, float)
    _, u0, _ = explicit_step(s, lam, R, Q, CaE, Eu, Eq, 0.0, gamma, eos, beta, xs)
    gE0, gI0 = surfactant_terms(s, u0, gamma, inv_pe)
    sh = dataclasses.replace(s, xcoef=s.xcoef + 0.5 * dt * u0)
    rhs = gamma + 0.5 * dt * gE0
    Gh = solve_surfactant_dense(sh, 0.5 * dt * inv_pe, rhs) if inv_pe > 0 else rhs
    _, uh, _ = explicit_step(sh, lam, R, Q, CaE, Eu, Eq, 0.0, Gh, eos, beta, xs)
    gEh, gIh = surfactant_terms(sh, uh, Gh, inv_pe)
    xnew = s.xcoef + dt * uh
    gnew = gamma + dt * (gEh + gIh)
    err_drop = np.abs(_node_values(s, dt * (uh - u0), 3)).max()
    err_surf = dt * np.abs(_node_values(s, (gEh + gIh) - (gE0 + gI0), 1)).max()
    return xnew, gnew, err_drop, err_surf
