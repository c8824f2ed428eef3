"""Pins of the oracle's surface quantities (mean curvature H = (1/2) div_S n
and the surface gradient, Sec. 1 after eq. interfacial_force):
closed forms on spheres and ellipsoids, scipy's spherical harmonics on the
unit sphere, and the surface divergence identity
    int_S grad_S g dA = int_S 2 H g n dA
on a deformed drop (it holds on any closed smooth surface)."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
from paper_1811_10270_amd import workloads as W
from test_oracle_pins import field, sphere_x, y_entry


def test_sphere_curvature_and_normal():
    p, R, c = 6, 2.0, np.array([0.3, -0.2, 1.0])
    x = sphere_x(p, R=R, centre=tuple(c))
    for th, ph in [(0.3, 0.1), (1.2, 2.0), (2.9, 5.0)]:
        xx, n, H, _ = oracle.surface_point(p, x, th, ph)
        assert abs(H - 1 / R) < 1e-14
        assert np.abs(n - (xx - c) / R).max() < 1e-14


def test_ellipsoid_mean_curvature():
    p, (a, b, c) = 5, (1.3, 0.8, 1.1)
    x = sphere_x(p, axes=(a, b, c))
    for th, ph in [(0.2, 0.4), (1.0, 2.2), (1.9, 4.1), (2.8, 5.9)]:
        (X, Y, Z), n, H, _ = oracle.surface_point(p, x, th, ph)
        h = 1.0 / math.sqrt(X * X / a**4 + Y * Y / b**4 + Z * Z / c**4)
        Hex = (a * a + b * b + c * c - X * X - Y * Y - Z * Z) * h**3 / (2 * a * a * b * b * c * c)
        assert abs(H - Hex) < 1e-13


@pytest.mark.parametrize("nm", [(1, 0), (2, 1), (3, 3), (5, 2)])
def test_unit_sphere_surface_gradient_of_Ynm(nm):
    n, m = nm
    p = 6
    g = field(p, y_entry(n, m))            # real field Re Y_nm (scaled as in y_entry)
    hstep = 1e-5
    for th, ph in [(0.4, 0.3), (1.3, 2.5), (2.6, 4.4)]:
        _, nrm, _, grad = oracle.surface_point(p, sphere_x(p), th, ph, gcoef=g, ng=1)

        def val(t, f):
            return np.real(sph_harm_y(n, m, t, f))
        gt = (val(th + hstep, ph) - val(th - hstep, ph)) / (2 * hstep)
        gp = (val(th, ph + hstep) - val(th, ph - hstep)) / (2 * hstep) / math.sin(th)
        et = np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)])
        ep = np.array([-math.sin(ph), math.cos(ph), 0.0])
        assert np.abs(grad[0] - (gt * et + gp * ep)).max() < 1e-8
        assert abs(float(grad[0] @ nrm)) < 1e-13


def test_surface_divergence_identity_on_deformed_drop():
    s = W.single_drop(p=8, seed=2, eps_y20=0.2, amp=0.02)
    p = 8
    rng = np.random.default_rng(3)
    g = np.zeros((p + 1) * (p + 2))
    for n in range(p + 1):
        for m in range(n + 1):
            k = n * (n + 1) // 2 + m
            g[2 * k] = rng.standard_normal() / (n + 1) ** 2
            if m:
                g[2 * k + 1] = rng.standard_normal() / (n + 1) ** 2
    errs = []
    for Q in (24, 40):
        t, w = oracle.gauss_legendre(Q + 1)
        nl = 2 * Q + 2
        lhs = np.zeros(3)
        rhs = np.zeros(3)
        for j in range(Q + 1):
            th = math.acos(t[j])
            for k in range(nl):
                ph = 2 * math.pi * k / nl
                _, nrm, H, grad = oracle.surface_point(p, s.xcoef, th, ph, gcoef=g, ng=1)
                _, _, J = oracle.geom_point(p, s.xcoef, th, ph)
                wt = 2 * math.pi / nl * w[j] * J
                gv = oracle.sh_point(p, g, th, ph)[0][0]
                lhs += wt * grad[0]
                rhs += wt * 2 * H * gv * nrm
        errs.append(np.abs(lhs - rhs).max())
    assert errs[-1] < 1e-11 and errs[-1] <= errs[0] + 1e-14, errs


@pytest.mark.parametrize("nm", [(1, 1), (2, 0), (4, 3)])
def test_sphere_laplace_beltrami_eigenvalues(nm):
    """Lap_S Y_nm = -n(n+1)/a^2 Y_nm on a sphere of radius a."""
    n, m = nm
    p, a = 6, 1.7
    g = field(p, y_entry(n, m))
    x = sphere_x(p, R=a, centre=(0.2, 0.1, -0.4))
    for th, ph in [(0.5, 0.2), (1.4, 3.0), (2.7, 5.5)]:
        _, _, _, _, lap = oracle.surface_point(p, x, th, ph, gcoef=g, ng=1, lap=True)
        val = oracle.sh_point(p, g, th, ph)[0][0]
        assert abs(lap[0] + n * (n + 1) / a**2 * val) < 1e-12


def test_laplace_beltrami_green_identities_on_deformed_drop():
    """int Lap_S g dA = 0, int f Lap_S g dA = int g Lap_S f dA and
    int g Lap_S g dA = -int |grad_S g|^2 dA on a closed deformed surface."""
    s = W.single_drop(p=7, seed=5, eps_y20=0.25, amp=0.03)
    p = 7
    rng = np.random.default_rng(8)
    fg = np.zeros(2 * (p + 1) * (p + 2))
    for c in range(2):
        for n in range(p + 1):
            for m in range(n + 1):
                k = c * (p + 1) * (p + 2) + 2 * (n * (n + 1) // 2 + m)
                fg[k] = rng.standard_normal() / (n + 1) ** 2
                if m:
                    fg[k + 1] = rng.standard_normal() / (n + 1) ** 2
    Q = 36
    t, w = oracle.gauss_legendre(Q + 1)
    nl = 2 * Q + 2
    i_lap = i_sym1 = i_sym2 = i_e1 = i_e2 = 0.0
    for j in range(Q + 1):
        th = math.acos(t[j])
        for k in range(nl):
            ph = 2 * math.pi * k / nl
            _, _, _, grad, lap = oracle.surface_point(p, s.xcoef, th, ph, gcoef=fg, ng=2, lap=True)
            _, _, J = oracle.geom_point(p, s.xcoef, th, ph)
            wt = 2 * math.pi / nl * w[j] * J
            fv, gv = oracle.sh_point(p, fg, th, ph, nf=2)[0]
            i_lap += wt * lap[1]
            i_sym1 += wt * fv * lap[1]
            i_sym2 += wt * gv * lap[0]
            i_e1 += wt * gv * lap[1]
            i_e2 -= wt * float(grad[1] @ grad[1])
    assert abs(i_lap) < 1e-10
    assert abs(i_sym1 - i_sym2) < 1e-10
    assert abs(i_e1 - i_e2) < 1e-10
