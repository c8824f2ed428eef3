"""Pins of the oracle's Galerkin systems (eq. galerkin_En, eq. BIM_galerkin).

On the unit sphere the singular rule is exact (pinned in test_oracle_pins)
and the systems have closed-form solutions:
  * uniform field E_u z: E_n = 3R/(R+2) E_u cos(theta);
  * quadrupole field: E_n = 10 R E_q P_2(cos theta) / (2R+3)
    (K*[Y_nm] = Y_nm / (2(2n+1)) on the unit sphere);
  * constant force density e: u = (2/3) e for every viscosity ratio
    (S[e] = (4/3) e and D[e] = e on the unit sphere);
  * an ellipsoid in a uniform field along a principal axis has a uniform
    interior field E / (1 + (R - 1) L) with L its depolarisation factor.
With R = 1 or lambda = 1 the systems reduce to projections, which pins the
right-hand sides on a deformed drop.
"""
import math

import numpy as np
import pytest

from oracle import galerkin as G
from paper_1811_10270_amd import workloads as W
from test_oracle_pins import make_susp, sphere_x, tri


@pytest.mark.parametrize("R", [0.5, 3.0])
def test_En_unit_sphere_uniform_field(R):
    p = 4
    s = make_susp(p, sphere_x(p), q_self=8)
    en = G.solve_En_dense(s, R, 1.0, 0.0)
    expect = np.zeros_like(en)
    expect[2 * tri(1, 0)] = 3 * R / (R + 2) * math.sqrt(4 * math.pi / 3)
    assert np.abs(en - expect).max() < 1e-12


def depolarisation(axes, i):
    """Depolarisation factor of the ellipsoid with semi-axes `axes` along
    axis i: (abc/2) times the integral over s > 0 of
    1 / ((s + a_i^2) sqrt((s + a^2)(s + b^2)(s + c^2))); 1/3 on a sphere."""
    from scipy.integrate import quad
    a, b, c = axes

    def f(t):
        return 1.0 / ((t + axes[i] ** 2) * math.sqrt((t + a * a) * (t + b * b) * (t + c * c)))
    return 0.5 * a * b * c * quad(f, 0.0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=200)[0]


def ellipsoid_En_error(axes, p, R, L=None):
    """Largest node error of the Galerkin E_n on the ellipsoid `axes` in a
    uniform field along z against the textbook solution: the interior field
    is uniform, E / (1 + (R - 1) L_z), so E_n = R E n_z / (1 + (R - 1) L_z)."""
    import oracle
    s = make_susp(p, sphere_x(p, axes=axes))
    en = G.solve_En_dense(s, R, 1.0, 0.0)
    td, tn = oracle.all_targets(s)
    _, n = oracle.targets(s, td, tn)
    Lz = depolarisation(axes, 2) if L is None else L
    return np.abs(G._node_values(s, en, 1)[:, 0] - R * n[2] / (1.0 + (R - 1.0) * Lz)).max()


def test_depolarisation_factors():
    assert abs(depolarisation((1.0, 1.0, 1.0), 2) - 1.0 / 3.0) < 1e-13
    axes = (1.15, 0.9, 1.0)
    assert abs(sum(depolarisation(axes, i) for i in range(3)) - 1.0) < 1e-12
    # prolate spheroid along z, eccentricity e: L_z = (1 - e^2)/e^3 (atanh e - e)
    e = math.sqrt(1.0 - 1.0 / 1.2 ** 2)
    assert abs(depolarisation((1.0, 1.0, 1.2), 2) - (1 - e * e) / e ** 3 * (math.atanh(e) - e)) < 1e-12


@pytest.mark.parametrize("R", [0.5, 3.0])
def test_En_prolate_spheroid_uniform_field(R):
    """A spheroid (the surface is exactly degree 1; only n_z is not band-
    limited): the Galerkin E_n at the nodes within 1e-7 of the ellipsoid's
    closed form at p = 8, while the sphere's factor 1/3 misses by 1e-2."""
    axes = (1.0, 1.0, 1.2)
    err = ellipsoid_En_error(axes, 8, R)
    assert err < 1e-7, err
    assert ellipsoid_En_error(axes, 8, R, L=1.0 / 3.0) > 1e-2


def test_En_triaxial_ellipsoid_converges():
    """A triaxial ellipsoid: the error against the closed form falls about
    tenfold per two degrees (spectral convergence to the exact solution)."""
    axes = (1.15, 0.9, 1.0)
    e6, e8 = ellipsoid_En_error(axes, 6, 3.0), ellipsoid_En_error(axes, 8, 3.0)
    assert e8 < 1e-4 and e8 < e6 / 5, (e6, e8)


@pytest.mark.parametrize("R", [0.25, 4.0])
def test_En_unit_sphere_quadrupole_field(R):
    p = 4
    s = make_susp(p, sphere_x(p), q_self=8)
    Eq = 0.7
    en = G.solve_En_dense(s, R, 0.0, Eq)
    expect = np.zeros_like(en)
    expect[2 * tri(2, 0)] = 10 * R * Eq / (2 * R + 3) * math.sqrt(4 * math.pi / 5)
    assert np.abs(en - expect).max() < 1e-12


@pytest.mark.parametrize("lam", [0.3, 2.0])
def test_velocity_unit_sphere_constant_traction(lam):
    p = 3
    nc2 = (p + 1) * (p + 2)
    e = np.array([0.3, -1.1, 0.7])
    f = np.zeros(3 * nc2)
    for c in range(3):
        f[c * nc2] = e[c] * math.sqrt(4 * math.pi)
    s = make_susp(p, sphere_x(p), f=f, q_self=6)
    u = G.solve_velocity_dense(s, lam, f)
    assert np.abs(u - 2.0 / 3.0 * f).max() < 1e-12


def test_R1_and_lambda1_reduce_to_projections():
    s = W.single_drop(p=5, seed=4)
    en = G.solve_En_dense(s, 1.0, 0.8, 0.3)
    direct = G.project(s, G.einf_dot_n(s, 0.8, 0.3)[None, :], 1)
    assert np.abs(en - direct).max() < 1e-12 * max(1.0, np.abs(direct).max())
    u = G.solve_velocity_dense(s, 1.0, s.fcoef)
    assert np.abs(u - 0.5 * G.velocity_rhs(s, s.fcoef)).max() < 1e-12


def test_dense_solution_satisfies_the_system():
    s = W.two_drops(3, seed=7)
    R = 2.5
    en = G.solve_En_dense(s, R, 1.0, 0.2)
    res = G.En_apply(s, R, en) - G.En_rhs(s, R, 1.0, 0.2)
    assert np.abs(res[G.unknown_mask(s, 1)]).max() < 1e-12
    assert np.all(en[~G.unknown_mask(s, 1)] == 0.0)


@pytest.mark.parametrize("R", [0.5, 3.0])
def test_tangential_field_on_sphere(R):
    """Unit sphere in a uniform field: the interior field is uniform,
    3/(R+2) E_u z, and E_t is its tangential part."""
    p = 4
    s = make_susp(p, sphere_x(p), q_self=8)
    en = G.solve_En_dense(s, R, 1.0, 0.0)
    _, Et = G.forces(s, R, 2.0, 1.0, 1.0, 0.0, en)
    for i, (d, th, ph) in enumerate(G.node_angles(s)):
        n = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        ez = np.array([0.0, 0.0, 1.0])
        assert np.abs(Et[:, i] - 3.0 / (R + 2) * (ez - math.cos(th) * n)).max() < 1e-12


def test_clean_sphere_without_field_stays_at_rest():
    p = 4
    s = make_susp(p, sphere_x(p, R=1.3), q_self=8)
    en, u, xnew = G.explicit_step(s, 2.0, 0.5, 2.0, 0.4, 0.0, 0.0, 0.05)
    assert np.abs(en).max() < 1e-13 and np.abs(u).max() < 1e-12
    assert np.abs(xnew - s.xcoef).max() < 1e-13


def test_uniform_surfactant_matches_clean_drop():
    """Gamma = 1 everywhere: gamma = 1 and grad_S gamma = 0 for every law."""
    s = W.two_drops(3, seed=21, gap=0.4)
    g1 = np.zeros(len(s.sigcoef))
    off = 0
    for p in (int(x) for x in s.p):
        g1[off] = math.sqrt(4 * math.pi)
        off += (p + 1) * (p + 2)
    en = G.solve_En_dense(s, 0.5, 1.0, 0.0)
    a, _ = G.forces(s, 0.5, 2.0, 0.3, 1.0, 0.0, en)
    b, _ = G.forces(s, 0.5, 2.0, 0.3, 1.0, 0.0, en, gamma=g1, eos=2, beta=0.5, xs=0.3)
    assert np.abs(a - b).max() < 1e-12


def test_surfactant_system_on_unit_sphere_is_diagonal():
    """Lap_S Y_nm = -n(n+1) Y_nm: the Galerkin system is diag(1 + kappa n(n+1))."""
    p = 5
    s = make_susp(p, sphere_x(p), q_self=10)
    rng = np.random.default_rng(41)
    b = rng.standard_normal((p + 1) * (p + 2))
    for n in range(p + 1):
        b[2 * tri(n, 0) + 1] = 0.0
    kappa = 0.07
    c = G.solve_surfactant_dense(s, kappa, b)
    expect = b.copy()
    for n in range(p + 1):
        for m in range(n + 1):
            expect[2 * tri(n, m):2 * tri(n, m) + 2] /= 1 + kappa * n * (n + 1)
    assert np.abs(c - expect).max() < 1e-12
