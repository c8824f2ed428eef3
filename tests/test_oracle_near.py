"""Accuracy of the upsampled direct sums near another drop (the regular rule
of eq. reg_quadrature on a degree-q grid; Sec. 2.1 replaces it by line
interpolation for nearly singular targets, pinned below and built on the
device as an option of the library).  Against the
exterior unit-sphere closed forms S_L[Y_nm](x0) = Y_nm(d)/((2n+1)|x0|^{n+1})
and L[Y_nm](x0) = n Y_nm(d)/((2n+1)|x0|^{n+1}), d = x0/|x0|: with q = 3p
(p = 32) the sums hold 1e-7 at a gap of 0.1 (the two-drop workload) and fail
at 0.03."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
from test_oracle_pins import field, make_susp, sphere_x, y_entry


def exterior(p, n, m, gap, q):
    th, ph = 1.1, 0.7
    d = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    r = 1.0 + gap
    y = float(np.real(sph_harm_y(n, m, th, ph)))          # the field of y_entry(n, m): Re Y_nm
    s = make_susp(p, sphere_x(p), sig=field(p, y_entry(n, m)), q_far=q)
    out = oracle.far_points(s, (r * d)[:, None], d[:, None])
    ex_sl, ex_l = y / ((2 * n + 1) * r ** (n + 1)), n * y / ((2 * n + 1) * r ** (n + 1))
    return abs(out[6, 0] / ex_sl - 1.0), abs(out[7, 0] / ex_l - 1.0)


@pytest.mark.parametrize("nm", [(2, 0), (5, 3)])
def test_upsampled_sums_near_a_drop(nm):
    p = 32
    e_sl, e_l = exterior(p, *nm, 0.1, 3 * p)
    assert e_sl < 1e-8 and e_l < 1e-7
    e_sl, e_l = exterior(p, *nm, 0.03, 3 * p)
    assert e_l > 1e-3                      # too close for the regular rule at q = 3p


# ---------------------------------------------------------------------------
# Line interpolation for nearly singular targets (the oracle's reading of
# Sec. 2.1's interpolation approach; the device path is checked against it
# in the GPU tests of the nearly singular correction)
# ---------------------------------------------------------------------------
def test_line_interpolation_laplace_near_the_unit_sphere():
    """S_L, L and K* (target normal radial) of sigma = Re Y_31 at 0.05, 0.01
    and 0.002 from the unit sphere (p = 16, q_far = 2p): the interpolated
    values match the closed forms within 1e-6 where the plain sums are off by
    1e-2 to O(1).  Check points on a degree-160 grid, delta = 0.06, m = 8."""
    from oracle import near as N
    p, n, m = 16, 3, 1
    s = make_susp(p, sphere_x(p), sig=field(p, y_entry(n, m)), q_far=2 * p)
    th, ph = 1.1, 0.7
    d = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    y = float(np.real(sph_harm_y(n, m, th, ph)))
    for gap in (0.05, 0.01, 0.002):
        r = 1.0 + gap
        exact = np.array([y / ((2 * n + 1) * r ** (n + 1)), n * y / ((2 * n + 1) * r ** (n + 1)),
                          (n + 1) * y / ((2 * n + 1) * r ** (n + 2))])
        corr, plain, info = N.near_value(s, 0, r * d, d, 0.06, 8, q_check=160)
        assert abs(info["dist"] - gap) < 1e-12
        assert np.abs(corr[6:9] / exact - 1.0).max() < 1e-6
        if gap <= 0.01:
            assert np.abs(plain[6:9] / exact - 1.0).max() > 1e-2


def test_line_interpolation_stokes_near_the_unit_sphere():
    """Constant traction e and velocity u = e on the unit sphere: outside,
    S[e] is the translating-sphere field and the double layer of a rigid
    translation vanishes.  At 0.005 from the surface the interpolated values
    hold 1e-6; the plain sums miss D by O(1)."""
    from oracle import near as N
    p = 8
    nc2 = (p + 1) * (p + 2)
    e = np.array([0.5, 1.0, -0.25])
    f = np.zeros(3 * nc2)
    for c in range(3):
        f[c * nc2] = e[c] * math.sqrt(4 * math.pi)
    s = make_susp(p, sphere_x(p), f=f, u=f.copy(), q_far=2 * p)
    dvec = np.array([0.3, -0.5, 0.8])
    dvec /= np.linalg.norm(dvec)
    x0 = 1.005 * dvec
    dn = np.linalg.norm(x0)
    S_ref = (np.eye(3) / dn + np.outer(x0, x0) / dn ** 3 + (np.eye(3) / dn ** 3 - 3 * np.outer(x0, x0) / dn ** 5) / 3.0) @ e
    corr, plain, _ = N.near_value(s, 0, x0, dvec, 0.06, 8, q_check=160)
    assert np.abs(corr[0:3] - S_ref).max() < 1e-6 * np.abs(S_ref).max()
    assert np.abs(corr[3:6]).max() < 1e-6
    assert np.abs(plain[3:6]).max() > 1e-2
