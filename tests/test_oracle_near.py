"""Accuracy of the upsampled direct sums near another drop (the regular rule
of eq. reg_quadrature on a degree-q grid; Sec. 2.1 replaces it by line
interpolation for nearly singular targets, which is not built).  Against the
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
