"""Pin of the oracle's explicit step against Taylor's small-deformation
theory (Sec. 3, linear theory; clean drop, viscosity ratio 1, uniform field).

At the first-order shape x = (1 + Ca_E F_20 P_2(cos theta)) r_hat with
F_20 = 3 (2 + 3R + 2R^2 - 7Q) / (8 (2 + R)^2) and E_u = 1, the O(1) electric
and capillary normal stresses balance, so the normal velocity of one step
vanishes to first order: |u.n| = O(Ca_E).  The sphere, or the shape with
twice that deformation, leaves an O(1) normal velocity.  A wrong sign or
factor in E_n, E_t, f^E, the mean curvature or the velocity solve breaks
the balance."""
import math

import numpy as np
import pytest

import oracle
from oracle import galerkin as G
from paper_1811_10270_amd import workloads as W
from test_oracle_pins import make_susp, sphere_x, tri


def taylor_f20(R, Q):
    return 3.0 * (2.0 + 3.0 * R + 2.0 * R * R - 7.0 * Q) / (8.0 * (2.0 + R) ** 2)


def p2_shape(p, a):
    """Coefficients of x = (1 + a P_2(cos theta)) r_hat (P_2 unnormalised)."""
    blk = sphere_x(p)
    nc2 = (p + 1) * (p + 2)
    eps = a / math.sqrt(5.0 / (4.0 * math.pi))       # a P_2 = eps Y_20
    for (c, n, m), v in W.Y20_STRETCH_TABLE.items():
        if n <= p:
            k = c * nc2 + 2 * tri(n, m)
            blk[k] += (v * eps).real
            blk[k + 1] += (v * eps).imag
    return blk


def normal_velocity_rms(p, a, R, Q, Ca):
    s = make_susp(p, p2_shape(p, a))
    _, u, _ = G.explicit_step(s, 1.0, R, Q, Ca, 1.0, 0.0, 0.0)
    _, n0 = oracle.targets(s, *oracle.all_targets(s))
    un = [oracle.sh_point(p, u, th, ph, nf=3)[0] @ n0[:, i] for i, (_, th, ph) in enumerate(G.node_angles(s))]
    return math.sqrt(np.mean(np.square(un)))


@pytest.mark.parametrize("R,Q", [(2.0, 1.0), (0.5, 2.0)])      # prolate (F_20 > 0), oblate (F_20 < 0)
def test_taylor_shape_is_stationary_to_first_order(R, Q):
    p = 4
    F = taylor_f20(R, Q)
    big, small = (normal_velocity_rms(p, Ca * F, R, Q, Ca) for Ca in (0.04, 0.02))
    assert 1.8 < big / small < 2.2                          # |u.n| = O(Ca_E)
    for wrong in (0.0, 2.0 * F):                            # the sphere, twice the deformation
        assert normal_velocity_rms(p, 0.02 * wrong, R, Q, 0.02) > 20.0 * small
