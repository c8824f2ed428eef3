"""Pins of the oracle's time step (Sec. 2.2, Algorithm 1).

* On a sphere at rest (clean drop, no field: the capillary force 2n/Ca_E
  drives no flow since S[n] = 0), only diffusion acts and Lap_S Y_nm =
  -n(n+1) Y_nm, so the IMEX scheme with its implicit stage at the half step
  multiplies each coefficient by exactly (1 - k)/(1 + k), k = dt n(n+1) / (2 Pe).
* Surfactant mass and drop volume are invariants of the continuous problem
  (surfactant conservation; an incompressible velocity).  With a flow and a
  Marangoni stress on a deformed drop, one second-order step changes them by
  far less than the step's own change of the drop, and the changes fall with
  dt faster than dt^2; a wrong sign or factor in the convective term would
  leave an O(dt) mass change.
* The error estimates compare with first-order updates: they fall as dt^2."""
import dataclasses
import math

import numpy as np

import oracle
from oracle import galerkin as G
from test_oracle_pins import make_susp, sphere_x, tri
from test_oracle_taylor import p2_shape


def rough_gamma(p, amp, seed):
    rng = np.random.default_rng(seed)
    g = np.zeros((p + 1) * (p + 2))
    g[0] = math.sqrt(4 * math.pi)
    for n in range(1, p + 1):
        for m in range(n + 1):
            k = 2 * tri(n, m)
            g[k] = amp * rng.standard_normal() / n
            if m:
                g[k + 1] = amp * rng.standard_normal() / n
    return g


def test_diffusion_on_a_sphere_at_rest():
    p, dt, inv_pe = 5, 0.1, 0.5
    s = make_susp(p, sphere_x(p))
    g = rough_gamma(p, 0.1, 1)
    xn, gn, ed, _ = G.evolve_step(s, 1.0, 2.0, 1.0, 0.2, 0.0, 0.0, inv_pe, dt, g)
    expect = g.copy()
    for n in range(p + 1):
        k = 0.5 * dt * inv_pe * n * (n + 1)
        for m in range(n + 1):
            expect[2 * tri(n, m):2 * tri(n, m) + 2] *= (1.0 - k) / (1.0 + k)
    assert np.abs(gn - expect).max() < 1e-13
    assert np.abs(xn - s.xcoef).max() < 1e-13 and ed < 1e-13


def invariants(s, g):
    w = G.area_weights(s)
    x0, n0 = oracle.targets(s, *oracle.all_targets(s))
    return (w * G._node_values(s, g, 1)[:, 0]).sum(), (w * (x0 * n0).sum(0)).sum() / 3.0


def test_mass_and_volume_conservation_and_error_order():
    p = 5
    s = make_susp(p, p2_shape(p, 0.15))
    g = rough_gamma(p, 0.05, 2)
    m0, v0 = invariants(s, g)
    res = []
    for dt in (0.04, 0.02):
        xn, gn, ed, es = G.evolve_step(s, 1.0, 2.0, 1.0, 0.2, 1.0, 0.0, 0.1, dt, g, eos=1, beta=0.3)
        m1, v1 = invariants(dataclasses.replace(s, xcoef=xn), gn)
        shape_change = np.abs(xn - s.xcoef).max()
        res.append((abs(m1 / m0 - 1.0), abs(v1 / v0 - 1.0), ed, es, shape_change))
    (dm1, dv1, ed1, es1, ch1), (dm2, dv2, ed2, es2, ch2) = res
    assert dm1 < 1e-3 * ch1 and dv1 < 1e-3 * ch1
    assert dm2 < dm1 / 4.0 and dv2 < dv1 / 4.0
    assert 3.5 < ed1 / ed2 < 4.5 and 3.5 < es1 / es2 < 4.5
