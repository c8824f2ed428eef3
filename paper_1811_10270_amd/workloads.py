"""Seeded synthetic drop suspensions (inputs only).

This module serves both the HIP path and the test oracle, so it holds no
layer-potential arithmetic: it only draws random numbers and places them in
the packed spherical-harmonic (SH) coefficient layout that the library and
the oracle both read.

Conventions (the paper, Sec. 2, eq. normalized_spharm and eq. pneg):
orthonormal complex SH with the Condon-Shortley phase.  A real field is
stored by its m >= 0 coefficients c_nm; the m < 0 ones follow from
c_{n,-m} = (-1)^m conj(c_nm).

Packed layout of a K-field array: drops one after another; drop d's block
starts at K * off[d] doubles with off[d] = sum_{e<d} (p_e+1)(p_e+2); inside a
block the K fields follow one another, each holding (p+1)(p+2)/2 complex
numbers, (re, im) interleaved, at index n(n+1)/2 + m.

Shapes are given directly by the coefficients of the three Cartesian
components of x (the paper represents x, not the radius):
  * a sphere of radius R centred at c has the degree-0/1 coefficients in
    ``SPHERE_TABLE`` (a fixed table of the SH normalisation constants);
  * the Taylor-type deformation r = 1 + eps*Y_20 of the single-drop case is
    added through ``Y20_STRETCH_TABLE``, the exact SH coefficients of
    Y_20(s) * s for the unit vector s (degree 1 and 3 terms only);
  * random shape perturbations are added to every Cartesian component,
    amplitude A * n^-2 * N(0,1) (real and imaginary parts for m > 0),
    degrees n = 1..p.
Densities have coefficients max(n,1)^-2 * N(0,1), n = 0..p.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# Fixed tables (SH normalisation constants; no method arithmetic)
# --------------------------------------------------------------------------
_S23 = math.sqrt(2.0 * math.pi / 3.0)
# unit vector s = (sin t cos p, sin t sin p, cos t): (component, n, m) -> complex
SPHERE_TABLE = {
    (0, 1, 1): complex(-_S23, 0.0),
    (1, 1, 1): complex(0.0, _S23),
    (2, 1, 0): complex(math.sqrt(4.0 * math.pi / 3.0), 0.0),
}
# Y_20(s) * s, with Y_20 = sqrt(5/4pi) P_2(cos t):
#   z: cos t P_2 = (3 P_3 + 2 P_1)/5 ; x,y: sin t P_2 = (P_1^1 - P_3^1)/5
_Y20 = math.sqrt(5.0 / (4.0 * math.pi))
_N11 = math.sqrt(3.0 / (8.0 * math.pi))
_N31 = math.sqrt(7.0 / (48.0 * math.pi))
Y20_STRETCH_TABLE = {
    (0, 1, 1): complex(_Y20 / (10.0 * _N11), 0.0),
    (0, 3, 1): complex(-_Y20 / (10.0 * _N31), 0.0),
    (1, 1, 1): complex(0.0, -_Y20 / (10.0 * _N11)),
    (1, 3, 1): complex(0.0, _Y20 / (10.0 * _N31)),
    (2, 1, 0): complex(0.4 * math.sqrt(5.0 / 3.0), 0.0),
    (2, 3, 0): complex(0.6 * math.sqrt(5.0 / 7.0), 0.0),
}


def ncoef(p: int) -> int:
    """Number of stored complex coefficients (m >= 0) of a degree-p field."""
    return (p + 1) * (p + 2) // 2


def tri(n: int, m: int) -> int:
    return n * (n + 1) // 2 + m


def grid_dims(P: int, grid_mode: int) -> tuple[int, int]:
    """(nlat, nlon) of the degree-P Gaussian grid.

    grid_mode 0: 2P+2 longitudes (the paper's grid, Sec. 2);
    grid_mode 1: 2P longitudes (the grids the workload descriptions quote)."""
    return P + 1, (2 * P + 2 if grid_mode == 0 else 2 * P)


def drop_offsets(p: np.ndarray) -> np.ndarray:
    """off[d] in doubles per field, plus the total as the last entry."""
    sizes = (p + 1) * (p + 2)
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


@dataclass
class Suspension:
    name: str
    p: np.ndarray                 # int32 [ndrops]
    q_self: np.ndarray            # int32 [ndrops]
    q_far: np.ndarray             # int32 [ndrops]
    grid_mode: int
    xcoef: np.ndarray             # float64 packed, 3 fields
    fcoef: np.ndarray             # float64 packed, 3 fields
    sigcoef: np.ndarray           # float64 packed, 1 field
    ucoef: np.ndarray | None = None   # float64 packed, 3 fields (None: u = f)
    centres: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    radius_bound: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def ndrops(self) -> int:
        return int(self.p.shape[0])

    def ntargets(self) -> int:
        return int(sum(grid_dims(int(pp), self.grid_mode)[0] * grid_dims(int(pp), self.grid_mode)[1]
                       for pp in self.p))

    def target_offsets(self) -> np.ndarray:
        sizes = [grid_dims(int(pp), self.grid_mode)[0] * grid_dims(int(pp), self.grid_mode)[1]
                 for pp in self.p]
        return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


# --------------------------------------------------------------------------
# Building blocks
# --------------------------------------------------------------------------
def _put(buf: np.ndarray, base: int, p: int, field_idx: int, n: int, m: int, val: complex):
    k = base + field_idx * 2 * ncoef(p) + 2 * tri(n, m)
    buf[k] += val.real
    buf[k + 1] += val.imag


def _random_field(rng: np.random.Generator, p: int, amp: float, nmin: int) -> np.ndarray:
    """One field's packed coefficients: amp * max(n,1)^-2 * N(0,1), n >= nmin.

    Draw order: n ascending, m ascending, real part then (m > 0) imaginary."""
    out = np.zeros(2 * ncoef(p))
    for n in range(nmin, p + 1):
        a = amp / float(max(n, 1)) ** 2
        for m in range(n + 1):
            k = 2 * tri(n, m)
            out[k] = a * rng.standard_normal()
            if m > 0:
                out[k + 1] = a * rng.standard_normal()
    return out


def shape_perturbation_bound(block3: np.ndarray, p: int) -> float:
    """Upper bound on |delta x(s)| over the sphere for the n >= 1 part of a
    3-field block, from Cauchy-Schwarz and sum_m |Y_nm|^2 = (2n+1)/(4 pi)."""
    tot = 0.0
    for c in range(3):
        fb = block3[c * 2 * ncoef(p):(c + 1) * 2 * ncoef(p)]
        bc = 0.0
        for n in range(1, p + 1):
            s = 0.0
            for m in range(n + 1):
                k = 2 * tri(n, m)
                mag2 = fb[k] ** 2 + fb[k + 1] ** 2
                s += mag2 if m == 0 else 2.0 * mag2
            bc += math.sqrt(s) * math.sqrt((2 * n + 1) / (4.0 * math.pi))
        tot += bc * bc
    return math.sqrt(tot)


def _drop_shape(rng, p: int, centre, radius: float, eps_y20: float, amp: float):
    """Packed 3-field block of one drop and a bound on the radius |x - c|."""
    blk = np.zeros(3 * 2 * ncoef(p))
    pert = np.zeros(3 * 2 * ncoef(p))
    for c in range(3):
        _put(blk, 0, p, c, 0, 0, complex(math.sqrt(4.0 * math.pi) * centre[c], 0.0))
    for (c, n, m), v in SPHERE_TABLE.items():
        _put(blk, 0, p, c, n, m, v * radius)
    if eps_y20 != 0.0:
        for (c, n, m), v in Y20_STRETCH_TABLE.items():
            if n <= p:
                _put(blk, 0, p, c, n, m, v * eps_y20 * radius)
    if amp > 0.0:
        for c in range(3):
            pert[c * 2 * ncoef(p):(c + 1) * 2 * ncoef(p)] = _random_field(rng, p, amp, 1)
    blk += pert
    # |Y_20| <= sqrt(5/4pi) < 0.64
    rbound = radius * (1.0 + 0.64 * abs(eps_y20)) + shape_perturbation_bound(pert, p)
    return blk, rbound


def _densities(rng, p_list, three: int) -> np.ndarray:
    parts = []
    for p in p_list:
        for _ in range(three):
            parts.append(_random_field(rng, int(p), 1.0, 0))
    return np.concatenate(parts) if parts else np.zeros(0)


def _rsa(rng, radii: np.ndarray, side: float, gap: float, max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition of centres in [0, side]^3 with
    |c_i - c_j| >= R_i + R_j + gap."""
    n = len(radii)
    cs = np.zeros((n, 3))
    placed = 0
    tries = 0
    while placed < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        c = rng.uniform(0.0, side, size=3)
        if placed:
            d = np.linalg.norm(cs[:placed] - c, axis=1)
            if np.any(d < radii[:placed] + radii[placed] + gap):
                continue
        cs[placed] = c
        placed += 1
    return cs


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
def single_drop(p: int = 16, seed: int = 1, grid_mode: int = 0, upsample: int = 2,
                eps_y20: float = 0.1, amp: float = 1e-3) -> Suspension:
    """One drop, shape r = 1 + eps*Y_20 plus random coefficients of amplitude
    amp*n^-2; densities f (3) and sigma (1) with coefficients ~ max(n,1)^-2."""
    rng = np.random.default_rng(seed)
    x, rb = _drop_shape(rng, p, (0.0, 0.0, 0.0), 1.0, eps_y20, amp)
    f = _densities(rng, [p], 3)
    s = _densities(rng, [p], 1)
    pa = np.array([p], np.int32)
    return Suspension("single_drop_p%d" % p, pa, pa * upsample, pa * upsample, grid_mode,
                      x, f, s, None, np.zeros((1, 3)), np.array([rb]))


def two_drops(p: int = 32, seed: int = 2, grid_mode: int = 0, gap: float = 0.1,
              q_self_mult: int = 2, q_far_mult: int = 3) -> Suspension:
    """Two unit spheres, surface gap `gap` along a random axis."""
    rng = np.random.default_rng(seed)
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    half = 0.5 * (2.0 + gap)
    centres = np.stack([-half * axis, half * axis])
    x = np.concatenate([_drop_shape(rng, p, centres[d], 1.0, 0.0, 0.0)[0] for d in range(2)])
    f = _densities(rng, [p, p], 3)
    s = _densities(rng, [p, p], 1)
    pa = np.array([p, p], np.int32)
    return Suspension("two_drops_p%d" % p, pa, pa * q_self_mult, pa * q_far_mult, grid_mode,
                      x, f, s, None, centres, np.ones(2))


def suspension(ndrops: int, p_choices, side: float, seed: int, grid_mode: int = 0,
               amp: float = 0.05, gap: float = 0.2, upsample: int = 2,
               name: str = "suspension", balanced: bool = True) -> Suspension:
    """`ndrops` drops with degrees drawn from `p_choices` (an equal number of
    each when `balanced`), random shape perturbations amp*n^-2, centres by
    random sequential addition in [0, side]^3 with surface clearance >= gap
    (clearance measured with a rigorous bound on each drop's radius)."""
    rng = np.random.default_rng(seed)
    p_choices = list(p_choices)
    if balanced:
        reps = -(-ndrops // len(p_choices))
        ps = np.array((p_choices * reps)[:ndrops], np.int32)
        rng.shuffle(ps)
    else:
        ps = rng.choice(np.array(p_choices, np.int32), size=ndrops)
    blocks = []
    bounds = np.zeros(ndrops)
    for d in range(ndrops):
        blk, bounds[d] = _drop_shape(rng, int(ps[d]), (0.0, 0.0, 0.0), 1.0, 0.0, amp)
        blocks.append(blk)
    centres = _rsa(rng, bounds, side, gap)
    for d in range(ndrops):
        p = int(ps[d])
        for c in range(3):
            blocks[d][c * 2 * ncoef(p)] += math.sqrt(4.0 * math.pi) * centres[d, c]
    x = np.concatenate(blocks)
    f = _densities(rng, ps, 3)
    s = _densities(rng, ps, 1)
    return Suspension(name, ps, ps * upsample, ps * upsample, grid_mode, x, f, s, None,
                      centres, bounds)


def batched_suspension(seed: int = 3, grid_mode: int = 0, ndrops: int = 64) -> Suspension:
    """64 drops, p in {16,24,32,48} (16 of each, shuffled), cube side 12."""
    return suspension(ndrops, [16, 24, 32, 48], 12.0, seed, grid_mode, name="batched_64_mixed_p")


def large_suspension(seed: int = 5, grid_mode: int = 0, ndrops: int = 256) -> Suspension:
    """256 drops at p=32, volume fraction 0.1: side (256 * 4pi/3 / 0.1)^(1/3)."""
    side = (ndrops * 4.0 * math.pi / 3.0 / 0.1) ** (1.0 / 3.0)
    return suspension(ndrops, [32], side, seed, grid_mode, name="large_256_p32")


def with_separate_u(s: Suspension, seed: int = 99) -> Suspension:
    """Copy of `s` with an independent double-layer density u."""
    rng = np.random.default_rng(seed)
    u = _densities(rng, s.p, 3)
    return Suspension(s.name + "_u", s.p, s.q_self, s.q_far, s.grid_mode, s.xcoef, s.fcoef,
                      s.sigcoef, u, s.centres, s.radius_bound)


def subset(s: Suspension, drops) -> Suspension:
    """A suspension made of some of `s`'s drops (same coefficients)."""
    drops = list(drops)
    off = drop_offsets(s.p.astype(np.int64))

    def take(arr, K):
        if arr is None:
            return None
        return np.concatenate([arr[K * off[d]:K * off[d + 1]] for d in drops])

    return Suspension(s.name + "_sub", s.p[drops].copy(), s.q_self[drops].copy(),
                      s.q_far[drops].copy(), s.grid_mode, take(s.xcoef, 3), take(s.fcoef, 3),
                      take(s.sigcoef, 1), take(s.ucoef, 3), s.centres[drops].copy(),
                      s.radius_bound[drops].copy())


WORKLOADS = {
    "single_drop_p16": lambda gm=0: single_drop(16, 1, gm),
    "two_drops_p32": lambda gm=0: two_drops(32, 2, gm),
    "batched_64_mixed_p": lambda gm=0: batched_suspension(3, gm),
    "large_256_p32": lambda gm=0: large_suspension(5, gm),
}
