"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, validates host-only arguments, and its host-built rotation
tables follow the defining relation of the rotation to the pole."""
import math
import os
import re

import numpy as np
import pytest
from scipy.special import sph_harm_y

from paper_1811_10270_amd import ehdbim as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(E.LIB_PATH):
        from paper_1811_10270_amd import build
        build.build()
    return E.load()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ehdbim.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ehd_[A-Za-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(E.EXPORTED) == syms


def test_grid_dims(lib):
    assert E.grid_dims(16, E.GRID_PAPER) == (17, 34)
    assert E.grid_dims(16, E.GRID_2P) == (17, 32)
    assert E.grid_dims(32, E.GRID_2P) == (33, 64)
    import ctypes as C
    a, b = C.c_int(), C.c_int()
    assert lib.ehd_grid_dims(0, 0, C.byref(a), C.byref(b)) == E.EHD_E_ARG
    assert lib.ehd_grid_dims(4, 7, C.byref(a), C.byref(b)) == E.EHD_E_ARG


def _rot_y(beta, v):
    c, s = math.cos(beta), math.sin(beta)
    return np.array([c * v[0] + s * v[2], v[1], -s * v[0] + c * v[2]])


def _angles(v):
    return math.acos(max(-1.0, min(1.0, v[2]))), math.atan2(v[1], v[0])


@pytest.mark.parametrize("n,beta", [(1, 0.4), (2, 1.3), (5, 2.2), (9, 0.05), (12, 3.0)])
def test_wigner_d_defining_relation(lib, n, beta):
    """Y_nm(Ry(beta) v) = sum_m' d^n_{m m'}(beta) Y_nm'(v), against scipy."""
    d = E.wigner_d(n, beta)
    rng = np.random.default_rng(n)
    for _ in range(4):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        th, ph = _angles(v)
        thr, phr = _angles(_rot_y(beta, v))
        for m in range(-n, n + 1):
            lhs = sph_harm_y(n, m, thr, phr)
            rhs = sum(d[m + n, mp + n] * sph_harm_y(n, mp, th, ph) for mp in range(-n, n + 1))
            assert abs(lhs - rhs) < 1e-12


@pytest.mark.parametrize("n", [16, 32, 48, 64])
def test_wigner_d_orthogonal_at_high_degree(lib, n):
    for beta in (0.03, 1.1, 2.9, math.pi - 0.02):
        d = E.wigner_d(n, beta)
        err = np.abs(d @ d.T - np.eye(2 * n + 1)).max()
        assert err < 1e-12, (n, beta, err)


def test_self_prefetch_candidates(lib):
    """Three Legendre prefetch batches per degree class, the default first,
    distinct; bad classes are refused (host only)."""
    for cls in range(4):
        c = E.self_config_candidates(cls)
        assert len(c) == 3 and len(set(c)) == 3 and all(1 <= v <= 8 for v in c)
    assert E.self_config_candidates(2)[0] == 3 and E.self_config_candidates(3)[0] == 5
    import ctypes
    pf, n = (ctypes.c_int * 3)(), ctypes.c_int()
    assert lib.ehd_self_config_candidates(4, pf, ctypes.byref(n)) == E.EHD_E_ARG
    assert lib.ehd_self_config_candidates(-1, pf, ctypes.byref(n)) == E.EHD_E_ARG


def test_rows_for_kinds():
    assert E.rows_for_kinds(E.ALL_KINDS) == list(range(9))
    assert E.rows_for_kinds(E.METRIC_KINDS) == list(range(8))
    assert E.rows_for_kinds(E.LAP_DL | E.STOKES_DL) == [3, 4, 5, 7]
