"""Pins of the oracle's refinement criterion (Eq. RefCrit), leaf masks and
level time steps (Eq. Ca, Eq. dt_cool, Eq. level_dt)."""
import math

import numpy as np

import oracle as O
from oracle import amr_time as AT

NG = 2


def box(n, f):
    k, j, i = np.indices((n + 2 * NG,) * 3) - NG
    return f(k, j, i).astype(np.float64)


def test_chi_vanishes_on_linear_data():
    s = box(6, lambda k, j, i: 2.0 + 0.3 * i - 0.2 * j + 0.7 * k)
    assert np.max(AT.lohner_chi(s, NG)) < 1e-13


def test_chi_closed_forms_at_a_step():
    eps = 0.01
    h = 3.0
    # sigma = 0 for i <= 2, h for i >= 3 (constant along y, z)
    s = box(6, lambda k, j, i: np.where(i >= 3, h, 0.0) + 0.0 * (j + k))
    chi = AT.lohner_chi(s, NG, eps)
    # last low cell: D+ = h, D- = 0, sigma_ref,x = h, sigma_ref,y/z = 0
    assert abs(chi[0, 0, 2] - 1.0 / (1.0 + eps)) < 1e-14
    # first high cell: D+ = 0, D- = h, sigma_ref,x = 3h, sigma_ref,y/z = 4h
    want = 1.0 / math.sqrt((1.0 + 3.0 * eps) ** 2 + 2.0 * (4.0 * eps) ** 2)
    assert abs(chi[0, 0, 3] - want) < 1e-14
    # away from the step: no curvature
    assert np.all(chi[:, :, :2] == 0.0) and np.all(chi[:, :, 4:] == 0.0)


def test_chi_small_ripples_need_the_eps_term():
    """a 1e-3 ripple on a unit background: without eps it reads as a full
    extremum (chi = 1), with eps = 0.01 the sigma_ref term suppresses it"""
    s = box(6, lambda k, j, i: 1.0 + 1e-3 * (i % 2) + 0.0 * (j + k))
    assert np.allclose(AT.lohner_chi(s, NG, 0.0), 1.0 / math.sqrt(1.0), atol=1e-12)
    assert np.max(AT.lohner_chi(s, NG, 0.01)) < 0.06


def test_chi_is_zero_where_sigma_vanishes():
    s = box(4, lambda k, j, i: 0.0 * i)
    assert np.all(AT.lohner_chi(s, NG) == 0.0)


def test_level_dt_combines_cfl_cooling_and_subcycling():
    rate = [10.0, 25.0, 36.0]
    dt_prev = [0.04, 0.02, 0.01]
    # CFL only: dt_l = 0.4 / rate_l -> 2^l dt_l = 0.04, 0.032, 0.0444 -> dt0 = 0.032
    got = AT.next_dt(rate, None, dt_prev, 0.4, 0.02)
    assert np.allclose(got, [0.032, 0.016, 0.008], rtol=1e-15)
    # cooling on level 2: eps_c dt^n / dpp = 0.02 * 0.01 / 0.05 = 0.004 -> 2^2 x = 0.016
    got = AT.next_dt(rate, [0.0, 0.0, 0.05], dt_prev, 0.4, 0.02)
    assert np.allclose(got, [0.016, 0.008, 0.004], rtol=1e-15)


def test_leaf_only_dpp_ignores_masked_cells():
    """the cooling limiter of a step taken with a leaf mask is the maximum
    of |dp/p| over the unmasked cells: masking everything gives 0, masking
    nothing gives the plain value, and a mask keeps a value no larger"""
    rng = np.random.default_rng(4)
    n, ng = 6, 4
    o = O.make_opts(dim=3, recon="ppm", cooling=True, cool_beta=0.5, T_floor=0.01, dx=(1 / 6,) * 3)
    V = np.zeros((9, n + 2 * ng, n + 2 * ng, n + 2 * ng))
    V[0] = 1.0 + 0.1 * rng.random(V[0].shape)
    V[4] = 1.0 + 0.1 * rng.random(V[0].shape)
    U = O.prim2cons(o, V)
    L0 = 0.5 + rng.random(V[0].shape)
    full = O.step(o, U, ng, 1e-3, 1.0, L0=L0)[2]
    none = O.step(o, U, ng, 1e-3, 1.0, L0=L0, leaf=np.zeros(V[0].shape, dtype=np.uint8))[2]
    ones = O.step(o, U, ng, 1e-3, 1.0, L0=L0, leaf=np.ones(V[0].shape, dtype=np.uint8))[2]
    half = np.zeros(V[0].shape, dtype=np.uint8)
    half[:, :, : ng + 3] = 1
    part = O.step(o, U, ng, 1e-3, 1.0, L0=L0, leaf=half)[2]
    assert full > 0.0 and none == 0.0 and ones == full and 0.0 < part <= full


def test_leaf_masks_mark_uncovered_interior_cells():
    class B:
        def __init__(self, lo, n):
            self.lo, self.n = lo, n
    levels = [[B((0, 0, 0), (8, 8, 8))], [B((4, 4, 4), (4, 6, 8))]]
    m = AT.leaf_masks(levels, 8, 2)
    assert m[0][0].sum() == 8 ** 3 - 2 * 3 * 4 and m[1][0].sum() == 4 * 6 * 8
    assert m[0][0][2 + 3, 2 + 3, 2 + 3] == 0 and m[0][0][2 + 1, 2 + 1, 2 + 1] == 1
