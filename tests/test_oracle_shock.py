"""Pins of the oracle's shock-adaptive hybrid integration (App. B): where
the flags fall, that flagging everything equals the plain scheme with HLL
and MinMod reconstruction, that smooth flows are untouched, and that the
hybrid only changes the neighbourhood of the flags."""
import numpy as np

import oracle as O

NG = 4


def tube(nx, ny, i0, left, right, gamma=5.0 / 3.0):
    """2D box (ghosted), primitive state `left` in columns < i0, `right` from
    i0 on (ghosted column indices); left/right = (rho, p, vx)"""
    NX, NY = nx + 2 * NG, ny + 2 * NG
    V = np.zeros((9, 1, NY, NX))
    for c, (rho, p, vx) in ((slice(0, i0), left), (slice(i0, NX), right)):
        V[0, :, :, c] = rho
        V[4, :, :, c] = p
        V[1, :, :, c] = vx
    V[5] = 0.3  # a uniform B_x keeps the field in play without jumps
    o = O.make_opts(dim=2, gamma=gamma, dx=(1.0 / nx, 1.0 / nx, 1.0))
    return O.prim2cons(o, V)


def opts(**kw):
    base = dict(dim=2, recon="ppm", riemann="hlld", dx=(1.0 / 16, 1.0 / 16, 1.0))
    base.update(kw)
    return O.make_opts(**base)


def test_flags_sit_on_the_compressive_jump():
    nx, ny, i0 = 16, 4, 12
    U = tube(nx, ny, i0, (3.0, 10.0, 1.0), (1.0, 1.0, 0.0))
    f = O.shock_flags(opts(shock_eps=5.0), U, NG)[0]
    NY, NX = f.shape
    hll = (f & 1).astype(bool)
    mm = (f & 2).astype(bool)
    # |p_{+1} - p_{-1}| / min = 9 > 5 with div v < 0 only across the jump:
    # columns i0-1 and i0, on rows that have both y neighbours
    want_hll = np.zeros_like(hll)
    want_hll[1:NY - 1, i0 - 1:i0 + 1] = True
    assert np.array_equal(hll, want_hll)
    # MinMod within the PPM radius 2 along x (rows 1..NY-2) and along y
    want_mm = np.zeros_like(mm)
    want_mm[1:NY - 1, i0 - 3:i0 + 3] = True
    want_mm[:, i0 - 1:i0 + 1] = True
    assert np.array_equal(mm, want_mm)
    # radius 1 for a linear reconstruction
    f1 = O.shock_flags(opts(recon="lin_mc", shock_eps=5.0), U, NG)[0]
    want_mm1 = np.zeros_like(mm)
    want_mm1[1:NY - 1, i0 - 2:i0 + 2] = True
    want_mm1[:, i0 - 1:i0 + 1] = True
    assert np.array_equal((f1 & 2).astype(bool), want_mm1)


def test_no_flags_on_an_expansion_or_below_threshold():
    nx, ny, i0 = 16, 4, 12
    U = tube(nx, ny, i0, (3.0, 10.0, -1.0), (1.0, 1.0, 0.0))  # div v > 0
    assert not O.shock_flags(opts(shock_eps=5.0), U, NG).any()
    U = tube(nx, ny, i0, (3.0, 10.0, 1.0), (1.0, 1.0, 0.0))
    assert not O.shock_flags(opts(shock_eps=9.5), U, NG).any()  # 9 < 9.5


def test_flagging_every_zone_equals_hll_with_minmod():
    """p grows by 7x every two cells and v_x decreases linearly: every
    tested zone is flagged, so the hybrid PPM/HLLD step must equal the plain
    step with HLL fluxes and MinMod-limited linear reconstruction."""
    nx, ny = 8, 4
    NX, NY = nx + 2 * NG, ny + 2 * NG
    i = np.arange(NX)
    V = np.zeros((9, 1, NY, NX))
    V[0] = 1.0 + 0.1 * np.cos(i)[None, None, :]
    V[4] = 7.0 ** (0.5 * i)[None, None, :]
    V[1] = -0.5 * i[None, None, :]
    V[2] = 0.1
    V[5], V[6], V[7] = 0.3, 0.1, -0.2
    o_h = opts(shock_eps=5.0)
    U = O.prim2cons(o_h, V)
    f = O.shock_flags(o_h, U, NG)[0]
    assert np.all(f[1:-1, 1:-1] & 1)
    dt, ch = 1e-6, 1.0
    a = O.step(o_h, U, NG, dt, ch)[0]
    b = O.step(opts(riemann="hll", recon="lin_minmod"), U, NG, dt, ch)[0]
    c = O.step(opts(), U, NG, dt, ch)[0]
    inner = (slice(None), 0, slice(NG, NG + ny), slice(NG, NG + nx))
    assert np.array_equal(a[inner], b[inner])
    assert not np.array_equal(a[inner], c[inner])


def test_smooth_flow_is_untouched():
    rng = np.random.default_rng(2)
    nx, ny = 12, 10
    NX, NY = nx + 2 * NG, ny + 2 * NG
    y, x = np.meshgrid(np.arange(NY) / ny, np.arange(NX) / nx, indexing="ij")
    V = np.zeros((9, 1, NY, NX))
    V[0] = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    V[4] = 1.0 + 0.2 * np.cos(2 * np.pi * y)
    V[1] = 0.5 * np.sin(2 * np.pi * (x + y))
    V[2] = -0.3 * np.cos(2 * np.pi * x)
    V[5], V[6] = 0.4, 0.2
    o = opts(dx=(1.0 / nx, 1.0 / ny, 1.0))
    U = O.prim2cons(o, V)
    assert not O.shock_flags(opts(dx=(1.0 / nx, 1.0 / ny, 1.0), shock_eps=5.0), U, NG).any()
    a = O.step(opts(dx=(1.0 / nx, 1.0 / ny, 1.0), shock_eps=5.0), U, NG, 0.01, 1.0)[0]
    b = O.step(o, U, NG, 0.01, 1.0)[0]
    assert np.array_equal(a, b)


def test_hybrid_changes_only_the_neighbourhood_of_the_flags():
    nx, ny, i0 = 32, 4, 20
    U = tube(nx, ny, i0, (3.0, 10.0, 1.0), (1.0, 1.0, 0.0))
    o_on, o_off = opts(dx=(1 / 32, 1 / 32, 1.0), shock_eps=5.0), opts(dx=(1 / 32, 1 / 32, 1.0))
    dt, ch = 2e-4, 1.0
    a = O.step(o_on, U, NG, dt, ch)[0]
    b = O.step(o_off, U, NG, dt, ch)[0]
    d = np.abs(a - b).max(axis=(0, 1, 2))  # per ghosted column
    cols = np.nonzero(d)[0]
    assert cols.size > 0
    # flagged columns i0-1, i0; MinMod reaches i0-3..i0+2; their final
    # fluxes touch the cells i0-4..i0+3
    assert cols.min() >= i0 - 4 and cols.max() <= i0 + 3, cols
