"""Pins of the two corner couplings of the oracle (Sec. 3.1): Eq. transv with
first-order t^n transverse fluxes (the default), and MT's form for runs
without parabolic terms, whose transverse fluxes are Riemann fluxes between
normal-predictor states.

A density pattern carried by a uniform flow through a uniform field (an
entropy wave: v, p and B stay uniform, HLLD resolves every face exactly)
reduces the whole MHD step to scalar corner-transport-upwind advection of
rho, which is written out here from its definition: MC-limited slopes,
upwind tracing to the half step, transverse upwind fluxes from the cell
values (t^n form) or from the traced face values (MT form), corner-coupled
face states, upwind final fluxes.  Both couplings must match it to
rounding in 2D and 3D for flows of either sign; with slopes that vanish
(zig-zag data, MinMod) both collapse onto the first-order donor-cell CTU
update.  Further: conservation and free streaming of an MT step."""
import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I

G53 = 5.0 / 3.0


def _mc(dp, dm):
    mm = lambda a, b: 0.5 * (np.sign(a) + np.sign(b)) * np.minimum(np.abs(a), np.abs(b))
    return mm(0.5 * (dp + dm), 2.0 * mm(dm, dp))


def _minmod(dp, dm):
    return 0.5 * (np.sign(dp) + np.sign(dm)) * np.minimum(np.abs(dp), np.abs(dm))


def scalar_ctu(rho, v, dt, dx, mode, limiter=_mc):
    """One corner-transport-upwind step of rho_t + v . grad rho = 0 on a
    periodic grid (axis a of the array is direction a)."""
    dim = rho.ndim
    nu = [v[d] * dt / dx[d] for d in range(dim)]
    rp, rm, L = [], [], []
    for d in range(dim):
        dp = np.roll(rho, -1, d) - rho
        dm = rho - np.roll(rho, 1, d)
        s = limiter(dp, dm)
        if nu[d] > 0:
            rp.append(rho + 0.5 * (1 - nu[d]) * s)
            rm.append(rho - 0.5 * s)
        else:
            rp.append(rho + 0.5 * s)
            rm.append(rho - 0.5 * (1 + nu[d]) * s)
        # transverse flux on the face below each cell
        if mode == "mt":
            up = np.roll(rp[d], 1, d) if v[d] > 0 else rm[d]
        else:
            up = np.roll(rho, 1, d) if v[d] > 0 else rho
        f = v[d] * up
        L.append(-(np.roll(f, -1, d) - f) / dx[d])
    out = rho.copy()
    for d in range(dim):
        tr = sum(L[e] for e in range(dim) if e != d)
        cp = rp[d] + 0.5 * dt * tr
        cm = rm[d] + 0.5 * dt * tr
        up = np.roll(cp, 1, d) if v[d] > 0 else cm
        f = v[d] * up
        out -= dt * (np.roll(f, -1, d) - f) / dx[d]
    return out


def _mhd_advect(rho, v, dt, dx, corner, recon="lin_mc"):
    """The oracle's MHD step on the entropy wave; rho has array axes
    (x, y[, z]); returns the new interior density in the same axes."""
    dim = rho.ndim
    ng = 4
    n = rho.shape
    shape = tuple(reversed([m + 2 * ng for m in n])) if dim == 3 else (1, n[1] + 2 * ng, n[0] + 2 * ng)
    V = np.zeros((9,) + shape)
    inner = np.transpose(rho) if dim == 3 else np.transpose(rho)[None]
    if dim == 3:
        V[0, ng:-ng, ng:-ng, ng:-ng] = inner
    else:
        V[0, :, ng:-ng, ng:-ng] = inner
    V[1], V[2] = v[0], v[1]
    V[3] = v[2] if dim == 3 else 0.3
    V[4] = 0.8
    V[5], V[6], V[7] = 0.6, -0.4, 0.5
    o = O.make_opts(dim=dim, recon=recon, riemann="hlld", gamma=G53, dx=tuple(dx) + (1.0,) * (3 - dim),
                    corner=corner)
    U = O.prim2cons(o, V)
    I.fill_periodic(U, ng, dim)
    Uo, _, _, fails = O.step(o, U, ng, dt, 1.0)
    assert fails == [0] * 5
    Vo, _ = O.cons2prim(o, Uo)
    r = Vo[0, ng:-ng, ng:-ng, ng:-ng] if dim == 3 else Vo[0, 0, ng:-ng, ng:-ng]
    # velocity and pressure stay uniform
    inn = (slice(None),) + ((slice(ng, -ng),) * 3 if dim == 3 else (0, slice(ng, -ng), slice(ng, -ng)))
    assert np.max(np.abs(Vo[4][inn[1:]] - 0.8)) < 1e-12
    return np.transpose(r)


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(m) / m for m in shape], indexing="ij")
    f = np.ones(shape)
    for _ in range(3):
        k = rng.integers(1, 3, len(shape))
        ph = rng.uniform(0, 2 * np.pi, len(shape))
        term = 0.15
        for a in range(len(shape)):
            term = term * np.cos(2 * np.pi * k[a] * grids[a] + ph[a])
        f = f + term
    return f


@pytest.mark.parametrize("corner", ["tn", "mt"])
@pytest.mark.parametrize("v", [(0.7, 0.4), (-0.5, 0.8), (0.6, -0.9)])
def test_entropy_wave_is_scalar_ctu_2d(corner, v):
    n = (24, 20)
    dx = (1.0 / 24, 1.0 / 20)
    rho = _field(n, 81)
    dt = 0.4 * min(dx[0] / abs(v[0]), dx[1] / abs(v[1]))
    got = _mhd_advect(rho, v, dt, dx, corner)
    ref = scalar_ctu(rho, v, dt, dx, corner)
    assert np.max(np.abs(got - ref)) < 1e-13
    other = scalar_ctu(rho, v, dt, dx, "tn" if corner == "mt" else "mt")
    assert np.max(np.abs(got - other)) > 1e-6  # the two couplings really differ


@pytest.mark.parametrize("corner", ["tn", "mt"])
def test_entropy_wave_is_scalar_ctu_3d(corner):
    n = (12, 10, 8)
    dx = (1.0 / 12, 1.0 / 10, 1.0 / 8)
    v = (0.5, -0.4, 0.3)
    rho = _field(n, 82)
    dt = 0.3 * min(dx[d] / abs(v[d]) for d in range(3))
    got = _mhd_advect(rho, v, dt, dx, corner)
    ref = scalar_ctu(rho, v, dt, dx, corner)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("corner", ["tn", "mt"])
def test_zero_slopes_give_donor_cell_ctu(corner):
    """Zig-zag data along both axes: every MinMod slope vanishes, traced
    states equal cell values, and one step is the donor-cell CTU update
    (1-nx)(1-ny) r_ij + nx (1-ny) r_i-1,j + (1-nx) ny r_i,j-1 + nx ny r_i-1,j-1."""
    n = (16, 16)
    dx = (1.0 / 16, 1.0 / 16)
    i, j = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    rho = 1.0 + 0.2 * (-1.0) ** i + 0.1 * (-1.0) ** j + 0.05 * (-1.0) ** (i + j)
    v = (0.6, 0.35)
    dt = 0.5 * dx[0] / v[0]
    nx, ny = v[0] * dt / dx[0], v[1] * dt / dx[1]
    got = _mhd_advect(rho, v, dt, dx, corner, recon="lin_minmod")
    sh = lambda a, di, dj: np.roll(np.roll(a, di, 0), dj, 1)
    ref = ((1 - nx) * (1 - ny) * rho + nx * (1 - ny) * sh(rho, 1, 0) + (1 - nx) * ny * sh(rho, 0, 1)
           + nx * ny * sh(rho, 1, 1))
    assert np.max(np.abs(got - ref)) < 1e-13


def test_mt_step_conserves_and_preserves_free_stream():
    V, meta = I.mhd3d_fields(n=12, ng=4, seed=2003)
    o = O.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=G53, dx=meta["dx"], corner="mt")
    U = O.prim2cons(o, V)
    rate = O.cfl_rate(o, U, 4)
    dt = 0.4 / rate
    ch = 0.4 * o.dx[0] / dt
    Uo, r, _, fails = O.step(o, U, 4, dt, ch)
    assert fails == [0] * 5 and r > 0
    a = I.interior(U, 4, 3).reshape(9, -1)
    b = I.interior(Uo, 4, 3).reshape(9, -1)
    for q in range(8):
        assert abs(b[q].sum() - a[q].sum()) <= 50 * a.shape[1] * 2.2e-16 * np.abs(a[q]).max()
    Vu = np.zeros((9, 16, 16, 16))
    Vu[:] = np.array([1.2, 0.3, -0.2, 0.4, 0.9, 0.5, -0.3, 0.2, 0.0])[:, None, None, None]
    Uu = O.prim2cons(o, Vu)
    Uuo, _, _, _ = O.step(o, Uu, 4, 0.01, 1.0)
    assert np.max(np.abs(I.interior(Uuo, 4, 3)[:8] - I.interior(Uu, 4, 3)[:8])) < 1e-13


def test_mt_rejects_parabolic_terms():
    o = O.make_opts(dim=2, recon="lin_mc", corner="mt", parabolic_mask=1, nu=0.01)
    V, meta = I.mhd2d_fields(n=16, ng=4, seed=1000)
    U = O.prim2cons(o, V)
    with pytest.raises(Exception):
        O.step(o, U, 4, 1e-3, 1.0)
