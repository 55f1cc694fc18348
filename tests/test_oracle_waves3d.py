"""Second-order convergence of the oracle's 3D CTU step on oblique linear
MHD eigenmodes (Sec. 3.1 unsplit step with Eq. transv in three dimensions,
Sec. 3.2 characteristic predictors).

The wave vector is k = 2 pi (1, 1, 1) or 2 pi (1, 2, -1), so every face
direction carries the wave and every transverse increment is nonzero.  The
eigenvector comes from numpy's eigen-solver on the primitive matrix written
from Eq. mhd in the (n, t, b) frame of k, rotated back to the grid; the
initial state holds the exact cell averages of the mode (sinc factors); after
one period the L1 error must fall by about 4 per doubling of the grid."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.test_oracle_pins import G53, prim_matrix


def wave3d_error(N, wave, recon, kint, eps=1e-6, ng=4):
    k = np.asarray(kint, float)
    kn = np.linalg.norm(k)
    nv = k / kn
    a = np.array([0.0, 0.0, 1.0]) if abs(nv[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    tv = a - (a @ nv) * nv
    tv /= np.linalg.norm(tv)
    bv = np.cross(nv, tv)
    vn0 = 1.0 if wave == "entropy" else 0.0
    rho, p, Bn, Bt, Bb = 1.0, 1.0 / G53, 1.0, math.sqrt(2.0), 0.5
    Vw = np.array([rho, vn0, 0, 0, p, Bn, Bt, Bb, 0.0])
    lam, R = np.linalg.eig(prim_matrix(Vw, 0, G53))
    lam, R = lam.real, R.real
    order = np.argsort(lam)
    lam, R = lam[order], R[:, order]
    j = {"fast": 6, "alfven": 5, "slow": 4, "entropy": 3}[wave]
    r, c = R[:, j], lam[j]
    dx = 1.0 / N
    X, Y, Z = I.cell_centres(I.Box((0, 0, 0), (N, N, N)), ng, (dx, dx, dx), 3)
    cav = np.cos(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z))
    for q in range(3):
        cav = cav * np.sinc(k[q] * dx)
    dq = eps * r[:, None, None, None] * cav[None]
    vn, vt, vb = vn0 + dq[1], dq[2], dq[3]
    bt, bb = Bt + dq[4], Bb + dq[5]
    V = np.zeros((9,) + X.shape)
    V[0] = rho + dq[0]
    V[4] = p + dq[6]
    for q in range(3):
        V[1 + q] = vn * nv[q] + vt * tv[q] + vb * bv[q]
        V[5 + q] = Bn * nv[q] + bt * tv[q] + bb * bv[q]
    o = O.make_opts(dim=3, recon=recon, riemann="hlld", gamma=G53, dx=(dx, dx, dx))
    U0 = O.prim2cons(o, V)
    U = U0.copy()
    T = (1.0 / kn) / abs(c)
    t = 0.0
    while t < T - 1e-14:
        dt0 = 0.4 / O.cfl_rate(o, U, ng)
        dt = min(dt0, T - t)
        U, _, _, fails = O.step(o, U, ng, dt, 0.4 * dx / dt0)
        assert fails == [0] * 5
        I.fill_periodic(U, ng, 3)
        t += dt
    return np.abs(I.interior(U, ng, 3) - I.interior(U0, ng, 3))[:8].sum(axis=0).mean() / eps


@pytest.mark.parametrize("wave,recon,kint", [("fast", "ppm", (1, 1, 1)), ("alfven", "ppm", (1, 2, -1)),
                                             ("slow", "lin_mc", (1, 1, 1)), ("entropy", "weno3", (1, 1, 1))])
def test_linear_wave_3d_second_order(wave, recon, kint):
    e = [wave3d_error(N, wave, recon, kint) for N in (16, 32)]
    order = math.log2(e[0] / e[1])
    assert order > 1.6, e


def test_planted_2d_corner_coupling_fails_in_3d():
    """Corner coupling that adds only one of the two transverse increments
    (a 2D habit carried into 3D) must fail the 3D pin."""
    from tests.plant import planted
    with planted("                            if (e != d) tr += Ln[(e * NVAR + q) * NC + c];",
                 "                            if (e == (d + 1) % 3) tr += Ln[(e * NVAR + q) * NC + c];"):
        try:
            e = [wave3d_error(N, "fast", "ppm", (1, 1, 1)) for N in (16, 32)]
            ok = math.log2(e[0] / e[1]) > 1.6
        except AssertionError:
            ok = False
    assert not ok
