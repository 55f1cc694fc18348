"""The oracle's cost structure and thread independence.

Riemann count (Sec. 3.1): the 3D CTU step with Eq. transv needs six Riemann
solves per zone, three for the t^n transverse fluxes and three at the half
step (four in 2D).  The instrumented oracle counts every solve of a step; on
boxes of n^3 interior zones the count is a cubic in n whose leading
coefficient is the per-zone count (the halo adds only lower powers), read
off exactly from the third finite difference (second in 2D).

Threads: the oracle's OpenMP loops must give bitwise the results of one
thread for every option family."""
import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I


def _count(o, n, dim, ng=4):
    shape = (9, 1, n + 2 * ng, n + 2 * ng) if dim == 2 else (9,) + (n + 2 * ng,) * 3
    V = np.zeros(shape)
    V[0], V[4], V[5], V[6], V[7] = 1.0, 0.6, 0.3, -0.2, 0.1
    V[1] = 0.1
    U = O.prim2cons(o, V)
    O.riemann_count(reset=True)
    O.step(o, U, ng, 1e-3, 1.0)
    return O.riemann_count(reset=True)


@pytest.mark.parametrize("dim,kw,per_zone", [
    (3, dict(recon="ppm", riemann="hlld"), 6),
    (3, dict(recon="lin_mc", riemann="hll", corner="mt"), 6),
    (3, dict(recon="ppm", riemann="hlld", shock_eps=5.0), 6),
    (2, dict(recon="lin_mc", riemann="hlld"), 4),
    (2, dict(recon="weno3", riemann="roe", corner="mt"), 4)])
def test_riemann_solves_per_zone(dim, kw, per_zone):
    o = O.make_opts(dim=dim, gamma=5.0 / 3.0, dx=(0.1, 0.1, 0.1), **kw)
    ns = [4, 5, 6, 7][: dim + 1]
    c = np.array([_count(o, n, dim) for n in ns], dtype=np.int64)
    lead = np.diff(c, n=dim)[0]  # dim! * leading coefficient
    assert lead == per_zone * (6 if dim == 3 else 2), (c, lead)


CASES = {
    "mhd_ppm_hlld": (dict(recon="ppm", riemann="hlld"), "mhd"),
    "mhd_mt_weno3_roe": (dict(recon="weno3", riemann="roe", corner="mt"), "mhd"),
    "mhd_hybrid": (dict(recon="ppm", riemann="hlld", shock_eps=0.05), "mhd"),
    "nonideal_cooling": (dict(recon="ppm", riemann="hlld", parabolic_mask=7, nu=1e-2, eta=5e-3, kappa_par=1e-2,
                              kappa_perp=1e-3, tc_phi=0.3, cooling=True), "mhd"),
    "rmhd_mh_hlld": (dict(physics="rmhd", predictor="mh", recon="lin_mc", riemann="hlld", gamma=4.0 / 3.0), "rmhd"),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_threads_give_bitwise_the_one_thread_result(case):
    kw, phys = CASES[case]
    kw = dict(kw)
    gamma = kw.pop("gamma", 5.0 / 3.0)
    if phys == "rmhd":
        V, meta = I.rmhd3d_fields(n=10, ng=4, seed=4003, gmax_cap=3.0)
    else:
        V, meta = I.mhd3d_fields(n=10, ng=4, seed=2003)
    o = O.make_opts(dim=3, gamma=gamma, dx=meta["dx"], **kw)
    U = O.prim2cons(o, V)
    L0 = np.full(U.shape[1:], 0.7) if kw.get("cooling") else None
    dt = 0.3 / O.cfl_rate(o, U, 4)
    out = {}
    try:
        for nt in (1, 3, 8):
            O.set_threads(nt)
            out[nt] = O.step(o, U, 4, dt, 0.3 * meta["dx"][0] / dt, L0=L0, want_faces=True)
    finally:
        O.set_threads(0)
    for nt in (3, 8):
        a, b = out[1], out[nt]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[4], b[4])
        assert a[1] == b[1] and a[2] == b[2] and a[3] == b[3]
