"""Pins of the oracle's refluxing (Sec. 4, Eq. fluxcorr / addreflux).

With every level advanced by the same dt (no subcycling), replacing each
coarse flux on a coarse-fine face by the sum of the fine fluxes makes the
composite state -- coarse cells not covered by the next level plus the
finest cells -- exactly conservative on the periodic domain."""
import numpy as np

import oracle as O
from oracle import amr_reflux
from paper_1110_0740_amd import inputs as I

NG = 4


def composite_totals(h, U):
    tot = np.zeros(9)
    for lev, L in enumerate(h.levels):
        V = h.dx(lev)[0] ** 3
        cov = amr_reflux.covered_map(h.levels[lev + 1], h.base << lev) if lev + 1 < len(h.levels) else None
        for B, u in zip(L, U[lev]):
            inner = I.interior(u, NG, 3)
            if cov is not None:
                mask = ~cov[B.lo[2]:B.lo[2] + B.n[2], B.lo[1]:B.lo[1] + B.n[1], B.lo[0]:B.lo[0] + B.n[0]]
            else:
                mask = np.ones(inner.shape[1:], dtype=bool)
            tot += (inner * mask[None]).reshape(9, -1).sum(axis=1) * V
    return tot


def test_reflux_makes_composite_state_conservative():
    h = I.amr_hierarchy(seed=3002, base=16, base_box=8, lattice=8, size_range=(4, 8), p1=(0.6, 1.0), p2=(0.6, 1.0))
    assert len(h.levels[1]) > 0 and len(h.levels[2]) > 0
    dt, ch = 1e-3, 2.0
    U0, U1, F1 = [], [], []
    for lev, L in enumerate(h.levels):
        oo = O.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=5.0 / 3.0, dx=h.dx(lev))
        Us = [O.prim2cons(oo, I.amr_fields(h, B, NG)) for B in L]
        res = [O.step(oo, U, NG, dt, ch, want_faces=True) for U in Us]
        U0.append(Us)
        U1.append([r[0] for r in res])
        F1.append([r[4] for r in res])
    before = composite_totals(h, U0)
    unfixed = composite_totals(h, U1)
    fixed = list(U1)
    for lev in range(len(h.levels) - 1):
        fixed[lev] = amr_reflux.reflux(h.levels[lev], U1[lev], F1[lev], h.dx(lev)[0], h.levels[lev + 1], F1[lev + 1],
                                       h.dx(lev + 1)[0], h.base << lev, NG)
    after = composite_totals(h, fixed)
    scale = np.abs(before[:8]) + 1e-3
    # without refluxing the coarse-fine flux mismatch shows up in the totals
    assert np.max(np.abs(unfixed[:8] - before[:8]) / scale) > 1e-9
    assert np.max(np.abs(after[:8] - before[:8]) / scale) < 1e-13
