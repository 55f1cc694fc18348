"""Pins of the oracle's Rusanov (local Lax-Friedrichs) solver, one of the
solvers that Sec. 3.1 lists as common to the classical and relativistic
modules: it must equal the separately written HLL flux whenever the HLL
bounds are symmetric (zero normal velocity on both sides), converge to the
exact Euler solution of the Sod tube while diffusing more than HLLD, and
keep the CTU step conservative."""
import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.exact_riemann import sample as euler_exact
from tests.test_oracle_pins import G53, _run_tube, random_mhd_states


@pytest.mark.parametrize("physics", ["mhd", "rmhd"])
def test_rusanov_equals_hll_for_symmetric_bounds(physics):
    """With v_n = 0 in both states the HLL bounds are -a and +a, and the HLL
    flux (S_R F_L - S_L F_R + S_L S_R dU)/(S_R - S_L) is then the Rusanov
    flux; a wrong dissipation coefficient or sign breaks the equality."""
    rng = np.random.default_rng(41)
    G = G53 if physics == "mhd" else 4.0 / 3.0
    kw = dict(physics=physics, gamma=G, predictor="char" if physics == "mhd" else "mh", recon="lin_mc")
    orus = O.make_opts(riemann="rusanov", **kw)
    ohll = O.make_opts(riemann="hll", **kw)
    for trial in range(40):
        VL, VR = random_mhd_states(rng, 2).T
        d = trial % 3
        for V in (VL, VR):
            V[1 + d] = 0.0
            if physics == "rmhd":
                V[1:4] *= 0.9 / max(1.0, np.linalg.norm(V[1:4]))
        Fr, ar = O.riemann(orus, VL, VR, d, 1.3)
        Fh, ah = O.riemann(ohll, VL, VR, d, 1.3)
        assert ar == ah
        assert np.max(np.abs(Fr - Fh)) <= 1e-13 * (1.0 + np.max(np.abs(Fh)))
        # and the dissipation is really there: states differ, so F differs
        # from the centred flux
        Fc = 0.5 * (O.flux(orus, VL, d, 1.3) + O.flux(orus, VR, d, 1.3))
        assert np.max(np.abs(Fr[:5] - Fc[:5])) > 1e-6


def test_rusanov_differs_from_hll_for_asymmetric_bounds():
    """A supersonic-ish normal flow makes the HLL bounds asymmetric: the two
    solvers then differ (Rusanov is not HLL in disguise)."""
    rng = np.random.default_rng(42)
    orus = O.make_opts(riemann="rusanov", gamma=G53, recon="lin_mc")
    ohll = O.make_opts(riemann="hll", gamma=G53, recon="lin_mc")
    VL, VR = random_mhd_states(rng, 2).T
    VL[1], VR[1] = 0.8, 0.6
    VR[0] *= 1.5
    Fr, _ = O.riemann(orus, VL, VR, 0, 1.0)
    Fh, _ = O.riemann(ohll, VL, VR, 0, 1.0)
    assert np.max(np.abs(Fr - Fh)) > 1e-3


def test_rusanov_sod_converges_and_diffuses_more_than_hlld():
    """B = 0: the Sod tube with Rusanov fluxes converges to the exact Euler
    solution at about first order in L1; at equal resolution its error is
    larger than with HLLD (the most diffusive of the solvers)."""
    g = 1.4
    VL = [1.0, 0, 0, 0, 1.0, 0, 0, 0, 0]
    VR = [0.125, 0, 0, 0, 0.1, 0, 0, 0, 0]
    errs = {}
    for solver in ("rusanov", "hlld"):
        o = O.make_opts(dim=2, recon="lin_mc", riemann=solver, gamma=g)
        e = []
        for N in (100, 200, 400):
            x, V = _run_tube(o, VL, VR, 0.0, 1.0, 0.5, N, 0.2, cfl=0.8)
            ex = euler_exact((x - 0.5) / 0.2, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g)
            e.append(np.mean(np.abs(V[0] - ex[0])))
        errs[solver] = e
    r = errs["rusanov"]
    assert r[2] < 0.01
    assert r[0] / r[1] > 1.4 and r[1] / r[2] > 1.4
    assert all(a > b for a, b in zip(errs["rusanov"], errs["hlld"]))


@pytest.mark.parametrize("physics", ["mhd", "rmhd"])
def test_rusanov_step_conserves(physics):
    if physics == "mhd":
        V, meta = I.mhd3d_fields(n=12, ng=4, seed=2003)
        o = O.make_opts(dim=3, recon="ppm", riemann="rusanov", gamma=G53, dx=meta["dx"])
        cfl = 0.4
    else:
        V, meta = I.rmhd3d_fields(n=12, ng=4, seed=4001, gmax_cap=3.0)
        o = O.make_opts(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", riemann="rusanov", gamma=4.0 / 3.0,
                        dx=meta["dx"])
        cfl = 0.3
    U = O.prim2cons(o, V)
    rate = O.cfl_rate(o, U, 4)
    dt = cfl / rate
    ch = min(cfl * o.dx[0] / dt, 1.0 if physics == "rmhd" else 1e30)
    Uo, r, _, fails = O.step(o, U, 4, dt, ch)
    assert fails == [0] * 5 and r > 0
    a = I.interior(U, 4, 3).reshape(9, -1)
    b = I.interior(Uo, 4, 3).reshape(9, -1)
    for q in range(8):
        assert abs(b[q].sum() - a[q].sum()) <= 50 * a.shape[1] * 2.2e-16 * np.abs(a[q]).max()
    # the step moved the state (the solver is live)
    assert np.max(np.abs(b - a)) > 1e-6
