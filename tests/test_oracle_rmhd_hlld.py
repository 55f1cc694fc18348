"""Pins of the oracle's HLLD solver for relativistic MHD (Sec. 3.1; Mignone,
Ugliano & Bodo 2009): consistency, exact upwinding of an isolated contact
and of an isolated rotational discontinuity, where the discontinuity is
built here by Newton iteration on the relativistic jump conditions
(physical fluxes only) along the Alfven branch; the B_n = 0 limit is HLLC;
and a conservative 3D step that differs from HLLC."""
import numpy as np
import pytest
from scipy.optimize import fsolve

import oracle as O
from paper_1110_0740_amd import inputs as I

G = 4.0 / 3.0


def _opts(eos="ideal", riemann="hlld", **kw):
    return O.make_opts(**dict(dict(physics="rmhd", predictor="mh", recon="lin_mc", riemann=riemann, gamma=G, eos=eos,
                                   glm=False), **kw))


def _phys(o, V, d):
    F = O.flux(o, V, d, 1.0)
    F[5 + d] = 0.0
    F[8] = 0.0
    return F


def _state(rng, vmax=0.9):
    V = np.zeros(9)
    V[0] = rng.uniform(0.2, 3.0)
    V[4] = rng.uniform(0.05, 3.0)
    v = rng.normal(size=3)
    V[1:4] = v / np.linalg.norm(v) * rng.uniform(0.0, vmax)
    V[5:8] = rng.normal(0, 1.0, 3)
    return V


@pytest.mark.parametrize("eos", ["ideal", "tm"])
def test_rmhd_hlld_consistency(eos):
    rng = np.random.default_rng(91)
    o = _opts(eos)
    for trial in range(60):
        d = trial % 3
        V = _state(rng, 0.95)
        F, _ = O.riemann(o, V, V, d, 1.0)
        Fp = _phys(o, V, d)
        assert np.max(np.abs(F - Fp)) <= 1e-13 * (1 + np.max(np.abs(Fp))), trial


@pytest.mark.parametrize("eos", ["ideal", "tm"])
def test_rmhd_hlld_resolves_an_isolated_contact(eos):
    rng = np.random.default_rng(92)
    o = _opts(eos)
    for trial in range(60):
        d = trial % 3
        V = _state(rng)
        VL, VR = V.copy(), V.copy()
        VR[0] = V[0] * rng.uniform(1.5, 5.0)
        F, _ = O.riemann(o, VL, VR, d, 1.0)
        Fu = _phys(o, VL if V[1 + d] >= 0 else VR, d)
        assert np.max(np.abs(F - Fu)) <= 1e-13 * (1 + np.max(np.abs(Fu))), trial


def _rotational_discontinuity(o, VL, dBy, lam0):
    """V_R and the speed of the discontinuity from V_L whose B_y jumps by dBy:
    the seven jump conditions lam (U_R - U_L) = F_R - F_L (D, m, E, B_t) are
    solved for (rho, v, p, B_z, lam) of the right state by Newton steps from
    V_L and an Alfven-speed guess, dBy being reached in ten increments."""
    UL = O.prim2cons(o, VL[:, None])[:, 0]
    FL = _phys(o, VL, 0)

    def eqs(x, By):
        rho, vx, vy, vz, p, Bz, lam = x
        if rho <= 0 or p <= 0 or vx * vx + vy * vy + vz * vz >= 1:
            return np.full(7, 1e3)
        VR = np.array([rho, vx, vy, vz, p, VL[5], By, Bz, 0.0])
        r = lam * (O.prim2cons(o, VR[:, None])[:, 0] - UL) - (_phys(o, VR, 0) - FL)
        return r[[0, 1, 2, 3, 4, 6, 7]]

    x = np.array([VL[0], VL[1], VL[2], VL[3], VL[4], VL[7], lam0])
    for s in np.linspace(0.1, 1.0, 10):
        x = fsolve(eqs, x, args=(VL[6] + s * dBy,), xtol=1e-14)
    rho, vx, vy, vz, p, Bz, lam = x
    VR = np.array([rho, vx, vy, vz, p, VL[5], VL[6] + dBy, Bz, 0.0])
    return VR, lam, np.max(np.abs(eqs(x, VL[6] + dBy)))


def _alfven_guesses(V):
    """Lab-frame Alfven speeds (b_x +- sqrt(w_t) g v_x)/(b^0 +- sqrt(w_t) g)."""
    v, B = V[1:4], V[5:8]
    g = 1.0 / np.sqrt(1.0 - v @ v)
    b0 = g * (v @ B)
    bx = B[0] / g + b0 * v[0]
    wt = V[0] + G / (G - 1) * V[4] + B @ B / g ** 2 + (v @ B) ** 2
    s = np.sqrt(wt)
    return [(bx + sg * s * g * v[0]) / (b0 + sg * s * g) for sg in (1.0, -1.0)]


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_rmhd_hlld_resolves_a_rotational_discontinuity():
    """On the Alfven branch rho, p (and w_t) do not jump; HLLD returns the
    upwind physical flux exactly there, HLLC does not."""
    rng = np.random.default_rng(93)
    o, oc = _opts(), _opts(riemann="hllc")
    found = 0
    for trial in range(24):
        VL = _state(rng, 0.6)
        VL[0] = rng.uniform(0.5, 2.0)
        VL[4] = rng.uniform(0.2, 2.0)
        VL[5] = np.sign(VL[5]) * max(abs(VL[5]), 0.5)
        lam0 = _alfven_guesses(VL)[trial % 2]
        VR, lam, res = _rotational_discontinuity(o, VL, 0.4 * rng.choice([-1.0, 1.0]), lam0)
        if not (res < 1e-12 and abs(VR[0] - VL[0]) < 1e-10 * VL[0] and abs(VR[4] - VL[4]) < 1e-10 * VL[4]):
            continue  # Newton left the Alfven branch
        found += 1
        F, _ = O.riemann(o, VL, VR, 0, 1.0)
        Fu = _phys(o, VL if lam >= 0 else VR, 0)
        assert np.max(np.abs(F - Fu)) <= 1e-11 * (1 + np.max(np.abs(Fu))), trial
        Fc, _ = O.riemann(oc, VL, VR, 0, 1.0)
        assert np.max(np.abs(Fc - Fu)) > 1e-6
    assert found >= 8


def test_rmhd_hlld_without_normal_field_is_hllc():
    rng = np.random.default_rng(94)
    o, oc = _opts(), _opts(riemann="hllc")
    for trial in range(30):
        d = trial % 3
        VL, VR = _state(rng), _state(rng)
        VL[5 + d] = VR[5 + d] = 0.0
        F, _ = O.riemann(o, VL, VR, d, 1.0)
        Fc, _ = O.riemann(oc, VL, VR, d, 1.0)
        assert np.array_equal(F, Fc)


@pytest.mark.parametrize("eos", ["ideal", "tm"])
def test_rmhd_hlld_step_conserves(eos):
    V, meta = I.rmhd3d_fields(n=12, ng=4, seed=4001, gmax_cap=3.0)
    kw = dict(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", gamma=G, eos=eos, dx=meta["dx"])
    o = O.make_opts(riemann="hlld", **kw)
    U = O.prim2cons(o, V)
    rate = O.cfl_rate(o, U, 4)
    dt = 0.3 / rate
    ch = min(0.3 * meta["dx"][0] / dt, 1.0)
    Uo, r, _, fails = O.step(o, U, 4, dt, ch)
    assert fails == [0] * 5 and r > 0
    a = I.interior(U, 4, 3).reshape(9, -1)
    b = I.interior(Uo, 4, 3).reshape(9, -1)
    for q in range(8):
        assert abs(b[q].sum() - a[q].sum()) <= 50 * a.shape[1] * 2.2e-16 * np.abs(a[q]).max()
    Uc, _, _, _ = O.step(O.make_opts(riemann="hllc", **kw), U, 4, dt, ch)
    assert np.max(np.abs(I.interior(Uc, 4, 3) - I.interior(Uo, 4, 3))) > 1e-8
