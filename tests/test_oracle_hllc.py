"""Pins of the oracle's HLLC solver for ideal MHD (one of the solvers that
Sec. 3.1 lists as common to the classical and relativistic modules; the
single-contact construction with HLL-averaged transverse field): it must
reduce to the hydrodynamic HLLC of Toro, Spruce & Speares when B = 0 (written
out here from the textbook star states, shear included), carry an isolated
entropy wave exactly (upwind flux, which HLL cannot), give the same flux on
both sides of a contact moving at zero speed, beat HLL on the Sod tube and
keep the CTU step conservative."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.exact_riemann import sample as euler_exact
from tests.test_oracle_pins import G53, _run_tube, random_mhd_states


def _opts(**kw):
    return O.make_opts(**dict(dict(physics="mhd", riemann="hllc", gamma=G53, recon="lin_mc"), **kw))


def _toro_hllc(VL, VR, d, g):
    """Hydrodynamic HLLC (Toro, Spruce & Speares 1994) in Toro's textbook
    form: outer speeds from the sound speeds, the contact speed from the
    pressure jump, star states
    U*_K = rho_K (S_K - u_K)/(S_K - S*) [1, S*, v_t, v_b,
            E_K/rho_K + (S* - u_K)(S* + p_K / (rho_K (S_K - u_K)))],
    and F*_K = F_K + S_K (U*_K - U_K)."""
    def cons(V):
        v2 = V[1] ** 2 + V[2] ** 2 + V[3] ** 2
        return np.array([V[0], V[0] * V[1], V[0] * V[2], V[0] * V[3], V[4] / (g - 1) + 0.5 * V[0] * v2])

    def flux(V, U):
        u = V[1 + d]
        F = U * u
        F[1 + d] += V[4]
        F[4] += V[4] * u
        return F

    UL, UR = cons(VL), cons(VR)
    FL, FR = flux(VL, UL), flux(VR, UR)
    uL, uR = VL[1 + d], VR[1 + d]
    cL, cR = math.sqrt(g * VL[4] / VL[0]), math.sqrt(g * VR[4] / VR[0])
    SL, SR = min(uL - cL, uR - cR), max(uL + cL, uR + cR)
    if SL >= 0:
        return FL
    if SR <= 0:
        return FR
    rL, rR, pL, pR = VL[0], VR[0], VL[4], VR[4]
    Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))
    V, U, F, S = (VL, UL, FL, SL) if Ss >= 0 else (VR, UR, FR, SR)
    u = V[1 + d]
    fac = V[0] * (S - u) / (S - Ss)
    Us = fac * np.array([1.0, V[1], V[2], V[3], U[4] / V[0] + (Ss - u) * (Ss + V[4] / (V[0] * (S - u)))])
    Us[1 + d] = fac * Ss
    return F + S * (Us - U)


def test_hllc_reduces_to_hydrodynamic_hllc_without_field():
    """B = 0, psi = 0: the MHD solver's density, momentum and energy fluxes
    are Toro's for the same states in every direction, including states with
    a shear jump (the transverse velocities of the two star states differ)."""
    rng = np.random.default_rng(51)
    g = 1.4
    o = _opts(gamma=g)
    for trial in range(60):
        VL, VR = np.zeros(9), np.zeros(9)
        for V in (VL, VR):
            V[0] = rng.uniform(0.1, 3.0)
            V[4] = rng.uniform(0.05, 3.0)
            V[1:4] = rng.normal(0, 1.2, 3)
        d = trial % 3
        F, smax = O.riemann(o, VL, VR, d, 1.0)
        Ft = _toro_hllc(VL, VR, d, g)
        assert np.max(np.abs(F[:5] - Ft)) <= 1e-13 * (1 + np.max(np.abs(Ft))), trial
        assert np.all(F[5:] == 0.0)


@pytest.mark.parametrize("u", [0.0, 0.37, -1.1])
def test_hllc_carries_an_entropy_wave_exactly(u):
    """Only the density jumps, velocity, pressure and the full (oblique) field
    are continuous: the exact flux is the upwind physical flux, which HLLC
    returns to rounding (also past the fast speed, where every solver
    upwinds); inside the fan HLL smears the jump and does not."""
    rng = np.random.default_rng(52)
    for trial in range(20):
        d = trial % 3
        V = random_mhd_states(rng, 1)[:, 0]
        V[8] = 0.0
        V[1 + d] = u
        VL, VR = V.copy(), V.copy()
        VR[0] = V[0] * rng.uniform(1.5, 6.0)
        o = _opts(glm=0)
        F, _ = O.riemann(o, VL, VR, d, 1.0)
        up = VL if u >= 0 else VR
        Fu = O.flux(o, up, d, 1.0)
        Fu[5 + d] = 0.0
        assert np.max(np.abs(F - Fu)) <= 1e-13 * (1 + np.max(np.abs(Fu))), trial
        subsonic = all(lo < 0 < hi for lo, hi in (O.speeds(o, VL, d), O.speeds(o, VR, d)))
        if u != 0.0 and subsonic:
            Fh, _ = O.riemann(_opts(glm=0, riemann="hll"), VL, VR, d, 1.0)
            assert np.max(np.abs(Fh[:5] - Fu[:5])) > 1e-4


def test_hllc_flux_is_continuous_across_a_contact_at_rest():
    """Shifting both states' normal velocity by w moves the contact speed by
    w.  Where it passes zero the solver switches from the left to the right
    star state; both star fluxes must agree there (the mass flux vanishes,
    the rest is set by the shared p_t*, B* and v*.B*), so the flux is
    continuous in w.  The zero is found by bisection on the sign of the mass
    flux."""
    rng = np.random.default_rng(53)
    o = _opts(glm=0)
    for trial in range(20):
        d = trial % 3
        VL, VR = random_mhd_states(rng, 2).T
        VR[5 + d] = VL[5 + d]

        def f(w):
            a, b = VL.copy(), VR.copy()
            a[1 + d] += w
            b[1 + d] += w
            return O.riemann(o, a, b, d, 1.0)[0]

        lo, hi = -20.0, 20.0
        assert f(lo)[0] < 0 < f(hi)[0]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid)[0] < 0:
                lo = mid
            else:
                hi = mid
            if hi - lo < 1e-13:
                break
        Fl, Fh = f(lo), f(hi)
        scale = 1 + np.max(np.abs(Fl))
        assert np.max(np.abs(Fl - Fh)) <= 1e-10 * scale, (trial, Fl - Fh)


def test_hllc_sod_converges_and_beats_hll():
    """B = 0: the Sod tube converges to the exact Euler solution at about
    first order in L1, with a smaller density error than HLL at every
    resolution (the contact is kept sharper)."""
    g = 1.4
    VL = [1.0, 0, 0, 0, 1.0, 0, 0, 0, 0]
    VR = [0.125, 0, 0, 0, 0.1, 0, 0, 0, 0]
    errs = {}
    for solver in ("hllc", "hll"):
        o = O.make_opts(dim=2, recon="lin_mc", riemann=solver, gamma=g)
        e = []
        for N in (100, 200, 400):
            x, V = _run_tube(o, VL, VR, 0.0, 1.0, 0.5, N, 0.2, cfl=0.8)
            ex = euler_exact((x - 0.5) / 0.2, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g)
            e.append(np.mean(np.abs(V[0] - ex[0])))
        errs[solver] = e
    c = errs["hllc"]
    assert c[2] < 0.006
    assert c[0] / c[1] > 1.4 and c[1] / c[2] > 1.4
    assert all(a < b for a, b in zip(errs["hllc"], errs["hll"]))


def test_hllc_step_conserves():
    V, meta = I.mhd3d_fields(n=12, ng=4, seed=2003)
    o = O.make_opts(dim=3, recon="ppm", riemann="hllc", gamma=G53, dx=meta["dx"])
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
    assert np.max(np.abs(b - a)) > 1e-6
    # and it is not HLLD or HLL under another name
    for other in ("hlld", "hll"):
        Ux, _, _, _ = O.step(O.make_opts(dim=3, recon="ppm", riemann=other, gamma=G53, dx=meta["dx"]), U, 4, dt, ch)
        assert np.max(np.abs(I.interior(Ux, 4, 3) - I.interior(Uo, 4, 3))) > 1e-8
