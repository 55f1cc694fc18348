"""Pins of the oracle's Roe solver for ideal MHD (Sec. 3.1's list; the solver
of the paper's own MHD tests).  Its defining property is that the averaged
matrix turns the conserved jump into the flux jump exactly, A (U_R - U_L) =
F_R - F_L: when every wave moves the same way the flux is then F_L or F_R
to rounding, which is checked for random states, degenerate fields
included.  Further: reduction to the textbook Euler Roe flux (Toro,
Sec. 11.2) when B = 0, written out here; invariance under rotations about
the normal, degenerate fields included; exact upwinding of single-wave
discontinuities (entropy wave, rotational discontinuity); first-order
convergence on the Sod tube with errors below HLL's; a conservative 3D
step."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.exact_riemann import sample as euler_exact
from tests.test_oracle_pins import G53, _run_tube, random_mhd_states


def _opts(**kw):
    return O.make_opts(**dict(dict(physics="mhd", riemann="roe", gamma=G53, recon="lin_mc", glm=False), **kw))


def _phys(o, V, d):
    F = O.flux(o, V, d, 1.0)
    F[5 + d] = 0.0
    F[8] = 0.0
    return F


@pytest.mark.parametrize("case", ["generic", "Bt0", "Bn0", "B0", "Bt_reversal"])
@pytest.mark.parametrize("sign", [1, -1])
def test_roe_property_for_one_sided_waves(case, sign):
    """Both states moving faster than every wave of both states and of the
    average: F = F_L (all waves right-going) or F_R (all left-going), which
    holds only if A dU = dF exactly."""
    rng = np.random.default_rng(61 + (sign > 0))
    o = _opts()
    worst = 0.0
    for trial in range(60):
        d = trial % 3
        VL, VR = random_mhd_states(rng, 2).T
        VL[8] = VR[8] = 0.0
        VR[5 + d] = VL[5 + d]
        t, b = [k for k in range(3) if k != d]
        if case == "Bt0":
            for V in (VL, VR):
                V[5 + t] = V[5 + b] = 0.0
        elif case == "Bn0":
            VL[5 + d] = VR[5 + d] = 0.0
        elif case == "B0":
            VL[5:8] = VR[5:8] = 0.0
        elif case == "Bt_reversal":
            VR[5 + t], VR[5 + b] = -VL[5 + t], -VL[5 + b]
        VL[1 + d] = VR[1 + d] = 0.0
        c = max(max(abs(x) for x in O.speeds(o, V, d)) for V in (VL, VR))
        shift = sign * (6.0 * c + 2.0)
        VL[1 + d] += shift + rng.uniform(-0.5, 0.5) * c
        VR[1 + d] += shift + rng.uniform(-0.5, 0.5) * c
        F, smax = O.riemann(o, VL, VR, d, 1.0)
        Fu = _phys(o, VL if sign > 0 else VR, d)
        worst = max(worst, np.max(np.abs(F - Fu)) / (1.0 + np.max(np.abs(Fu))))
        assert smax >= max(abs(x) for V in (VL, VR) for x in O.speeds(o, V, d)) - 1e-12
    assert worst < 5e-14, worst


def _euler_roe(VL, VR, d, g):
    """Textbook Roe flux for the 3D Euler equations (Toro, Sec. 11.2): Roe
    averages u~, H~, a~^2 = (g - 1)(H~ - |u~|^2/2); wave strengths
      a2 = (g-1)/a~^2 (drho (H~ - u~^2) + u~ dm_n - dE'),
      dE' = dE - (dm_t - v~_t drho) v~_t - (dm_b - v~_b drho) v~_b,
      a1 = (drho (u~ + a~) - dm_n - a~ a2)/(2 a~),  a5 = drho - a1 - a2,
      a3, a4 = dm_t - v~_t drho, dm_b - v~_b drho."""
    t, b = [k for k in range(3) if k != d]

    def cons(V):
        v2 = V[1] ** 2 + V[2] ** 2 + V[3] ** 2
        return np.array([V[0], V[0] * V[1 + d], V[0] * V[1 + t], V[0] * V[1 + b], V[4] / (g - 1) + 0.5 * V[0] * v2])

    def flux(V, U):
        u = V[1 + d]
        F = U * u
        F[1] += V[4]
        F[4] += V[4] * u
        return F

    UL, UR = cons(VL), cons(VR)
    FL, FR = flux(VL, UL), flux(VR, UR)
    sL, sR = math.sqrt(VL[0]), math.sqrt(VR[0])
    avg = lambda a, c: (sL * a + sR * c) / (sL + sR)
    u, v, w = avg(VL[1 + d], VR[1 + d]), avg(VL[1 + t], VR[1 + t]), avg(VL[1 + b], VR[1 + b])
    H = avg((UL[4] + VL[4]) / VL[0], (UR[4] + VR[4]) / VR[0])
    q2 = u * u + v * v + w * w
    a = math.sqrt((g - 1) * (H - 0.5 * q2))
    dU = UR - UL
    a3 = dU[2] - v * dU[0]
    a4 = dU[3] - w * dU[0]
    dE = dU[4] - a3 * v - a4 * w
    a2 = (g - 1) / a ** 2 * (dU[0] * (H - u * u) + u * dU[1] - dE)
    a1 = (dU[0] * (u + a) - dU[1] - a * a2) / (2 * a)
    a5 = dU[0] - a1 - a2
    K1 = np.array([1, u - a, v, w, H - u * a])
    K2 = np.array([1, u, v, w, 0.5 * q2])
    K3 = np.array([0, 0, 1, 0, v])
    K4 = np.array([0, 0, 0, 1, w])
    K5 = np.array([1, u + a, v, w, H + u * a])
    D = abs(u - a) * a1 * K1 + abs(u) * (a2 * K2 + a3 * K3 + a4 * K4) + abs(u + a) * a5 * K5
    F = 0.5 * (FL + FR) - 0.5 * D
    out = np.zeros(5)
    out[0], out[1 + d], out[1 + t], out[1 + b], out[4] = F[0], F[1], F[2], F[3], F[4]
    return out


@pytest.mark.parametrize("shear", [True, False])
def test_roe_reduces_to_euler_roe_without_field(shear):
    """B = 0: Toro's Euler Roe flux in every direction, for random states
    with shear, and for states without shear around a left sonic point."""
    rng = np.random.default_rng(62 + shear)
    g = 1.4
    o = _opts(gamma=g)
    for trial in range(80):
        d = trial % 3
        VL, VR = np.zeros(9), np.zeros(9)
        for V in (VL, VR):
            V[0] = rng.uniform(0.1, 3.0)
            V[4] = rng.uniform(0.05, 3.0)
            V[1:4] = rng.normal(0, 1.2, 3)
        if not shear:
            VR[1:4] = VL[1:4]
            VR[1 + d] = VL[1 + d] + rng.uniform(0, 3.0)
            cL = math.sqrt(g * VL[4] / VL[0])
            VL[1 + d] = cL * rng.uniform(0.5, 1.2)   # around the left sonic point
        F, _ = O.riemann(o, VL, VR, d, 1.0)
        Ft = _euler_roe(VL, VR, d, g)
        assert np.max(np.abs(F[:5] - Ft)) <= 1e-13 * (1 + np.max(np.abs(Ft))), trial


@pytest.mark.parametrize("case", ["generic", "Bt0_a_below_ca", "Bt0_a_above_ca", "Bn0"])
def test_roe_is_invariant_under_rotation_about_the_normal(case):
    """Rotating the transverse velocity and field of both states by phi
    rotates the transverse fluxes by phi and leaves the rest unchanged.  With
    B_t = 0 the eigenvectors of one polarisation are a fast or slow pair and
    of the other the Alfven pair, at equal speeds; they must be damped
    alike (the averaged state may order a~ and c_a~ differently from the
    two states)."""
    rng = np.random.default_rng(65)
    o = _opts()
    for trial in range(40):
        d = trial % 3
        t, b = [k for k in range(3) if k != d]
        VL, VR = random_mhd_states(rng, 2).T
        VL[8] = VR[8] = 0.0
        VR[5 + d] = VL[5 + d]
        if case.startswith("Bt0"):
            for V in (VL, VR):
                V[5 + t] = V[5 + b] = 0.0
                # sound speed below or above the Alfven speed in both states
                ca2 = V[5 + d] ** 2 / V[0]
                V[4] = V[0] * ca2 / G53 * (0.3 if case.endswith("below_ca") else 3.0)
        elif case == "Bn0":
            VL[5 + d] = VR[5 + d] = 0.0
        # near-sonic normal flow
        VL[1 + d] = rng.uniform(-0.5, 0.5)
        VR[1 + d] = VL[1 + d] + rng.uniform(0.0, 1.5)
        F, s0 = O.riemann(o, VL, VR, d, 1.0)
        phi = rng.uniform(0, 2 * math.pi)
        c, s = math.cos(phi), math.sin(phi)
        WL, WR = VL.copy(), VR.copy()
        for V, W in ((VL, WL), (VR, WR)):
            for base in (1, 5):
                W[base + t] = c * V[base + t] - s * V[base + b]
                W[base + b] = s * V[base + t] + c * V[base + b]
        G, s1 = O.riemann(o, WL, WR, d, 1.0)
        Fr = F.copy()
        for base in (1, 5):
            Fr[base + t] = c * F[base + t] - s * F[base + b]
            Fr[base + b] = s * F[base + t] + c * F[base + b]
        assert np.max(np.abs(G - Fr)) <= 1e-12 * (1 + np.max(np.abs(F))), (trial, G - Fr)
        assert abs(s1 - s0) <= 1e-13 * s0


@pytest.mark.parametrize("u", [0.0, 0.37, -1.1])
def test_roe_carries_an_entropy_wave_exactly(u):
    """Density jump only (continuous v, p and oblique B): the exact flux is
    the upwind physical flux."""
    rng = np.random.default_rng(64)
    o = _opts()
    for trial in range(20):
        d = trial % 3
        V = random_mhd_states(rng, 1)[:, 0]
        V[8] = 0.0
        V[1 + d] = u
        VL, VR = V.copy(), V.copy()
        VR[0] = V[0] * rng.uniform(1.5, 6.0)
        F, _ = O.riemann(o, VL, VR, d, 1.0)
        Fu = _phys(o, VL if u >= 0 else VR, d)
        assert np.max(np.abs(F - Fu)) <= 1e-13 * (1 + np.max(np.abs(Fu))), trial


@pytest.mark.parametrize("w", [0.0, 0.3, -0.45])
def test_roe_resolves_rotational_discontinuity(w):
    """A rotational discontinuity (|B_t|, rho, p, v_n continuous; B_t turned
    by 0.9 rad; v_t - B_t/sqrt(rho) continuous) moves at v_n - c_a; in the
    frame where it moves at w its jump is an Alfven eigenvector of the Roe
    matrix, and the flux is the upwind one exactly."""
    o = _opts()
    rho, p, Bn = 1.3, 0.5, 0.8
    ca = Bn / math.sqrt(rho)
    th = 0.9
    BtL = np.array([0.6, 0.0])
    BtR = np.array([0.6 * math.cos(th), 0.6 * math.sin(th)])
    vtL = np.array([0.1, -0.2])
    vtR = vtL + (BtR - BtL) / math.sqrt(rho)
    vn = ca + w
    VL = np.array([rho, vn, vtL[0], vtL[1], p, Bn, BtL[0], BtL[1], 0.0])
    VR = np.array([rho, vn, vtR[0], vtR[1], p, Bn, BtR[0], BtR[1], 0.0])
    FL, FR = _phys(o, VL, 0), _phys(o, VR, 0)
    UL = O.prim2cons(o, VL[:, None])[:, 0]
    UR = O.prim2cons(o, VR[:, None])[:, 0]
    # the set-up satisfies the jump condition at speed w
    assert np.max(np.abs((FR - FL)[:8] - w * (UR - UL)[:8])) < 1e-14
    F, _ = O.riemann(o, VL, VR, 0, 1.0)
    Fu = FL if w >= 0 else FR
    assert np.max(np.abs(F - Fu)) < 1e-13


def test_roe_sod_converges_and_beats_hll():
    """B = 0: the Sod tube converges to the exact Euler solution at about
    first order in L1, with a smaller density error than HLL."""
    g = 1.4
    VL = [1.0, 0, 0, 0, 1.0, 0, 0, 0, 0]
    VR = [0.125, 0, 0, 0, 0.1, 0, 0, 0, 0]
    errs = {}
    for solver in ("roe", "hll"):
        o = O.make_opts(dim=2, recon="lin_mc", riemann=solver, gamma=g)
        e = []
        for N in (100, 200, 400):
            x, V = _run_tube(o, VL, VR, 0.0, 1.0, 0.5, N, 0.2, cfl=0.8)
            ex = euler_exact((x - 0.5) / 0.2, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g)
            e.append(np.mean(np.abs(V[0] - ex[0])))
        errs[solver] = e
    r = errs["roe"]
    assert r[2] < 0.006
    assert r[0] / r[1] > 1.4 and r[1] / r[2] > 1.4
    assert all(a < b for a, b in zip(errs["roe"], errs["hll"]))


def test_roe_step_conserves():
    V, meta = I.mhd3d_fields(n=12, ng=4, seed=2003)
    o = O.make_opts(dim=3, recon="ppm", riemann="roe", gamma=G53, dx=meta["dx"])
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
    for other in ("hlld", "hllc"):
        Ux, _, _, _ = O.step(O.make_opts(dim=3, recon="ppm", riemann=other, gamma=G53, dx=meta["dx"]), U, 4, dt, ch)
        assert np.max(np.abs(I.interior(Ux, 4, 3) - I.interior(Uo, 4, 3))) > 1e-8
