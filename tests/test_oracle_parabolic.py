"""Pins of the oracle's parabolic fluxes on oblique and compressive modes.

What is pinned: Eq. visc_tens (with its compressive -2/3 div v term), the
resistive flux of -curl(eta J), the anisotropic conduction flux of Eq.
tc_flux (the b b projection, classical limit), the four-point transverse
gradients of App. A, the energy fluxes v.tau and -eta (J x B)_n, and the
unsplit midpoint update of Sec. 3.1 (Pi^n for the half step, Pi^{n+1/2} for
the update).

With the hyperbolic flux off and uniform density, one step maps a Fourier
mode of velocity, field or temperature linearly: the amplitude vector is
multiplied by G = I + dt T + dt^2 T^2 / 2, where T is the discrete symbol of
the operator.  T is derived here from the face stencils:
  * at a face normal to n, the normal derivative is the two-point difference,
    symbol 2i sin(k_n dx/2)/dx relative to the face value;
  * a transverse derivative (e != n) averages the centred differences of the
    two cells of the face, symbol i cos(k_n dx/2) sin(k_e dx)/dx;
  * the cell's flux difference multiplies by s_n = 2i sin(k_n dx/2)/dx.
Three kinds of check follow:
  1. exact: the oracle's one-step field equals Re(G a e^{i k.x}) to
     round-off, for modes along (1,1), (1,2) in 2D and (1,1,1), (1,2,-1)
     in 3D, including compressive velocity and non-solenoidal field modes;
  2. continuum: the decay rate read off the oracle's step converges at second
     order to nu k^2 (shear), 4/3 nu k^2 (compressive), eta k^2 and
     (Gamma-1)[kpar (b.k)^2 + kperp (k^2 - (b.k)^2)]/rho;
  3. heating: the pressure change of a step converges at second order to the
     time integral of the dissipation, rho nu k^2 |a|^2 cos^2 (shear),
     4/3 rho nu k^2 |a|^2 cos^2 (compressive) and eta k^2 |a|^2 cos^2, which
     fixes the energy fluxes (a dropped or reversed one moves the heat to
     sin^2 or flips its sign).
Each check is shown to fail on a planted mistake in a copy of the oracle."""
import math

import numpy as np
import pytest

import oracle as O
from tests.plant import planted

G53 = 5.0 / 3.0
NG = 4
KPAR, KPERP = 5e-3, 1e-3


def coords(n, dim):
    dx = 1.0 / n
    x = (np.arange(-NG, n + NG) + 0.5) * dx
    if dim == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        return X[None], Y[None], np.zeros_like(X)[None], dx
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z, dx


def interior(a, dim):
    if dim == 2:
        return a[..., :, NG:-NG, NG:-NG]
    return a[..., NG:-NG, NG:-NG, NG:-NG]


def face_derivs(kv, dx, dim, n):
    """Symbols of the derivatives along e at a face normal to n."""
    D = np.zeros(3, complex)
    for e in range(dim):
        if e == n:
            D[e] = 2j * math.sin(kv[n] * dx / 2) / dx
        else:
            D[e] = 1j * math.cos(kv[n] * dx / 2) * math.sin(kv[e] * dx) / dx
    return D


def symbol(kind, kv, dx, dim, bhat=None):
    """Discrete symbol T of the parabolic operator (3x3 for velocity or
    field, 1x1 for temperature), unit coefficient (nu, eta; conduction with
    its own kappas and Gamma - 1)."""
    if kind == "tc":
        K = KPERP * np.eye(3) + (KPAR - KPERP) * np.outer(bhat, bhat)
        lam = 0.0
        for n in range(dim):
            D = face_derivs(kv, dx, dim, n)
            lam += 2j * math.sin(kv[n] * dx / 2) / dx * (K[n] @ D)
        return np.array([[(G53 - 1.0) * lam]])
    T = np.zeros((3, 3), complex)
    for n in range(dim):
        D = face_derivs(kv, dx, dim, n)
        s = 2j * math.sin(kv[n] * dx / 2) / dx
        for c in range(3):
            for cp in range(3):
                if kind == "visc":  # rho nu (d_n v_c + d_c v_n - 2/3 delta_nc div v)
                    t = (D[n] if c == cp else 0) + (D[c] if cp == n else 0) - (2.0 / 3.0 * D[cp] if c == n else 0)
                else:  # eta (d_n B_c - d_c B_n)
                    t = (D[n] if c == cp else 0) - (D[c] if cp == n else 0)
                T[c, cp] += s * t
    return T


def run_mode(kind, dim, n, kint, amp, bvec=(0.0, 0.0, 0.0), zdt=0.2):
    """One oracle step of a mode with the hyperbolic flux off.

    kind: 'visc' (velocity amp sin(k.x)), 'res' (field amp sin(k.x) on top
    of bvec), 'tc' (pressure 1 + amp sin(k.x), field bvec).  Returns the
    initial and final primitive interiors, the phase, dt, dx, k."""
    X, Y, Z, dx = coords(n, dim)
    kv = 2.0 * math.pi * np.asarray(kint, float)
    th = kv[0] * X + kv[1] * Y + kv[2] * Z
    V = np.zeros((9,) + X.shape)
    V[0] = 1.0
    V[4] = 1.0
    for c in range(3):
        V[5 + c] = bvec[c]
    coef = dict(nu=0.0, eta=0.0, kappa_par=0.0, kappa_perp=0.0)
    if kind == "visc":
        for c in range(3):
            V[1 + c] = amp[c] * np.sin(th)
        mask, coef["nu"], D = O.PARAB_VISC, 3e-3, 3e-3
    elif kind == "res":
        for c in range(3):
            V[5 + c] += amp[c] * np.sin(th)
        mask, coef["eta"], D = O.PARAB_RES, 2e-3, 2e-3
    else:
        V[4] = 1.0 + amp * np.sin(th)
        mask, coef["kappa_par"], coef["kappa_perp"] = O.PARAB_TC, KPAR, KPERP
        D = (G53 - 1.0) * KPAR
    o = O.make_opts(dim=dim, recon="lin_mc", gamma=G53, dx=(dx, dx, dx if dim == 3 else 1.0),
                    parabolic_mask=mask, tc_phi=0.0, hyperbolic_off=True, glm=False, **coef)
    U = O.prim2cons(o, V)
    dt = zdt * dx * dx / D
    Uo, _, _, fails = O.step(o, U, NG, dt, 1.0)
    assert fails == [0] * 5
    Vo, _ = O.cons2prim(o, Uo)
    return interior(V, dim), interior(Vo, dim), interior(th, dim), dt, dx, kv, coef


def exact_error(kind, dim, n, kint, amp, bvec=(0.0, 0.0, 0.0)):
    """max |oracle - Re(G a e^{i th})| / |a| after one step."""
    V0, V1, th, dt, dx, kv, coef = run_mode(kind, dim, n, kint, amp, bvec)
    if kind == "tc":
        b = np.asarray(bvec, float)
        T = symbol("tc", kv, dx, dim, b / np.linalg.norm(b))
        a = np.array([amp], complex)
        got = V1[4:5]  # rho = 1: temperature = pressure
        base = 1.0
    else:
        c = coef["nu"] if kind == "visc" else coef["eta"]
        T = c * symbol(kind, kv, dx, dim)
        a = np.asarray(amp, complex)
        got = V1[1:4] if kind == "visc" else V1[5:8]
        base = 0.0 if kind == "visc" else np.asarray(bvec, float)[:, None, None, None]
    G = np.eye(len(a)) + dt * T + 0.5 * dt * dt * (T @ T)
    ahat = G @ (-1j * a)  # a sin(th) = Re(-i a e^{i th})
    want = np.real(ahat[:, None, None, None] * np.exp(1j * th)[None])
    return np.abs(got - base - want).max() / np.linalg.norm(np.atleast_1d(amp))


def rate_error(kind, dim, n, kint, amp, bvec=(0.0, 0.0, 0.0)):
    """Relative difference between the decay rate of the oracle's step and
    the continuum rate of the mode."""
    V0, V1, th, dt, dx, kv, coef = run_mode(kind, dim, n, kint, amp, bvec)
    k2 = float(kv @ kv)
    if kind == "tc":
        f = V1[4] - 1.0
        b = np.asarray(bvec, float) / np.linalg.norm(bvec)
        bk = float(b @ kv)
        cont = (G53 - 1.0) * (KPAR * bk * bk + KPERP * (k2 - bk * bk))
        a0 = amp
    else:
        a = np.asarray(amp, float)
        fld = V1[1:4] if kind == "visc" else V1[5:8] - np.asarray(bvec, float)[:, None, None, None]
        f = np.tensordot(a / np.linalg.norm(a), fld, axes=1)
        a0 = np.linalg.norm(a)
        if kind == "visc":
            comp = abs(float(a @ kv)) > 0.5 * np.linalg.norm(a) * math.sqrt(k2)
            cont = coef["nu"] * k2 * (4.0 / 3.0 if comp else 1.0)
        else:
            cont = coef["eta"] * k2
    s = np.sin(th).ravel()
    g = float(f.ravel() @ s / (s @ s)) / a0  # amplification of the mode
    z = 1.0 - math.sqrt(2.0 * g - 1.0)       # g = 1 - z + z^2 / 2 (midpoint rule)
    return abs(z / dt - cont) / cont


def heating_error(kind, dim, n, kint, amp):
    """Relative L-inf difference between the step's pressure change and
    (Gamma-1) times the time integral of the dissipation over the step."""
    V0, V1, th, dt, dx, kv, coef = run_mode(kind, dim, n, kint, amp)
    k2 = float(kv @ kv)
    a = np.asarray(amp, float)
    a2 = float(a @ a)
    if kind == "visc":
        comp = abs(float(a @ kv)) > 0.5 * math.sqrt(a2 * k2)
        fac = 4.0 / 3.0 if comp else 1.0
        lam = coef["nu"] * k2 * fac
        phi0 = coef["nu"] * k2 * a2 * fac * np.cos(th) ** 2
    else:
        lam = coef["eta"] * k2
        phi0 = coef["eta"] * k2 * a2 * np.cos(th) ** 2
    # amplitude ~ exp(-lam t): dissipation ~ exp(-2 lam t)
    want = (G53 - 1.0) * phi0 * (1.0 - math.exp(-2.0 * lam * dt)) / (2.0 * lam)
    got = V1[4] - V0[4]
    return np.abs(got - want).max() / np.abs(want).max()


# ---------------------------------------------------------------------------
# mode catalogue: (kind, dim, k, amplitude, background field)
SQ2 = 1.0 / math.sqrt(2.0)
EXACT = {
    "visc_shear_2d": ("visc", 2, (1, 1, 0), (0.1 * SQ2, -0.1 * SQ2, 0.05), (0, 0, 0)),
    "visc_comp_2d": ("visc", 2, (1, 2, 0), (0.03, 0.06, 0.0), (0, 0, 0)),
    "visc_mixed_3d": ("visc", 3, (1, 2, -1), (0.05, -0.02, 0.07), (0, 0, 0)),
    "res_2d": ("res", 2, (1, 1, 0), (0.05, -0.02, 0.08), (0.3, -0.2, 0.1)),
    "res_3d": ("res", 3, (1, 1, 1), (0.04, 0.01, -0.06), (0.0, 0.0, 0.0)),
    "tc_2d": ("tc", 2, (1, 1, 0), 0.01, (0.5, 0.5 * math.sqrt(3.0), 0.0)),
    "tc_3d": ("tc", 3, (1, 1, 1), 0.01, (1.0, 1.0, 0.0)),
    "tc_3d_oblique_b": ("tc", 3, (1, 2, -1), 0.01, (1.0, 2.0, 2.0)),
}


@pytest.mark.parametrize("case", sorted(EXACT))
def test_parabolic_mode_matches_discrete_symbol(case):
    kind, dim, k, amp, b = EXACT[case]
    n = 16 if dim == 2 else 8
    assert exact_error(kind, dim, n, k, amp, b) < 1e-12


CONT = {
    "visc_shear_2d": ("visc", 2, (1, 1, 0), (SQ2, -SQ2, 0.0), (0, 0, 0)),
    "visc_comp_2d": ("visc", 2, (1, 1, 0), (SQ2, SQ2, 0.0), (0, 0, 0)),
    "visc_comp_3d": ("visc", 3, (1, 1, 1), (1.0, 1.0, 1.0), (0, 0, 0)),
    "res_2d": ("res", 2, (1, 1, 0), (SQ2, -SQ2, 0.0), (0, 0, 0)),
    "res_3d": ("res", 3, (1, 1, 1), (1.0, -1.0, 0.0), (0, 0, 0)),
    "tc_2d": ("tc", 2, (1, 1, 0), 0.01, (0.5, 0.5 * math.sqrt(3.0), 0.0)),
    "tc_3d": ("tc", 3, (1, 1, 1), 0.01, (1.0, 1.0, 0.0)),
}


def _scale_amp(kind, amp):
    return amp if kind == "tc" else tuple(0.05 * x for x in amp)


@pytest.mark.parametrize("case", sorted(CONT))
def test_parabolic_rate_converges_to_continuum(case):
    kind, dim, k, amp, b = CONT[case]
    ns = (16, 32, 64) if dim == 2 else (8, 16, 32)
    e = [rate_error(kind, dim, n, k, _scale_amp(kind, amp), b) for n in ns]
    assert e[-1] < 0.02, e
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.7, e


HEAT = {
    "visc_shear_2d": ("visc", 2, (1, 1, 0), (0.1 * SQ2, -0.1 * SQ2, 0.0)),
    "visc_comp_2d": ("visc", 2, (1, 1, 0), (0.1 * SQ2, 0.1 * SQ2, 0.0)),
    "res_2d": ("res", 2, (1, 1, 0), (0.1 * SQ2, -0.1 * SQ2, 0.05)),
    "res_3d": ("res", 3, (1, 1, 1), (0.1 * SQ2, -0.1 * SQ2, 0.0)),
}


@pytest.mark.parametrize("case", sorted(HEAT))
def test_parabolic_heating_converges(case):
    kind, dim, k, amp = HEAT[case]
    ns = (16, 32, 64) if dim == 2 else (8, 16, 32)
    e = [heating_error(kind, dim, n, k, amp) for n in ns]
    assert e[-1] < 0.05, e
    assert e[0] / e[1] > 3.0 and e[1] / e[2] > 3.5, e


# ---------------------------------------------------------------------------
# planted mistakes: each must fail at least one of the checks above

PLANTS = {
    "dropped -2/3 div v": ("(c == n ? 2.0 / 3.0 * divv : 0.0)", "(c == n ? 0.0 * divv : 0.0)",
                           [("exact", "visc_comp_2d"), ("rate", "visc_comp_2d"), ("heat", "visc_comp_2d")]),
    "transverse average over 2 dx": ("grad[f][e] = (up - dn) / (4.0 * o->dx[e]);",
                                     "grad[f][e] = (up - dn) / (2.0 * o->dx[e]);",
                                     [("exact", "visc_shear_2d"), ("rate", "visc_shear_2d"),
                                      ("rate", "tc_2d"), ("rate", "res_3d")]),
    "transverse difference of one cell": (
        "double up = FVAL(i + ei, j + ej, k + ek) + FVAL(ai + ei, aj + ej, ak + ek);",
        "double up = 2.0 * FVAL(i + ei, j + ej, k + ek);",
        [("exact", "visc_shear_2d"), ("exact", "tc_2d"), ("rate", "visc_shear_2d")]),
    "b b projection without cross terms": (
        "double bgT = bh[0] * grad[6][0] + bh[1] * grad[6][1] + bh[2] * grad[6][2];",
        "double bgT = bh[n] * grad[6][n];",
        [("exact", "tc_2d"), ("exact", "tc_3d_oblique_b"), ("rate", "tc_3d")]),
    "reversed v.tau energy flux": ("Pi[ENG] += vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2];",
                                   "Pi[ENG] -= vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2];",
                                   [("heat", "visc_shear_2d"), ("heat", "visc_comp_2d")]),
    "no v.tau energy flux": ("Pi[ENG] += vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2];",
                             "Pi[ENG] += 0.0 * vf[0];",
                             [("heat", "visc_shear_2d")]),
    "reversed ohmic energy flux": ("Pi[ENG] += -o->eta * JxB_n;", "Pi[ENG] += o->eta * JxB_n;",
                                   [("heat", "res_2d"), ("heat", "res_3d")]),
    "J_y with the wrong sign": ("J[1] = grad[3][2] - grad[5][0];", "J[1] = grad[5][0] - grad[3][2];",
                                [("exact", "res_2d"), ("exact", "res_3d")]),
}


def _check_fails(what, case):
    if what == "exact":
        kind, dim, k, amp, b = EXACT[case]
        return exact_error(kind, dim, 16 if dim == 2 else 8, k, amp, b) >= 1e-12
    if what == "rate":
        kind, dim, k, amp, b = CONT[case]
        ns = (16, 32, 64) if dim == 2 else (8, 16, 32)
        e = [rate_error(kind, dim, n, k, _scale_amp(kind, amp), b) for n in ns]
        return not (e[-1] < 0.02 and e[0] / e[1] > 3.5 and e[1] / e[2] > 3.7)
    kind, dim, k, amp = HEAT[case]
    ns = (16, 32, 64) if dim == 2 else (8, 16, 32)
    e = [heating_error(kind, dim, n, k, amp) for n in ns]
    return not (e[-1] < 0.05 and e[0] / e[1] > 3.0 and e[1] / e[2] > 3.5)


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_parabolic_mistake_fails_a_pin(plant):
    old, new, checks = PLANTS[plant]
    with planted(old, new):
        for what, case in checks:
            assert _check_fails(what, case), (plant, what, case)
