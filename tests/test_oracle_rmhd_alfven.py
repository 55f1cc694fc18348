"""Pin of the oracle's relativistic MHD step with a magnetic field: the
large-amplitude circularly polarised Alfven wave, an exact smooth solution of
Eq. rmhd (Del Zanna et al. 2007, ECHO paper, Sec. 4).

Along the wave normal n: rho = p = 1, B.n = B0, the transverse field of
magnitude eta B0 rotating with phase phi = k (xi - v_A t), the transverse
velocity -v_A B_perp / B0, and
    v_A^2 = B0^2 / K * 2 / (1 + sqrt(1 - (2 eta B0^2 / K)^2)),
    K = w + B0^2 (1 + eta^2),   w = rho + Gamma p / (Gamma - 1).
That this is a travelling solution is checked first, independently of the
oracle: F_n(U) - v_A U must be the same at every phase, with U and F_n
written in the covariant form T^{mu nu} = (w + b^2) u^mu u^nu
+ (p + b^2/2) eta^{mu nu} - b^mu b^nu (not the oracle's three-vector form).
Then the oracle's MUSCL-Hancock + MC + HLL + GLM step (Sec. 3.3) must
converge to it at second order on oblique grids (2D along (1,2), 3D along
(0,1,1)).  In this wave E = -v x B is normal to the wave vector, so the
divergence of the E_n E_c stress vanishes; that term, and every other one of
the three-vector flux, is pinned directly against the covariant tensor on
random states.  Planted mistakes in the flux fail one pin or both."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.plant import planted

G = 4.0 / 3.0
NG = 4


def alfven_speed(B0=1.0, eta=1.0, rho=1.0, p=1.0):
    w = rho + G / (G - 1.0) * p
    K = w + B0 * B0 * (1.0 + eta * eta)
    return math.sqrt(B0 * B0 / K * 2.0 / (1.0 + math.sqrt(1.0 - (2.0 * eta * B0 * B0 / K) ** 2)))


def covariant_flux(rho, p, v, B, n, eos="ideal"):
    """Conserved (D, m, E - D, B) and their flux along unit vector n from the
    stress-energy tensor of ideal RMHD (c = 1, Heaviside-Lorentz units)."""
    g = 1.0 / math.sqrt(1.0 - v @ v)
    if eos == "tm":  # Eq. TMEos
        w = 2.5 * p + math.sqrt(2.25 * p * p + rho * rho)
    else:            # Eq. gammaEos
        w = rho + G / (G - 1.0) * p
    b0 = g * (v @ B)
    bv = B / g + b0 * v
    b2 = (B @ B) / g ** 2 + (v @ B) ** 2
    wt, pt = w + b2, p + 0.5 * b2
    u = g * v
    m = wt * g * u - b0 * bv
    E = wt * g * g - pt - b0 * b0
    un, bn = u @ n, bv @ n
    Fm = wt * un * u - bn * bv + pt * n
    FB = (v @ n) * B - (B @ n) * v
    U = np.concatenate([[rho * g], m, [E - rho * g], B])
    F = np.concatenate([[rho * un], Fm, [m @ n - rho * un], FB])
    return U, F


@pytest.mark.parametrize("eos", ["ideal", "tm"])
def test_rmhd_state_and_flux_match_the_stress_energy_tensor(eos):
    """The oracle's conserved variables and physical fluxes (three-vector
    form with E = -v x B) against T^{0 mu} and T^{d mu} of the covariant
    form, for random states with fields in every direction; every magnetic
    term of the flux (B_n B_c, E_n E_c, the E^2 / 2 pressure) is nonzero."""
    rng = np.random.default_rng(4242)
    o = O.make_opts(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", gamma=G, eos=eos,
                    glm=False)
    for _ in range(200):
        rho = 10 ** rng.uniform(-1, 1)
        p = 10 ** rng.uniform(-2, 1)
        u = rng.normal(size=3)
        v = u / np.linalg.norm(u) * rng.uniform(0.0, 0.99)
        B = rng.uniform(-3, 3, size=3)
        V = np.array([rho, *v, p, *B, 0.0])
        Uo = O.prim2cons(o, V)
        for d in range(3):
            n = np.eye(3)[d]
            U, F = covariant_flux(rho, p, v, B, n, eos)
            Fo = O.flux(o, V, d)
            sU = np.abs(U).max()
            assert np.abs(Uo[:8] - U).max() < 1e-12 * sU
            assert np.abs(Fo[:8] - F).max() < 1e-12 * (np.abs(F).max() + sU)


def frame(kint):
    k = np.asarray(kint, float)
    n = k / np.linalg.norm(k)
    a = np.array([0.0, 0.0, 1.0]) if abs(n[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    t = a - (a @ n) * n
    t /= np.linalg.norm(t)
    return n, t, np.cross(n, t)


def wave_state(phi, n, t, b, B0=1.0, eta=1.0):
    vA = alfven_speed(B0, eta)
    Bp = eta * B0 * (np.cos(phi) * t + np.sin(phi) * b)
    return 1.0, 1.0, -vA * Bp / B0, B0 * n + Bp


def test_cp_alfven_wave_is_a_travelling_solution():
    vA = alfven_speed()
    for kint in ((1, 0, 0), (1, 2, 0), (0, 1, 1)):
        n, t, b = frame(kint)
        rows = []
        for phi in np.linspace(0.0, 2.0 * math.pi, 17):
            rho, p, v, B = wave_state(phi, n, t, b)
            U, F = covariant_flux(rho, p, v, B, n)
            rows.append(F - vA * U)
        rows = np.array(rows)
        assert np.abs(rows - rows[0]).max() < 1e-14


def fields(kint, N, dim, time):
    dx = 1.0 / N
    x = (np.arange(-NG, N + NG) + 0.5) * dx
    if dim == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        X, Y, Z = X[None], Y[None], np.zeros_like(X)[None]
    else:
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    n, t, b = frame(kint)
    kn = 2.0 * math.pi * np.linalg.norm(kint)
    phi = 2.0 * math.pi * (kint[0] * X + kint[1] * Y + kint[2] * Z) - kn * alfven_speed() * time
    V = np.zeros((9,) + X.shape)
    rho, p, v, B = wave_state(phi[None], n[:, None, None, None], t[:, None, None, None], b[:, None, None, None])
    V[0], V[4] = rho, p
    V[1:4] = v
    V[5:8] = B
    return V, dx


def alfven_error(kint, N, dim, frac=0.5):
    """L1 error (mean over cells, summed over the 8 conserved variables
    other than psi) after `frac` of a wave period."""
    V, dx = fields(kint, N, dim, 0.0)
    o = O.make_opts(dim=dim, physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", gamma=G,
                    dx=(dx, dx, dx if dim == 3 else 1.0))
    U = O.prim2cons(o, V)
    T = frac / (np.linalg.norm(kint) * alfven_speed())
    t = 0.0
    while t < T - 1e-14:
        dt0 = 0.3 / O.cfl_rate(o, U, NG)
        dt = min(dt0, T - t)
        U, _, _, fails = O.step(o, U, NG, dt, min(0.3 * dx / dt0, 1.0))
        assert fails == [0] * 5
        I.fill_periodic(U, NG, dim)
        t += dt
    Ve, _ = fields(kint, N, dim, T)
    Ue = O.prim2cons(o, Ve)
    d = np.abs(I.interior(U, NG, dim) - I.interior(Ue, NG, dim))[:8]
    return d.reshape(8, -1).mean(axis=1).sum()


CASES = {"2d_k12": ((1, 2, 0), 2, (16, 32, 64)), "3d_k011": ((0, 1, 1), 3, (8, 16, 32))}


def converges(case):
    kint, dim, ns = CASES[case]
    e = [alfven_error(kint, n, dim) for n in ns]
    return e, (e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5)


@pytest.mark.parametrize("case", sorted(CASES))
def test_rmhd_cp_alfven_wave_second_order(case):
    e, ok = converges(case)
    assert ok, e


PLANTS = {
    "dropped E_n E_c": ("- E[n] * E[c] + (c == n ? pt : 0.0);", "- 0.0 * E[c] + (c == n ? pt : 0.0);"),
    "total pressure without E^2": ("double pt = V[PRS] + 0.5 * (B2 + E2);", "double pt = V[PRS] + 0.5 * B2;"),
    "dropped B_n B_c": ("- V[BX1 + n] * V[BX1 + c] - E[n] * E[c]", "- 0.0 * V[BX1 + c] - E[n] * E[c]"),
    "induction sign": ("F[BX1 + t] = vn * V[BX1 + t] - V[BX1 + n] * V[MX1 + t];",
                       "F[BX1 + t] = vn * V[BX1 + t] + V[BX1 + n] * V[MX1 + t];"),
}


def _fails(test, *args):
    try:
        test(*args)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_rmhd_flux_mistake_fails(plant):
    """Each planted mistake fails the tensor pin, the wave pin or both (the
    E_n E_c term cannot show in the wave: there E is normal to the wave
    vector, so its divergence vanishes)."""
    old, new = PLANTS[plant]
    with planted(old, new):
        tensor = _fails(test_rmhd_state_and_flux_match_the_stress_energy_tensor, "ideal")
        wave = _fails(test_rmhd_cp_alfven_wave_second_order, "2d_k12") if plant != "dropped E_n E_c" else False
        assert tensor or wave
