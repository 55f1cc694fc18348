"""Pins of the oracle's exact relativistic fast magnetosonic speeds (the
outermost roots of the lab-frame dispersion quartic, the alternative to the
isotropic bound; used by HLL / Rusanov and the CFL rate): closed forms of
special cases -- sound waves boosted by relativistic velocity addition
(B = 0), the rest-frame fast speed across the field
(c_s^2 + c_a^2 - c_s^2 c_a^2) and along it (max(c_s, c_a)), the boosted
parallel case -- then agreement with a brute-force root scan and the
enclosing bound for general states, and the step's conservation."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.test_oracle_pins import rmhd_quartic

G = 4.0 / 3.0


def opts(exact=True, eos="ideal"):
    return O.make_opts(physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", gamma=G, eos=eos,
                       exact_speeds=exact)


def state(rho, p, v=(0, 0, 0), B=(0, 0, 0)):
    V = np.zeros(9)
    V[0], V[4] = rho, p
    V[1:4] = v
    V[5:8] = B
    return V


def cs2_ca2(rho, p, B2):
    w = rho + G * p / (G - 1)
    return G * p / w, B2 / (w + B2)


@pytest.mark.parametrize("vd", [0.0, 0.5, -0.9, 0.99])
def test_unmagnetised_speeds_are_boosted_sound_speeds(vd):
    rho, p = 1.3, 0.7
    cs = math.sqrt(cs2_ca2(rho, p, 0.0)[0])
    for d in range(3):
        v = [0.0, 0.0, 0.0]
        v[d] = vd
        lmin, lmax = O.speeds(opts(), state(rho, p, v), d)
        assert abs(lmax - (vd + cs) / (1 + vd * cs)) < 1e-14
        assert abs(lmin - (vd - cs) / (1 - vd * cs)) < 1e-14


@pytest.mark.parametrize("B", [0.2, 1.0, 5.0])
def test_rest_frame_fast_speed_across_and_along_the_field(B):
    rho, p = 1.0, 0.4
    cs2, ca2 = cs2_ca2(rho, p, B * B)
    # across: B along y, propagation along x
    lmin, lmax = O.speeds(opts(), state(rho, p, B=(0, B, 0)), 0)
    cf = math.sqrt(cs2 + ca2 - cs2 * ca2)
    assert abs(lmax - cf) < 1e-13 and abs(lmin + cf) < 1e-13
    # along: B along x
    lmin, lmax = O.speeds(opts(), state(rho, p, B=(B, 0, 0)), 0)
    cf = math.sqrt(max(cs2, ca2))
    assert abs(lmax - cf) < 1e-14 and abs(lmin + cf) < 1e-14
    # the isotropic bound is exact across the field, an overestimate along it
    _, lb = O.speeds(opts(False), state(rho, p, B=(B, 0, 0)), 0)
    assert lb >= cf - 1e-15


def test_boosted_parallel_fast_speed():
    """B, v and the direction all along x: the boost leaves B unchanged and
    the fast speed is the rest-frame max(c_s, c_a) added to v."""
    rho, p, B = 0.8, 0.5, 1.5
    cs2, ca2 = cs2_ca2(rho, p, B * B)
    c = math.sqrt(max(cs2, ca2))
    for v in (0.3, -0.7, 0.95):
        lmin, lmax = O.speeds(opts(), state(rho, p, (v, 0, 0), (B, 0, 0)), 0)
        assert abs(lmax - (v + c) / (1 + v * c)) < 1e-14
        assert abs(lmin - (v - c) / (1 - v * c)) < 1e-14


def test_general_states_against_the_root_scan_and_the_bound():
    rng = np.random.default_rng(19)
    lam = np.linspace(-1 + 1e-9, 1 - 1e-9, 40001)
    for trial in range(120):
        V = np.zeros(9)
        V[0] = 10 ** rng.uniform(-1, 1)
        V[4] = V[0] * 10 ** rng.uniform(-2, 1.5)
        lor = rng.uniform(1, 8)
        dv = rng.normal(size=3)
        V[1:4] = dv / np.linalg.norm(dv) * math.sqrt(1 - 1 / lor ** 2)
        w = V[0] + G * V[4] / (G - 1)
        db = rng.normal(size=3)
        V[5:8] = db / np.linalg.norm(db) * math.sqrt(rng.uniform(0, 1) * w)
        d = trial % 3
        lmin, lmax = O.speeds(opts(), V, d)
        bmin, bmax = O.speeds(opts(False), V, d)
        assert bmin <= lmin + 1e-14 and lmax <= bmax + 1e-14
        f = rmhd_quartic(lam, V, G, d)
        idx = np.nonzero(np.sign(f[:-1]) != np.sign(f[1:]))[0]
        roots = lam[idx]
        assert abs(lmax - roots.max()) < 1e-4 and abs(lmin - roots.min()) < 1e-4


def test_exact_speed_step_conserves():
    V, meta = I.rmhd3d_fields(n=12, ng=4, seed=4001, gmax_cap=3.0)
    o = O.make_opts(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", gamma=G, dx=meta["dx"],
                    exact_speeds=True)
    U = O.prim2cons(o, V)
    rate = O.cfl_rate(o, U, 4)
    rate_b = O.cfl_rate(O.make_opts(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", gamma=G,
                                    dx=meta["dx"]), U, 4)
    assert rate <= rate_b
    dt = 0.3 / rate
    ch = min(0.3 * meta["dx"][0] / dt, 1.0)
    Uo, r, _, fails = O.step(o, U, 4, dt, ch)
    assert fails == [0] * 5 and r > 0
    a = I.interior(U, 4, 3).reshape(9, -1)
    b = I.interior(Uo, 4, 3).reshape(9, -1)
    for q in range(8):
        assert abs(b[q].sum() - a[q].sum()) <= 50 * a.shape[1] * 2.2e-16 * np.abs(a[q]).max()
