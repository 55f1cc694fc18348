"""Median forms of the slope limiters (Sec. 3.2) and of the PPM constraints
(Eq. ppm_parabolic_lim), checked in FP32 on the CPU against their select
forms.  The FP32 kernels evaluate minmod(a, b) as med3(a, b, 0), the MC limiter
as med3((dp + dm)/2, 2 med3(dp, dm, 0), 0), PPM on half slopes with 1/3 in
place of 1/6, and the constraints as med3(P, -2M, 0) and med3(M, -2P, 0).
These tests pin the identities those rewrites rely on: equal values (== treats
the two zeros as equal) wherever the select form's sign product does not
underflow, and bit-equal PPM interface offsets from the half slopes."""
import numpy as np

F = np.float32


def med3(a, b, c):
    return np.maximum(np.minimum(a, b), np.minimum(np.maximum(a, b), c))


def minmod_sel(a, b):
    m = np.where(np.abs(a) < np.abs(b), a, b)
    return np.where(a * b > 0, m, F(0))


def mc_sel(dp, dm):
    c = F(0.5) * (dp + dm)
    m = np.minimum(np.minimum(np.abs(c), F(2) * np.abs(dp)), F(2) * np.abs(dm))
    return np.where(dp * dm > 0, np.copysign(m, c), F(0))


def mc_med(dp, dm):
    return med3(F(0.5) * (dp + dm), F(2) * med3(dp, dm, F(0)), F(0))


def mc_half(dp, dm):
    return med3(F(0.25) * (dp + dm), med3(dp, dm, F(0)), F(0))


def constraint_sel(P, M):
    keep = ~(P * M > 0)
    dp = np.where(np.abs(P) >= F(2) * np.abs(M), F(-2) * M, P)
    dm = np.where(np.abs(M) >= F(2) * np.abs(P), F(-2) * P, M)
    return np.where(keep, dp, F(0)), np.where(keep, dm, F(0))


def _samples(rng, n):
    """Mixed signs, magnitudes 1e-6..1e3 (no sign product underflows) and
    10 % exact zeros; the tests add ties of equal magnitude."""
    x = (rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(-6, 3, n)).astype(F)
    x[rng.random(n) < 0.1] = 0
    return x


def test_minmod_and_mc_medians_match_selects():
    rng = np.random.default_rng(31)
    a, b = _samples(rng, 200000), _samples(rng, 200000)
    b[:2000] = a[:2000]                      # equal arguments
    b[2000:4000] = -a[2000:4000]             # equal magnitudes, opposite signs
    assert np.array_equal(med3(a, b, F(0)), minmod_sel(a, b))
    assert np.array_equal(mc_med(a, b), mc_sel(a, b))
    # ties inside the MC minimum: |dp + dm| / 2 = 2 |dp|
    dp = _samples(rng, 5000)
    dm = F(3) * dp
    assert np.array_equal(mc_med(dp, dm), mc_sel(dp, dm))


def test_half_slopes_are_exact_halves():
    rng = np.random.default_rng(32)
    dp, dm = _samples(rng, 200000), _samples(rng, 200000)
    assert np.array_equal(F(2) * mc_half(dp, dm), mc_med(dp, dm))


def test_ppm_offsets_from_half_slopes_are_bit_equal():
    """w_+ - w_0 = d/2 - (s_+ - s_0)/6 from full slopes and d/2 - (h_+ - h_0)/3
    from half slopes h = s/2: the same FP32 bits (1/3 and 1/6 differ by a
    power of two in FP32 too)."""
    assert F(1.0 / 3.0) == F(2) * F(1.0 / 6.0)
    rng = np.random.default_rng(33)
    d = [_samples(rng, 100000) for _ in range(4)]
    s0, sp, sm = mc_sel(d[2], d[1]), mc_sel(d[3], d[2]), mc_sel(d[1], d[0])
    h0, hp, hm = mc_half(d[2], d[1]), mc_half(d[3], d[2]), mc_half(d[1], d[0])
    P6 = F(0.5) * d[2] - (sp - s0) * F(1.0 / 6.0)
    P3 = F(0.5) * d[2] - (hp - h0) * F(1.0 / 3.0)
    M6 = F(-0.5) * d[1] + (sm - s0) * F(1.0 / 6.0)
    M3 = F(-0.5) * d[1] + (hm - h0) * F(1.0 / 3.0)
    assert np.array_equal(P6.view(np.uint32), P3.view(np.uint32))
    assert np.array_equal(M6.view(np.uint32), M3.view(np.uint32))


def test_parabolic_constraint_medians_match_selects():
    rng = np.random.default_rng(34)
    P, M = _samples(rng, 200000), _samples(rng, 200000)
    M[:3000] = F(-0.5) * P[:3000]            # |P| = 2|M| exactly, opposite signs
    M[3000:6000] = F(0.5) * P[3000:6000]     # same signs
    dp_s, dm_s = constraint_sel(P, M)
    assert np.array_equal(med3(P, F(-2) * M, F(0)), dp_s)
    assert np.array_equal(med3(M, F(-2) * P, F(0)), dm_s)


def test_underflowing_sign_product_is_the_one_difference():
    """Where the sign product underflows to 0 the select form returns 0 and
    the median the exact smaller difference.  The FP32 kernels flush
    subnormal results to zero, so there this starts with differences below
    ~1e-19; numpy keeps subnormals, so the case here is below ~1e-23."""
    a, b = np.array([1e-25], F), np.array([3e-25], F)
    assert (a * b)[0] == 0
    assert minmod_sel(a, b)[0] == 0
    assert med3(a, b, F(0))[0] == a[0]
