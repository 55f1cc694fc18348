"""Plain AMR refinement criterion and level time steps for the oracle
(Sec. 4): the second-derivative error norm of Eq. RefCrit, the leaf (not
refined) cells of a level, and the next base-level step from Eq. Ca,
Eq. dt_cool and Eq. level_dt.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from .amr_reflux import covered_map


def lohner_chi(sigma: np.ndarray, ng: int, eps: float = 0.01) -> np.ndarray:
    """Eq. RefCrit on the interior of a ghosted [NZ, NY, NX] array of sigma:
    chi = sqrt( sum_d |D+ - D-|^2 / sum_d (|D+| + |D-| + eps sigma_ref,d)^2 )
    with the undivided differences D+ = s_{+1} - s_0, D- = s_0 - s_{-1} and
    sigma_ref,d = |s_{+1}| + 2|s_0| + |s_{-1}| along d.  chi = 0 where the
    denominator vanishes (sigma = 0 around the cell)."""
    NZ, NY, NX = sigma.shape
    c = (slice(ng, NZ - ng), slice(ng, NY - ng), slice(ng, NX - ng))
    s0 = sigma[c]
    num = np.zeros_like(s0)
    den = np.zeros_like(s0)
    for axis in range(3):
        up = [slice(ng, NZ - ng), slice(ng, NY - ng), slice(ng, NX - ng)]
        dn = list(up)
        up[axis] = slice(up[axis].start + 1, up[axis].stop + 1)
        dn[axis] = slice(dn[axis].start - 1, dn[axis].stop - 1)
        sp, sm = sigma[tuple(up)], sigma[tuple(dn)]
        dp, dm = sp - s0, s0 - sm
        num += (dp - dm) ** 2
        ref = np.abs(sp) + 2.0 * np.abs(s0) + np.abs(sm)
        den += (np.abs(dp) + np.abs(dm) + eps * ref) ** 2
    out = np.zeros_like(s0)
    m = den > 0.0
    out[m] = np.sqrt(num[m] / den[m])
    return out


def leaf_masks(levels, base: int, ng: int):
    """Per level, per box: ghosted [NZ, NY, NX] uint8 masks, 1 on interior
    cells not covered by the next finer level, 0 elsewhere."""
    out = []
    for lev, L in enumerate(levels):
        N = base << lev
        cov = covered_map(levels[lev + 1], N) if lev + 1 < len(levels) else np.zeros((N, N, N), dtype=bool)
        ms = []
        for B in L:
            m = np.zeros((B.n[2] + 2 * ng, B.n[1] + 2 * ng, B.n[0] + 2 * ng), dtype=np.uint8)
            sub = cov[B.lo[2]:B.lo[2] + B.n[2], B.lo[1]:B.lo[1] + B.n[1], B.lo[0]:B.lo[0] + B.n[0]]
            m[ng:ng + B.n[2], ng:ng + B.n[1], ng:ng + B.n[0]] = ~sub
            ms.append(m)
        out.append(ms)
    return out


def next_dt(rate, dpp, dt_prev, cfl: float, eps_c: float):
    """Next step of every level: dt_l = min(C_a / rate_l, eps_c dt_l^n /
    dpp_l) (Eq. Ca, Eq. dt_cool; the cooling term only where dpp_l > 0),
    dt0 = min_l 2^l dt_l (Eq. level_dt), and level l takes dt0 / 2^l."""
    nlev = len(rate)
    cand = []
    for l in range(nlev):
        d = cfl / rate[l]
        if dpp is not None and dpp[l] > 0.0:
            d = min(d, eps_c * dt_prev[l] / dpp[l])
        cand.append(d * (1 << l))
    dt0 = min(cand)
    return [dt0 / (1 << l) for l in range(nlev)]
