"""Plain AMR level cycle for the oracle (Sec. 4): ghost filling, coarse-to-fine
prolongation (Eq. prolong) of time-interpolated coarse data (Eq. intalpha),
restriction (Eq. avgdown) and the recursive subcycled advance of a
refinement-ratio-2 hierarchy with refluxing (Eq. fluxcorr, Eq. addreflux).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Everything works on
whole numpy arrays of one level at a time, in FP64, with no tiling:

* the domain is the periodic cube of ``base`` level-0 cells per side; level l
  has ``base * 2**l`` cells per side; a box is (lo, n) in level-l indices and
  its state is a ghosted array [9, n2 + 2 ng, n1 + 2 ng, n0 + 2 ng];
* a ghost cell takes the value of the same-level box whose interior holds
  its periodic image; otherwise it is prolonged from the coarser level:
  U* = (1 - alpha) U(t) + alpha U(t + dt) on the parent cell and its six
  face neighbours (Eq. intalpha), slopes Delta_d = MC of the two one-sided
  differences (Eq. MClim with Eq. minmod), and U_fine = U*_parent + sum_d
  (x_fine - x_parent)_d / dx_coarse Delta_d (Eq. prolong; the offset is
  -1/4 or +1/4 for ratio 2).  Every coarse value must lie in a coarse box
  interior (proper nesting), else ValueError;
* restriction replaces each coarse cell covered by a fine box by the mean of
  its 8 children (Eq. avgdown with equal Cartesian volumes);
* the cycle advances level l by dt, then level l+1 twice by dt / 2 (ghosts
  at alpha = 0 and 1/2), restricts, and refluxes level l with the fine face
  fluxes summed over the two substeps.
"""
from __future__ import annotations

import numpy as np

from . import amr_reflux, prim2cons, step  # noqa: F401  (prim2cons re-exported for tests)


def minmod(a, b):
    """Eq. minmod: (sign a + sign b)/2 min(|a|, |b|)."""
    return 0.5 * (np.sign(a) + np.sign(b)) * np.minimum(np.abs(a), np.abs(b))


def mc_slope(dp, dm):
    """Eq. MClim: mm((dp + dm)/2, 2 mm(dm, dp))."""
    return minmod(0.5 * (dp + dm), 2.0 * minmod(dm, dp))


def owner_map(boxes, N):
    """Dense [N, N, N] (k, j, i) array of the box whose interior holds each
    cell of the level, -1 elsewhere."""
    own = -np.ones((N, N, N), dtype=np.int64)
    for b, B in enumerate(boxes):
        sl = tuple(slice(B.lo[q], B.lo[q] + B.n[q]) for q in (2, 1, 0))
        if np.any(own[sl] >= 0):
            raise ValueError("boxes of one level overlap")
        own[sl] = b
    return own


def gather(boxes, U, own, ng, gk, gj, gi):
    """Values [9, m] of level cells (global, already wrapped) from the box
    interiors; ValueError where no box holds a cell."""
    ob = own[gk, gj, gi]
    if np.any(ob < 0):
        raise ValueError("a needed coarse cell lies outside every coarse box (nesting)")
    out = np.empty((9, gk.size))
    for b in np.unique(ob):
        m = ob == b
        B = boxes[b]
        out[:, m] = U[b][:, gk[m] - B.lo[2] + ng, gj[m] - B.lo[1] + ng, gi[m] - B.lo[0] + ng]
    return out


def ghost_cells(B, ng):
    """Local (k, j, i) index arrays of the ghost cells of a box."""
    shape = (B.n[2] + 2 * ng, B.n[1] + 2 * ng, B.n[0] + 2 * ng)
    k, j, i = np.indices(shape)
    inner = ((i >= ng) & (i < ng + B.n[0]) & (j >= ng) & (j < ng + B.n[1]) & (k >= ng) & (k < ng + B.n[2]))
    g = ~inner
    return k[g], j[g], i[g]


def prolong(cboxes, Uc_old, Uc_new, alpha, Nc, ng, fk, fj, fi):
    """Eq. prolong on time-interpolated coarse data (Eq. intalpha) at fine
    cells (wrapped global level-(l+1) indices); returns [9, m]."""
    own = owner_map(cboxes, Nc)
    ck, cj, ci = fk // 2, fj // 2, fi // 2

    def coarse(dk, dj, di):
        k = (ck + dk) % Nc
        j = (cj + dj) % Nc
        i = (ci + di) % Nc
        a = gather(cboxes, Uc_old, own, ng, k, j, i)
        if alpha == 0.0:
            return a
        b = gather(cboxes, Uc_new, own, ng, k, j, i)
        return (1.0 - alpha) * a + alpha * b

    u0 = coarse(0, 0, 0)
    out = u0.copy()
    for d, f in ((0, fi), (1, fj), (2, fk)):
        e = [0, 0, 0]
        e[2 - d] = 1  # (dk, dj, di) of the unit step along d
        up = coarse(*e)
        dn = coarse(*[-x for x in e])
        slope = mc_slope(up - u0, u0 - dn)
        off = np.where(f % 2 == 0, -0.25, 0.25)
        out += off[None, :] * slope
    return out


def fill_ghosts(boxes, U, N, ng, coarse=None):
    """Fill the ghost cells of every box of one level in place.
    coarse = (cboxes, Uc_old, Uc_new, alpha) for levels >= 1, None on level 0
    (which must cover the periodic domain)."""
    own = owner_map(boxes, N)
    for b, B in enumerate(boxes):
        lk, lj, li = ghost_cells(B, ng)
        gk = (lk - ng + B.lo[2]) % N
        gj = (lj - ng + B.lo[1]) % N
        gi = (li - ng + B.lo[0]) % N
        ob = own[gk, gj, gi]
        same = ob >= 0
        if np.any(same):
            U[b][:, lk[same], lj[same], li[same]] = gather(boxes, U, own, ng, gk[same], gj[same], gi[same])
        rest = ~same
        if np.any(rest):
            if coarse is None:
                raise ValueError("level-0 ghost cell outside every box")
            cboxes, Uc_old, Uc_new, alpha = coarse
            U[b][:, lk[rest], lj[rest], li[rest]] = prolong(cboxes, Uc_old, Uc_new, alpha, N // 2, ng, gk[rest],
                                                            gj[rest], gi[rest])


def average_down(fboxes, Uf, cboxes, Uc, Nc, ng):
    """Eq. avgdown (ratio 2, equal volumes): every coarse cell under a fine
    box interior becomes the mean of its 8 children.  Uc is updated in place."""
    own = owner_map(cboxes, Nc)
    for F, u in zip(fboxes, Uf):
        inner = u[:, ng:ng + F.n[2], ng:ng + F.n[1], ng:ng + F.n[0]]
        avg = np.zeros((9, F.n[2] // 2, F.n[1] // 2, F.n[0] // 2))
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    avg += inner[:, a::2, b::2, c::2]
        avg /= 8.0
        k, j, i = np.indices(avg.shape[1:])
        gk = (k + F.lo[2] // 2).ravel()
        gj = (j + F.lo[1] // 2).ravel()
        gi = (i + F.lo[0] // 2).ravel()
        ob = own[gk, gj, gi]
        if np.any(ob < 0):
            raise ValueError("fine box outside the coarse level")
        flat = avg.reshape(9, -1)
        for cb in np.unique(ob):
            m = ob == cb
            C = cboxes[cb]
            Uc[cb][:, gk[m] - C.lo[2] + ng, gj[m] - C.lo[1] + ng, gi[m] - C.lo[0] + ng] = flat[:, m]


def cycle(levels, U, base, ng, opts_for_level, dt0, ch):
    """One level-0 step of the whole hierarchy with subcycling (ratio 2).
    U[l] = list of ghosted conserved states of level l (modified: the
    interiors hold the new states on return, ghosts the values used).
    opts_for_level(l) gives the oracle options (dx of level l).  Returns
    the list of per-level lists of states."""
    nlev = len(levels)
    U = [[u.copy() for u in L] for L in U]

    def advance(lev, dt, coarse):
        N = base << lev
        fill_ghosts(levels[lev], U[lev], N, ng, coarse)
        o = opts_for_level(lev)
        old = [u.copy() for u in U[lev]]
        faces = []
        for b, u in enumerate(U[lev]):
            un, _, _, _, f = step(o, u, ng, dt, ch, want_faces=True)
            U[lev][b] = un
            faces.append(f)
        if lev + 1 < nlev:
            acc = None
            for q in (0, 1):
                f_fine = advance(lev + 1, 0.5 * dt, (levels[lev], old, U[lev], 0.5 * q))
                acc = f_fine if acc is None else [a + g for a, g in zip(acc, f_fine)]
            average_down(levels[lev + 1], U[lev + 1], levels[lev], U[lev], N, ng)
            dxc = opts_for_level(lev).dx[0]
            dxf = opts_for_level(lev + 1).dx[0]
            U[lev] = amr_reflux.reflux(levels[lev], U[lev], faces, dxc, levels[lev + 1], acc, dxf, N, ng)
        return faces

    advance(0, dt0, None)
    return U


def totals(levels, U, base, ng):
    """Volume integrals of the 9 conserved variables over the composite
    grid: each level's cells not covered by the next finer level."""
    nlev = len(levels)
    tot = np.zeros(9)
    for lev in range(nlev):
        N = base << lev
        vol = (1.0 / N) ** 3
        cov = None
        if lev + 1 < nlev:
            cov = amr_reflux.covered_map(levels[lev + 1], N)
        for B, u in zip(levels[lev], U[lev]):
            inner = u[:, ng:ng + B.n[2], ng:ng + B.n[1], ng:ng + B.n[0]]
            if cov is not None:
                m = ~cov[B.lo[2]:B.lo[2] + B.n[2], B.lo[1]:B.lo[1] + B.n[1], B.lo[0]:B.lo[0] + B.n[0]]
                tot += (inner * m[None]).sum(axis=(1, 2, 3)) * vol
            else:
                tot += inner.sum(axis=(1, 2, 3)) * vol
    return tot
