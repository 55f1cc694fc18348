"""Plain refluxing of a coarse level from per-box face fluxes (Sec. 4,
Eq. fluxcorr and Eq. addreflux), for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Brute force: every
interior cell of every coarse box is visited; a face whose neighbour cell is
covered by the fine level while the cell itself is not receives
  U += -side * (sum over the r^2 fine faces of dt_f A_f (F - Pi)
                - dt_c A_c (F - Pi)) / V_c
with side = +1 when the fine cells lie on the cell's high face.  Face fluxes
come from ``oracle.step(..., want_faces=True)`` (dt * (F - Pi) per unit area).
"""
import numpy as np


def covered_map(fine_boxes, Nc):
    cov = np.zeros((Nc, Nc, Nc), dtype=bool)
    for F in fine_boxes:
        cov[F.lo[2] // 2:(F.lo[2] + F.n[2]) // 2, F.lo[1] // 2:(F.lo[1] + F.n[1]) // 2,
            F.lo[0] // 2:(F.lo[0] + F.n[0]) // 2] = True
    return cov


def fine_owner(fine_boxes, Nf):
    own = -np.ones((Nf, Nf, Nf), dtype=np.int64)
    for b, F in enumerate(fine_boxes):
        own[F.lo[2]:F.lo[2] + F.n[2], F.lo[1]:F.lo[1] + F.n[1], F.lo[0]:F.lo[0] + F.n[0]] = b
    return own


def reflux(coarse_boxes, U_coarse, faces_coarse, dx_c, fine_boxes, faces_fine, dx_f, Nc, ng):
    """Return corrected copies of the coarse boxes' states.
    U_coarse[b]: [9, NZ, NY, NX]; faces_*[b]: [3, 9, NZ, NY, NX]."""
    cov = covered_map(fine_boxes, Nc)
    own = fine_owner(fine_boxes, 2 * Nc)
    Vc = dx_c ** 3
    Ac, Af = dx_c ** 2, dx_f ** 2
    out = [u.copy() for u in U_coarse]
    for b, C in enumerate(coarse_boxes):
        for k in range(C.n[2]):
            for j in range(C.n[1]):
                for i in range(C.n[0]):
                    g = (C.lo[0] + i, C.lo[1] + j, C.lo[2] + k)
                    if cov[g[2], g[1], g[0]]:
                        continue
                    loc = (i + ng, j + ng, k + ng)
                    for d in range(3):
                        for side in (+1, -1):
                            nb = list(g)
                            nb[d] += side
                            if not (0 <= nb[d] < Nc) or not cov[nb[2], nb[1], nb[0]]:
                                continue
                            # coarse face: the cell's high face (stored at loc + e_d) or low face (at loc)
                            cl = list(loc)
                            if side == +1:
                                cl[d] += 1
                            fc = faces_coarse[b][d][:, cl[2], cl[1], cl[0]] * Ac
                            # fine faces on the same plane, 2 x 2 of them
                            plane = 2 * (g[d] + (1 if side == +1 else 0))
                            t = [e for e in range(3) if e != d]
                            fsum = np.zeros(9)
                            for a in (0, 1):
                                for c in (0, 1):
                                    fcell = [0, 0, 0]
                                    fcell[d] = plane if side == +1 else plane - 1
                                    fcell[t[0]] = 2 * g[t[0]] + a
                                    fcell[t[1]] = 2 * g[t[1]] + c
                                    fb = own[fcell[2], fcell[1], fcell[0]]
                                    F = fine_boxes[fb]
                                    fl = [fcell[q] - F.lo[q] + ng for q in range(3)]
                                    fl[d] = plane - F.lo[d] + ng
                                    fsum += faces_fine[fb][d][:, fl[2], fl[1], fl[0]] * Af
                            out[b][:, loc[2], loc[1], loc[0]] += -side * (fsum - fc) / Vc
    return out
