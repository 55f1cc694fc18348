"""Host-side geometry of a block-structured AMR level pair (Sec. 4): which
faces need flux registers and which coarse cells receive a reflux
correction (Eq. fluxcorr, Eq. addreflux), for refinement ratio 2 in 3D.

Pure index bookkeeping on the box lists; the arithmetic (register
accumulation and the correction itself) runs in libctu.  Outputs feed
``ctu.Plan(regfaces=...)`` and ``Plan.set_reflux``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LevelTables:
    regfaces: list = field(default_factory=list)   # (box, dir, face, (tlo0, tlo1), (tn0, tn1), slot)
    reflux: list = field(default_factory=list)     # (box, (i, j, k), dir, side, coarse_slot, [fine slots])


def _transverse(d):
    return [e for e in range(3) if e != d]


def build_tables(levels, base: int, ng: int):
    """levels[l] = list of boxes with .lo/.n in level-l indices (level 0 covers
    the periodic base^3 domain).  Returns (tables per level, total register
    slots).  Every box of level l >= 1 registers its six faces in full; each
    coarse box registers the rectangles of its faces that lie under a fine
    box face; one reflux entry is made per (coarse cell outside level l+1,
    face under level l+1)."""
    nlev = len(levels)
    tables = [LevelTables() for _ in range(nlev)]
    slot = 0
    fine_face = {}  # (level, box, dir, side) -> (slot base, tlo, tn)
    for lev in range(1, nlev):
        for b, B in enumerate(levels[lev]):
            for d in range(3):
                t = _transverse(d)
                tlo = (B.lo[t[0]], B.lo[t[1]])
                tn = (B.n[t[0]], B.n[t[1]])
                for side in (0, 1):
                    face = B.lo[d] + (B.n[d] if side else 0)
                    tables[lev].regfaces.append((b, d, face, tlo, tn, slot))
                    fine_face[(lev, b, d, side)] = (slot, tlo, tn)
                    slot += tn[0] * tn[1]
    for lev in range(1, nlev):
        Nc = base << (lev - 1)
        coarse = levels[lev - 1]
        owner = -np.ones((Nc, Nc, Nc), dtype=np.int32)  # [k, j, i] coarse box id
        for cb, C in enumerate(coarse):
            owner[C.lo[2]:C.lo[2] + C.n[2], C.lo[1]:C.lo[1] + C.n[1], C.lo[0]:C.lo[0] + C.n[0]] = cb
        covered = np.zeros((Nc, Nc, Nc), dtype=bool)
        for F in levels[lev]:
            covered[F.lo[2] // 2:(F.lo[2] + F.n[2]) // 2, F.lo[1] // 2:(F.lo[1] + F.n[1]) // 2,
                    F.lo[0] // 2:(F.lo[0] + F.n[0]) // 2] = True
        coarse_rect = {}  # (coarse box, dir, face, fine box, side) -> (slot base, tlo, tn)
        for fb, F in enumerate(levels[lev]):
            for d in range(3):
                t = _transverse(d)
                for side in (0, 1):
                    ff = F.lo[d] + (F.n[d] if side else 0)
                    fc = ff // 2
                    cd = fc - 1 if side == 0 else fc          # coarse cell outside the fine box
                    sgn = +1 if side == 0 else -1              # fine region on the cell's high / low side
                    t0r = range(F.lo[t[0]] // 2, (F.lo[t[0]] + F.n[t[0]]) // 2)
                    t1r = range(F.lo[t[1]] // 2, (F.lo[t[1]] + F.n[t[1]]) // 2)
                    fslot, ftlo, ftn = fine_face[(lev, fb, d, side)]
                    for a in t0r:
                        for c in t1r:
                            idx = [0, 0, 0]
                            idx[d], idx[t[0]], idx[t[1]] = cd, a, c
                            if covered[idx[2], idx[1], idx[0]]:
                                continue
                            cb = int(owner[idx[2], idx[1], idx[0]])
                            if cb < 0:
                                raise ValueError("coarse cell outside every coarse box")
                            C = coarse[cb]
                            key = (cb, d, fc, fb, side)
                            if key not in coarse_rect:
                                # faces of this coarse box under the fine box face
                                lo0 = max(F.lo[t[0]] // 2, C.lo[t[0]])
                                hi0 = min((F.lo[t[0]] + F.n[t[0]]) // 2, C.lo[t[0]] + C.n[t[0]])
                                lo1 = max(F.lo[t[1]] // 2, C.lo[t[1]])
                                hi1 = min((F.lo[t[1]] + F.n[t[1]]) // 2, C.lo[t[1]] + C.n[t[1]])
                                coarse_rect[key] = (slot, (lo0, lo1), (hi0 - lo0, hi1 - lo1))
                                tables[lev - 1].regfaces.append((cb, d, fc, (lo0, lo1), (hi0 - lo0, hi1 - lo1), slot))
                                slot += (hi0 - lo0) * (hi1 - lo1)
                            cslot0, ctlo, ctn = coarse_rect[key]
                            cslot = cslot0 + (c - ctlo[1]) * ctn[0] + (a - ctlo[0])
                            fsl = []
                            for db in (0, 1):
                                for da in (0, 1):
                                    u0 = 2 * a + da - ftlo[0]
                                    u1 = 2 * c + db - ftlo[1]
                                    fsl.append(fslot + u1 * ftn[0] + u0)
                            loc = (idx[0] - C.lo[0] + ng, idx[1] - C.lo[1] + ng, idx[2] - C.lo[2] + ng)
                            tables[lev - 1].reflux.append((cb, loc, d, sgn, cslot, fsl))
    return tables, slot
