"""Host logic of the AMR tables: the reflux entries of amr.build_tables are
exactly the coarse-fine faces found by a brute-force scan, and the register
slots they name are consistent with the register rectangles."""
import numpy as np

from paper_1110_0740_amd import amr, inputs as I

NG = 4


def brute_force_faces(h, lev):
    Nc = h.base << lev
    cov = np.zeros((Nc,) * 3, dtype=bool)
    for F in h.levels[lev + 1]:
        cov[F.lo[2] // 2:(F.lo[2] + F.n[2]) // 2, F.lo[1] // 2:(F.lo[1] + F.n[1]) // 2,
            F.lo[0] // 2:(F.lo[0] + F.n[0]) // 2] = True
    out = set()
    for b, C in enumerate(h.levels[lev]):
        for k in range(C.n[2]):
            for j in range(C.n[1]):
                for i in range(C.n[0]):
                    g = (C.lo[0] + i, C.lo[1] + j, C.lo[2] + k)
                    if cov[g[2], g[1], g[0]]:
                        continue
                    for d in range(3):
                        for side in (1, -1):
                            nb = list(g)
                            nb[d] += side
                            if 0 <= nb[d] < Nc and cov[nb[2], nb[1], nb[0]]:
                                out.add((b, (i + NG, j + NG, k + NG), d, side))
    return out


def test_reflux_entries_match_brute_force():
    h = I.amr_hierarchy(seed=3001, base=32, base_box=16, lattice=16, size_range=(8, 16), p1=(0.5, 1.0), p2=(0.5, 1.0))
    tables, nslots = amr.build_tables(h.levels, h.base, NG)
    for lev in range(len(h.levels) - 1):
        got = {(e[0], tuple(e[1]), e[2], e[3]) for e in tables[lev].reflux}
        assert len(got) == len(tables[lev].reflux)
        assert got == brute_force_faces(h, lev)
    # every slot named by a reflux entry lies inside the rectangle of its box / direction
    rects = {}
    for lev, T in enumerate(tables):
        for (b, d, face, tlo, tn, slot) in T.regfaces:
            rects.setdefault(lev, []).append((b, d, slot, slot + tn[0] * tn[1]))
    for lev, T in enumerate(tables):
        for (b, loc, d, side, cs, fs) in T.reflux:
            assert any(rb == b and rd == d and s0 <= cs < s1 for (rb, rd, s0, s1) in rects[lev])
            assert len(fs) == 4 and len(set(fs)) == 4
            assert all(any(rd == d and s0 <= f < s1 for (rb, rd, s0, s1) in rects[lev + 1]) for f in fs)
    assert max(s1 for r in rects.values() for (_, _, _, s1) in r) == nslots


def test_workload_hierarchy_is_disjoint_and_nested():
    h = I.amr_hierarchy()
    for lev in (1, 2):
        N = h.base << lev
        occ = np.zeros((N,) * 3, dtype=np.int32)
        for B in h.levels[lev]:
            occ[B.lo[2]:B.lo[2] + B.n[2], B.lo[1]:B.lo[1] + B.n[1], B.lo[0]:B.lo[0] + B.n[0]] += 1
            assert all(B.lo[q] % 2 == 0 and B.n[q] % 2 == 0 and 16 <= B.n[q] <= 32 for q in range(3))
        assert occ.max() == 1
    # each level-2 box inside one level-1 box shrunk by one level-1 cell
    for B in h.levels[2]:
        assert any(all(2 * P.lo[q] + 2 <= B.lo[q] and B.lo[q] + B.n[q] <= 2 * (P.lo[q] + P.n[q]) - 2 for q in range(3))
                   for P in h.levels[1])
    assert 1200 <= sum(len(L) for L in h.levels) <= 1800
