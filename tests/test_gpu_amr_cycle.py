"""GPU parity of the AMR level cycle (Sec. 4) through the C ABI: ghost
filling (same-level periodic copy, Eq. prolong on Eq. intalpha data),
restriction (Eq. avgdown) and the subcycled, refluxed level-0 step of a
3-level hierarchy, against the oracle's plain numpy implementation; and
conservation of the GPU cycle itself."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import amr_cycle as AC
from paper_1110_0740_amd import amr, ctu, inputs as I
from tests.gpu_common import DEV, assert_parity

pytestmark = pytest.mark.gpu

NG = 4
GAMMA = 5.0 / 3.0
# ghost widths: 4, and 3 (the PPM stencil's minimum, which the AMR benchmark runs)
NGS = [3, 4]


def hierarchy():
    return I.amr_hierarchy(seed=3001, base=32, base_box=16, lattice=16, size_range=(8, 16), p1=(0.5, 1.0),
                           p2=(0.5, 1.0), nest=3)


def level_states(h, perturb=0.0, seed=0, ng=NG):
    """conserved ghosted states per level (FP64 numpy) and element offsets"""
    rng = np.random.default_rng(seed)
    U, offs = [], []
    for lev, L in enumerate(h.levels):
        o = O.make_opts(dim=3, gamma=GAMMA, dx=h.dx(lev))
        Ul, ol, pos = [], [], 0
        for B in L:
            V = I.amr_fields(h, B, ng)
            if perturb:
                V = V * (1.0 + perturb * rng.standard_normal(V.shape))
            u = O.prim2cons(o, V)
            Ul.append(u)
            ol.append(pos)
            pos += u.size
        U.append(Ul)
        offs.append(ol)
    return U, offs


def pack(Ul, dtype):
    return torch.from_numpy(np.concatenate([u.reshape(-1) for u in Ul])).to(dtype).to(DEV)


def unpack(t, Ul):
    host = t.cpu().numpy().astype(np.float64)
    out, pos = [], 0
    for u in Ul:
        out.append(host[pos:pos + u.size].reshape(u.shape))
        pos += u.size
    return out


def make_hier(h, offs, precision, ng=NG):
    levels = [[(B.lo, B.n, off) for B, off in zip(L, offs[lev])] for lev, L in enumerate(h.levels)]
    return ctu.Hier(precision, h.base, levels, ng)


@pytest.mark.parametrize("ng", NGS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ghost_fill_matches_oracle(precision, ng):
    h = hierarchy()
    U, offs = level_states(h, ng=ng)
    U2, _ = level_states(h, perturb=0.05, seed=1, ng=ng)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    hier = make_hier(h, offs, precision, ng)
    missing = torch.zeros(1, dtype=torch.int32, device=DEV)
    for lev in range(len(h.levels)):
        N = h.base << lev
        for alpha in ((0.0,) if lev == 0 else (0.0, 0.5)):
            ref = [u.copy() for u in U[lev]]
            coarse = None if lev == 0 else (h.levels[lev - 1], U[lev - 1], U2[lev - 1], alpha)
            AC.fill_ghosts(h.levels[lev], ref, N, ng, coarse)
            Ud = pack(U[lev], dtype)
            if lev == 0:
                hier.fill_ghosts(0, Ud, missing=missing)
            else:
                hier.fill_ghosts(lev, Ud, pack(U[lev - 1], dtype), pack(U2[lev - 1], dtype), alpha, missing=missing)
            torch.cuda.synchronize()
            got = unpack(Ud, U[lev])
            for b, (g, r) in enumerate(zip(got, ref)):
                scale = np.abs(r).max()
                err = np.abs(g - r).max() / scale
                # FP32: inputs rounded to 2^-24 relative, a prolonged value adds
                # three quarter-slopes of rounded differences and ~6 roundings:
                # below ~16 half-ulps of the box's largest value
                if precision == "fp64":
                    assert err <= 1e-14, (lev, alpha, b, err)
                else:
                    assert err <= 1e-6, (lev, alpha, b, err)
    assert missing.item() == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_average_down_matches_oracle(precision):
    h = hierarchy()
    U, offs = level_states(h, perturb=0.02, seed=3)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    hier = make_hier(h, offs, precision)
    for fine in range(1, len(h.levels)):
        ref = [u.copy() for u in U[fine - 1]]
        AC.average_down(h.levels[fine], U[fine], h.levels[fine - 1], ref, h.base << (fine - 1), NG)
        Uc = pack(U[fine - 1], dtype)
        hier.average_down(fine, pack(U[fine], dtype), Uc)
        torch.cuda.synchronize()
        got = unpack(Uc, U[fine - 1])
        for g, r in zip(got, ref):
            if precision == "fp64":
                assert np.array_equal(g, r)  # same summation order, exact division by 8
            else:
                assert np.abs(g - r).max() <= 2e-7 * np.abs(r).max()


def run_gpu_cycle(h, U, offs, precision, dt0, ch, ncycles=1, ng=NG):
    dtype = torch.float64 if precision == "fp64" else torch.float32
    nlev = len(h.levels)
    tables, nslots = amr.build_tables(h.levels, h.base, ng)
    plans = []
    for lev, L in enumerate(h.levels):
        go = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=GAMMA, dx=h.dx(0), precision=precision)
        p = ctu.Plan(go, [(B.lo, B.n, lev, off) for B, off in zip(L, offs[lev])], ng, regfaces=tables[lev].regfaces)
        if tables[lev].reflux:
            p.set_reflux(tables[lev].reflux)
        plans.append(p)
    hier = make_hier(h, offs, precision, ng)
    Ua = [pack(U[lev], dtype) for lev in range(nlev)]
    Ub = [torch.zeros_like(t) for t in Ua]
    cur = [0] * nlev
    params = [torch.tensor([dt0 / (1 << lev), ch], dtype=torch.float64, device=DEV) for lev in range(nlev)]
    reg = torch.zeros(9 * max(1, nslots), dtype=torch.float64, device=DEV)
    rate = torch.zeros(nlev, dtype=torch.float64, device=DEV)
    fails = torch.zeros(5, dtype=torch.int32, device=DEV)
    missing = torch.zeros(1, dtype=torch.int32, device=DEV)
    for _ in range(ncycles):
        hier.advance(plans, Ua, Ub, cur, params, reg, rate, fails=fails, missing=missing)
    torch.cuda.synchronize()
    out = [unpack(Ub[lev] if cur[lev] else Ua[lev], U[lev]) for lev in range(nlev)]
    return out, fails.cpu().tolist(), int(missing.item()), reg


def oracle_opts(h):
    return lambda lev: O.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=GAMMA, dx=h.dx(lev))


@pytest.mark.parametrize("ng", NGS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_subcycled_cycle_matches_oracle(precision, tol, ng):
    h = hierarchy()
    U, offs = level_states(h, ng=ng)
    dt0 = 0.2 / h.base
    ch = 0.4 * h.dx(0)[0] / dt0 * 0.5
    ref = AC.cycle(h.levels, U, h.base, ng, oracle_opts(h), dt0, ch)
    got, fails, missing, reg = run_gpu_cycle(h, U, offs, precision, dt0, ch, ng=ng)
    assert fails == [0] * 5 and missing == 0
    for lev in range(len(h.levels)):
        for b in range(len(h.levels[lev])):
            assert_parity(got[lev][b], ref[lev][b], ng, 3, ch, tol, what=(lev, b))


@pytest.mark.parametrize("ng", NGS)
def test_gpu_cycle_conserves_and_consumes_registers(ng):
    """FP64, two cycles: the composite totals of every conserved variable but
    psi are unchanged to round-off, and the registers the refluxes read are
    cleared after each use."""
    h = hierarchy()
    U, offs = level_states(h, ng=ng)
    dt0 = 0.2 / h.base
    ch = 0.4 * h.dx(0)[0] / dt0 * 0.5
    before = AC.totals(h.levels, U, h.base, ng)
    got, fails, missing, reg = run_gpu_cycle(h, U, offs, "fp64", dt0, ch, ncycles=2, ng=ng)
    after = AC.totals(h.levels, got, h.base, ng)
    scale = np.abs(before).max()
    assert np.max(np.abs(after[:8] - before[:8])) <= 2e-13 * scale, after - before
    tables, _ = amr.build_tables(h.levels, h.base, ng)
    r = reg.cpu().numpy().reshape(-1, 9)
    read = sorted({s for T in tables for e in T.reflux for s in [e[4]] + list(e[5])})
    assert np.all(r[read] == 0.0)
