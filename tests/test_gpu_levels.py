"""One plan over every level of a hierarchy (CTU_PLAN_LEVEL_DT, Sec. 4 with
ratio 2): a level-l box steps by dt / 2^l inside a single launch chain.
Against one plan per level with params dt / 2^l: bitwise the same states and
flux registers, the rate equal to max_l rate_l / 2^l, and one reflux table
over the combined plan (box indices shifted by level) equal to the per-level
refluxes; the combined step also matches the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1110_0740_amd import amr, ctu, inputs as I
from tests.gpu_common import DEV, assert_parity

pytestmark = pytest.mark.gpu

NG = 4
GAMMA = 5.0 / 3.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_multilevel_plan_equals_per_level_plans(precision):
    h = I.amr_hierarchy(seed=3001, base=32, base_box=16, lattice=16, size_range=(8, 16), p1=(0.5, 1.0),
                        p2=(0.5, 1.0))
    nlev = len(h.levels)
    tables, nslots = amr.build_tables(h.levels, h.base, NG)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    okw = dict(recon="ppm", riemann="hlld")
    dt0 = 2e-3
    ch = 0.4 * h.dx(0)[0] / dt0 * 0.5
    # states of every level, packed into one array for the combined plan
    Us, offs, base_box = [], [], []
    o = 0
    for lev, L in enumerate(h.levels):
        base_box.append(sum(len(x) for x in h.levels[:lev]))
        oo = O.make_opts(dim=3, gamma=GAMMA, dx=h.dx(lev), **okw)
        for B in L:
            u = O.prim2cons(oo, I.amr_fields(h, B, NG))
            Us.append((lev, B, u))
            offs.append(o)
            o += u.size
    Uall = torch.from_numpy(np.concatenate([u.reshape(-1) for _, _, u in Us])).to(dtype).to(DEV)
    go = ctu.make_opts(dim=3, gamma=GAMMA, dx=h.dx(0), precision=precision, **okw)
    # per-level plans over slices of the same array (offsets into it)
    ref_out = torch.zeros_like(Uall)
    reg_ref = torch.zeros(9 * nslots, dtype=torch.float64, device=DEV)
    rates = []
    fails = torch.zeros(5, dtype=torch.int32, device=DEV)
    per_plans = []
    k = 0
    for lev, L in enumerate(h.levels):
        boxes = [(B.lo, B.n, lev, offs[k + q]) for q, B in enumerate(L)]
        k += len(L)
        p = ctu.Plan(go, boxes, NG, regfaces=tables[lev].regfaces,
                     reflux=[(cb, loc, d, sg, cs, fs) for (cb, loc, d, sg, cs, fs) in tables[lev].reflux] or None)
        per_plans.append(p)
        rate = torch.zeros(1, dtype=torch.float64, device=DEV)
        params = torch.tensor([dt0 / (1 << lev), ch], dtype=torch.float64, device=DEV)
        p.step(Uall, ref_out, params, rate, reg=reg_ref, fails=fails)
        torch.cuda.synchronize()
        rates.append(rate.item())
    assert fails.sum().item() == 0
    # one plan over every level
    all_boxes = [(B.lo, B.n, lev, offs[q]) for q, (lev, B, _) in enumerate(Us)]
    regs = [(base_box[lev] + b, d, f, tlo, tn, sl) for lev in range(nlev)
            for (b, d, f, tlo, tn, sl) in tables[lev].regfaces]
    refl = [(base_box[lev] + cb, loc, d, sg, cs, fs) for lev in range(nlev)
            for (cb, loc, d, sg, cs, fs) in tables[lev].reflux]
    comb = ctu.Plan(go, all_boxes, NG, regfaces=regs, reflux=refl, level_dt=True)
    out = torch.zeros_like(Uall)
    reg = torch.zeros(9 * nslots, dtype=torch.float64, device=DEV)
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    params = torch.tensor([dt0, ch], dtype=torch.float64, device=DEV)
    comb.step(Uall, out, params, rate, reg=reg, fails=fails)
    torch.cuda.synchronize()
    assert fails.sum().item() == 0
    assert torch.equal(out, ref_out)
    assert torch.equal(reg, reg_ref)
    assert rate.item() == max(r / (1 << lev) for lev, r in enumerate(rates))
    # the combined plan against the oracle, box by box
    host = out.cpu().numpy().astype(np.float64)
    tol = 1e-12 if precision == "fp64" else 2e-6
    for q, (lev, B, u) in enumerate(Us[::7]):
        qq = q * 7
        oo = O.make_opts(dim=3, gamma=GAMMA, dx=h.dx(lev), **okw)
        ref, _, _, f = O.step(oo, u, NG, dt0 / (1 << lev), ch)
        got = host[offs[qq]:offs[qq] + u.size].reshape(u.shape)
        assert_parity(got, ref, NG, 3, ch, tol, what=(lev, qq))
    # reflux: the combined table against the per-level tables
    a, b = out.clone(), ref_out.clone()
    comb.reflux(a, reg)
    for lev in range(nlev - 1):
        per_plans[lev].reflux(b, reg_ref)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and not torch.equal(a, out)
