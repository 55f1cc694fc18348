"""GPU parity of the batched AMR step: every patch of every level advanced
by one launch chain per level, FP64 flux registers on the coarse-fine
faces, and refluxing (Eq. fluxcorr, Eq. addreflux) against the oracle's
per-box steps and its brute-force reflux."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import amr_reflux
from paper_1110_0740_amd import amr, ctu, inputs as I
from tests.gpu_common import DEV, assert_parity

pytestmark = pytest.mark.gpu

NG = 4
GAMMA = 5.0 / 3.0


def small_hierarchy():
    return I.amr_hierarchy(seed=3001, base=32, base_box=16, lattice=16, size_range=(8, 16), p1=(0.5, 1.0),
                           p2=(0.5, 1.0))


def level_arrays(h, lev):
    Vs = [I.amr_fields(h, B, NG) for B in h.levels[lev]]
    offs, o = [], 0
    for V in Vs:
        offs.append(o)
        o += V.size
    return Vs, offs, o


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_amr_batch_step_registers_and_reflux(precision):
    h = small_hierarchy()
    nlev = len(h.levels)
    assert all(len(L) > 0 for L in h.levels)
    tables, nslots = amr.build_tables(h.levels, h.base, NG)
    assert any(len(T.reflux) for T in tables)
    dt0 = 2e-3
    ch = 0.4 * h.dx(0)[0] / dt0 * 0.5
    dtype = torch.float64 if precision == "fp64" else torch.float32
    reg = torch.zeros(9 * nslots, dtype=torch.float64, device=DEV)
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    fails = torch.zeros(5, dtype=torch.int32, device=DEV)
    ref_U, ref_F, got_U, plans, states = [], [], [], [], []
    for lev in range(nlev):
        dt = dt0 / (1 << lev)
        dx = h.dx(lev)
        oo = O.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=GAMMA, dx=dx)
        Vs, offs, total = level_arrays(h, lev)
        Us = [O.prim2cons(oo, V) for V in Vs]
        outs = [O.step(oo, U, NG, dt, ch, want_faces=True) for U in Us]
        ref_U.append([r[0] for r in outs])
        ref_F.append([r[4] for r in outs])
        go = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=GAMMA, dx=h.dx(0), precision=precision)
        boxes = [(B.lo, B.n, lev, off) for B, off in zip(h.levels[lev], offs)]
        plan = ctu.Plan(go, boxes, NG, regfaces=tables[lev].regfaces)
        Uin = torch.from_numpy(np.concatenate([U.reshape(-1) for U in Us])).to(dtype).to(DEV)
        Uout = Uin.clone()
        params = torch.tensor([dt, ch], dtype=torch.float64, device=DEV)
        plan.step(Uin, Uout, params, rate, reg=reg, fails=fails)
        torch.cuda.synchronize()
        assert fails.sum().item() == 0
        plans.append(plan)
        states.append((Uout, offs, [U.shape for U in Us]))
        host = Uout.cpu().numpy().astype(np.float64)
        got_U.append([host[o:o + int(np.prod(s))].reshape(s) for o, s in zip(offs, [U.shape for U in Us])])
    tol = 1e-12 if precision == "fp64" else 2e-6
    # 1. every patch of every level
    for lev in range(nlev):
        for b in range(len(h.levels[lev])):
            assert_parity(got_U[lev][b], ref_U[lev][b], NG, 3, ch, tol, what=(lev, b))
    # 2. registers: dt * A * (F - Pi) of the oracle's faces
    regh = reg.cpu().numpy().reshape(-1, 9)
    worst = 0.0
    for lev in range(nlev):
        A = h.dx(lev)[0] ** 2
        for (b, d, face, tlo, tn, slot) in tables[lev].regfaces:
            B = h.levels[lev][b]
            t = [e for e in range(3) if e != d]
            for u1 in range(tn[1]):
                for u0 in range(tn[0]):
                    idx = [0, 0, 0]
                    idx[d] = face - B.lo[d] + NG
                    idx[t[0]] = tlo[0] + u0 - B.lo[t[0]] + NG
                    idx[t[1]] = tlo[1] + u1 - B.lo[t[1]] + NG
                    want = ref_F[lev][b][d][:, idx[2], idx[1], idx[0]] * A
                    got = regh[slot + u1 * tn[0] + u0]
                    scale = np.abs(want).max() + 1e-300
                    worst = max(worst, np.abs(got - want).max() / scale)
    assert worst <= (1e-12 if precision == "fp64" else 5e-5), worst
    # 3. reflux of each coarse level against the brute-force oracle reflux
    for lev in range(nlev - 1):
        Nc = h.base << lev
        want = amr_reflux.reflux(h.levels[lev], ref_U[lev], ref_F[lev], h.dx(lev)[0], h.levels[lev + 1],
                                 ref_F[lev + 1], h.dx(lev + 1)[0], Nc, NG)
        plans[lev].set_reflux(tables[lev].reflux)
        Uout, offs, shapes = states[lev]
        plans[lev].reflux(Uout, reg)
        torch.cuda.synchronize()
        host = Uout.cpu().numpy().astype(np.float64)
        for b, (o, s) in enumerate(zip(offs, shapes)):
            g = host[o:o + int(np.prod(s))].reshape(s)
            assert_parity(g, want[b], NG, 3, ch, tol * 5, what=(lev, b))
            # the correction is not zero where the box touches the fine level
            moved = np.abs(I.interior(want[b], NG, 3) - I.interior(ref_U[lev][b], NG, 3)).max()
            if any(ent[0] == b for ent in tables[lev].reflux):
                assert moved > 0
