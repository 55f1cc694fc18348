"""GPU parity of the AMR time-step and tagging kernels (Sec. 4) through the
C ABI: leaf masks, the refinement criterion (Eq. RefCrit), the next level
steps (Eq. Ca, Eq. dt_cool, Eq. level_dt) and the leaf-only cooling
time-step estimate of a step, against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import amr_time as AT
from paper_1110_0740_amd import ctu, inputs as I
from tests.gpu_common import DEV
from tests.test_gpu_amr_cycle import hierarchy, level_states, make_hier, pack

pytestmark = pytest.mark.gpu

NG = 4


def planes(Ul):
    """byte arrays per box in the layout of cool_L0 (state / 9)"""
    return [np.zeros(u.shape[1:], dtype=np.uint8) for u in Ul]


def unpack_planes(t, Ul):
    host = t.cpu().numpy()
    out, pos = [], 0
    for u in Ul:
        n = u[0].size
        out.append(host[pos:pos + n].reshape(u.shape[1:]))
        pos += n
    return out


def test_leaf_masks_match_oracle():
    h = hierarchy()
    U, offs = level_states(h)
    hier = make_hier(h, offs, "fp64")
    ref = AT.leaf_masks(h.levels, h.base, NG)
    for lev in range(len(h.levels)):
        n = sum(u[0].size for u in U[lev])
        leaf = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
        hier.leaf_mask(lev, leaf)
        torch.cuda.synchronize()
        for g, r in zip(unpack_planes(leaf, U[lev]), ref[lev]):
            assert np.array_equal(g, r)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tags_match_oracle(precision):
    h = hierarchy()
    U, offs = level_states(h)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    hier = make_hier(h, offs, precision)
    eps, chi_r = 0.01, 0.05
    total = 0
    for lev in range(len(h.levels)):
        Ud = pack(U[lev], dtype)
        n = sum(u[0].size for u in U[lev])
        tags = torch.zeros(n, dtype=torch.uint8, device=DEV)
        ntag = torch.zeros(1, dtype=torch.int32, device=DEV)
        hier.tag(lev, Ud, 0, eps, chi_r, tags, ntag)
        torch.cuda.synchronize()
        got = unpack_planes(tags, U[lev])
        cnt = 0
        for g, u in zip(got, U[lev]):
            # the decision is taken in FP64 on the stored (rounded) values on both sides
            sig = u[0].astype(np.float32).astype(np.float64) if precision == "fp32" else u[0]
            chi = AT.lohner_chi(sig, NG, eps)
            inner = g[NG:-NG, NG:-NG, NG:-NG]
            want = (chi > chi_r).astype(np.uint8)
            close = np.abs(chi - chi_r) < 1e-12
            assert np.array_equal(inner[~close], want[~close])
            cnt += int(inner.sum())
        assert ntag.item() == cnt
        total += cnt
    assert total > 0


def test_next_dt_matches_oracle():
    h = hierarchy()
    U, offs = level_states(h)
    hier = make_hier(h, offs, "fp64")
    rate = [12.5, 30.0, 47.0]
    dt_prev = [0.03, 0.015, 0.0075]
    for dpp in (None, [0.0, 0.01, 0.08]):
        params = [torch.tensor([dt_prev[l], 0.7], dtype=torch.float64, device=DEV) for l in range(3)]
        rd = torch.tensor(rate, dtype=torch.float64, device=DEV)
        dd = None if dpp is None else torch.tensor(dpp, dtype=torch.float64, device=DEV)
        hier.next_dt(rd, dd, 0.4, 0.02, params)
        torch.cuda.synchronize()
        want = AT.next_dt(rate, dpp, dt_prev, 0.4, 0.02)
        for l in range(3):
            got = params[l].cpu().numpy()
            assert got[0] == want[l] and got[1] == 0.7


# max |dp/p| (~4e-3 here) is a difference of nearly equal pressures: in FP32
# the pressure after the step carries ~2e-6 relative error, ~5e-4 of dp
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-3)])
def test_leaf_only_cooling_estimate_matches_oracle(precision, tol):
    n = 12
    V, meta = I.mhd3d_fields(n=n, ng=NG, seed=2003)
    G = meta["gamma"]
    oo = O.make_opts(dim=3, gamma=G, dx=meta["dx"], recon="ppm", riemann="hlld", cooling=True, cool_beta=0.5,
                     T_floor=0.01)
    U = O.prim2cons(oo, V)
    rng = np.random.default_rng(11)
    L0 = 0.5 + rng.random(V[0].shape)
    if precision == "fp32":
        L0 = L0.astype(np.float32).astype(np.float64)
    leaf = np.zeros(V[0].shape, dtype=np.uint8)
    leaf[:, :, : NG + n // 2] = 1   # the low-x half of the box counts
    dt, ch = 5e-3, 1.0
    _, _, dpp_ref, _ = O.step(oo, U, NG, dt, ch, L0=L0, leaf=leaf)
    _, _, dpp_all, _ = O.step(oo, U, NG, dt, ch, L0=L0)
    go = ctu.make_opts(dim=3, gamma=G, dx=meta["dx"], recon="ppm", riemann="hlld", cooling=True, cool_beta=0.5,
                       T_floor=0.01, precision=precision)
    plan = ctu.Plan(go, [((0, 0, 0), (n, n, n), 0, 0)], NG)
    dtype = torch.float64 if precision == "fp64" else torch.float32
    Ud = torch.from_numpy(U.reshape(-1)).to(dtype).to(DEV)
    Uo = torch.zeros_like(Ud)
    L0d = torch.from_numpy(L0.reshape(-1)).to(dtype).to(DEV)
    lf = torch.from_numpy(leaf.reshape(-1)).to(DEV)
    params = torch.tensor([dt, ch], dtype=torch.float64, device=DEV)
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    dpp = torch.zeros(1, dtype=torch.float64, device=DEV)
    plan.set_leaf_mask(lf)
    plan.step(Ud, Uo, params, rate, L0=L0d, dpp=dpp)
    torch.cuda.synchronize()
    got_leaf = dpp.item()
    plan.set_leaf_mask(None)
    plan.step(Ud, Uo, params, rate, L0=L0d, dpp=dpp)
    torch.cuda.synchronize()
    got_all = dpp.item()
    assert 0.0 < dpp_ref <= dpp_all
    assert abs(got_leaf - dpp_ref) <= tol * dpp_ref and abs(got_all - dpp_all) <= tol * dpp_all
