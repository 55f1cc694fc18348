"""GPU parity of relativistic MHD with the Taub-Matthews equation of state
(Sec. 2.2, Eq. TMEos) through the C ABI, against the oracle: the CTU step
(MUSCL-Hancock, HLL and Rusanov, FP64 and FP32 with the FP64 inversion),
the primitive <-> conserved maps over Lorentz factors up to 10, and the CFL
rate."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1110_0740_amd import ctu, inputs as I
from tests.gpu_common import DEV
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step

pytestmark = pytest.mark.gpu

KW = dict(physics="rmhd", recon="lin_mc", predictor="mh", eos="tm")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_tm_step_hll(precision, tol):
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), riemann="hll", **KW)


def test_tm_step_rusanov():
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4004, gmax_cap=4.0)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), riemann="rusanov", **KW)


def random_states(n, seed):
    rng = np.random.default_rng(seed)
    V = np.zeros((9, n))
    V[0] = 10 ** rng.uniform(-1, 1, n)
    V[4] = V[0] * 10 ** rng.uniform(-3, 2, n)
    lor = rng.uniform(1.0, 10.0, n)
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    V[1:4] = d * np.sqrt(1 - 1 / lor ** 2)
    w = 2.5 * V[4] + np.sqrt(2.25 * V[4] ** 2 + V[0] ** 2)
    b = rng.normal(size=(3, n))
    b /= np.linalg.norm(b, axis=0)
    V[5:8] = b * np.sqrt(rng.uniform(0, 1, n) * w)
    return V, w * lor ** 2


def test_tm_maps_and_cfl_rate_match_oracle():
    m = 8
    n = m ** 3
    Vf, W = random_states(n, 21)
    oo = O.make_opts(dim=3, dx=(0.1, 0.1, 0.1), riemann="hll", **KW)
    go = ctu.make_opts(dim=3, dx=(0.1, 0.1, 0.1), riemann="hll", precision="fp64", **KW)
    # one box of (m - 2 ng)^3 interior cells holding the m^3 states (ghosts included)
    plan = ctu.Plan(go, [((0, 0, 0), (m - 6, m - 6, m - 6), 0, 0)], 3)
    Vd = torch.from_numpy(Vf.reshape(-1).copy()).to(DEV)
    Ud = torch.zeros_like(Vd)
    plan.prim_to_cons(Vd, Ud)
    torch.cuda.synchronize()
    Uref = O.prim2cons(oo, Vf)
    Ug = Ud.cpu().numpy().reshape(9, n)
    assert np.max(np.abs(Ug - Uref) / (np.abs(Uref) + W)) < 1e-14
    V2 = torch.zeros_like(Vd)
    fails = torch.zeros(5, dtype=torch.int32, device=DEV)
    plan.cons_to_prim(Ud, V2, fails)
    torch.cuda.synchronize()
    assert fails.cpu().tolist() == [0] * 5
    Vg = V2.cpu().numpy().reshape(9, n)
    assert np.max(np.abs(Vg[0] - Vf[0]) / Vf[0]) < 1e-12
    assert np.max(np.abs(Vg[1:4] - Vf[1:4])) < 1e-12
    assert np.max(np.abs(Vg[4] - Vf[4]) / W) < 1e-13
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    plan.cfl_rate(Ud, rate)
    torch.cuda.synchronize()
    rref = O.cfl_rate(oo, Uref.reshape(9, m, m, m), 3)
    assert abs(rate.item() - rref) <= 1e-13 * rref
