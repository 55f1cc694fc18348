"""GPU parity of relativistic MHD with the exact fast magnetosonic speeds
(the outermost roots of the dispersion quartic, in HLL / Rusanov and the
CFL rate) through the C ABI, against the oracle: the step under the ideal
and the Taub-Matthews EOS, FP64 and FP32, and the cell-centred CFL rate."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1110_0740_amd import ctu, inputs as I
from tests.gpu_common import DEV
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step

pytestmark = pytest.mark.gpu

KW = dict(physics="rmhd", recon="lin_mc", predictor="mh", exact_speeds=True)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_exact_speed_step_ideal(precision, tol):
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), riemann="hll", **KW)


def test_exact_speed_step_tm_rusanov():
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4004, gmax_cap=4.0)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), riemann="rusanov", eos="tm", **KW)


def test_exact_speed_cfl_rate():
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=6.0)
    kw = dict(dim=3, dx=meta["dx"], gamma=meta["gamma"], riemann="hll", **KW)
    oo = O.make_opts(**kw)
    U = O.prim2cons(oo, V)
    ref = O.cfl_rate(oo, U, 4)
    ref_bound = O.cfl_rate(O.make_opts(**dict(kw, exact_speeds=False)), U, 4)
    plan = ctu.Plan(ctu.make_opts(precision="fp64", **kw), [((0, 0, 0), (16, 16, 16), 0, 0)], 4)
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    plan.cfl_rate(torch.from_numpy(U.reshape(-1)).to(DEV), rate)
    torch.cuda.synchronize()
    assert abs(rate.item() - ref) <= 1e-13 * ref
    assert ref < ref_bound
