"""GPU parity of the HLLD solver for relativistic MHD (Mignone, Ugliano &
Bodo 2009: closed-form fast-wave states, secant iteration on the total
pressure) through the C ABI, against the oracle: MUSCL-Hancock + MC on the
relativistic workload under the ideal and Taub-Matthews equations of state,
with the isotropic and the exact fast speeds, and with the MT corner
coupling."""
import pytest

from paper_1110_0740_amd import inputs as I
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_rmhd_hlld_ideal(precision, tol):
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="hlld")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_rmhd_hlld_taub_matthews(precision, tol):
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="hlld", eos="tm")


def test_rmhd_hlld_exact_speeds_ragged_box():
    V, meta = I.rmhd3d_fields(n=19, ng=4, seed=4004, gmax_cap=3.0)
    V = V[:, :11 + 8, :13 + 8, :]
    meta = dict(meta)
    meta["box"] = I.Box((0, 0, 0), (19, 13, 11))
    _compare_one_step(V, meta, "fp64", TOL64, (19, 13, 11), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="hlld", exact_speeds=True)


def test_rmhd_hlld_mt_corner():
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="hlld", corner="mt")
