"""GPU parity of the Rusanov (local Lax-Friedrichs) solver through the C
ABI, against the oracle: 3D MHD with PPM characteristic tracing on a ragged
box (t^n and time-centred solves), the 2D workload with MC-linear tracing,
MUSCL-Hancock MHD, relativistic MHD with the FP64 inversion, and the generic
option variant."""
import pytest

from paper_1110_0740_amd import inputs as I
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd3d_ppm_rusanov_ragged_box(precision, tol):
    V, meta = I.mhd3d_fields(n=19, ng=4, seed=2006)
    # a 19^3 generator box cut to 19 x 13 x 11 interior cells: several tiles
    # along x, ragged tails along y and z
    V = V[:, :11 + 8, :13 + 8, :]
    meta = dict(meta)
    meta["box"] = I.Box((0, 0, 0), (19, 13, 11))
    _compare_one_step(V, meta, precision, tol, (19, 13, 11), recon="ppm", riemann="rusanov")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd2d_mc_rusanov(precision, tol):
    V, meta = I.mhd2d_fields(n=128, ng=4, seed=1000)
    _compare_one_step(V, meta, precision, tol, (128, 128), recon="lin_mc", riemann="rusanov")


def test_mhd3d_muscl_hancock_rusanov():
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=2007)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), recon="lin_vanleer", predictor="mh", riemann="rusanov")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_rmhd_rusanov(precision, tol):
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="rusanov")



@pytest.mark.parametrize("recon,wref", [("ppm", "cw84"), ("lin_mc", "cell")])
def test_generic_variant_rusanov(recon, wref):
    """A reference state other than the face value selects the kernels'
    generic option variant (the tests above run the fixed-option one)."""
    V, meta = I.mhd2d_fields(n=40, ng=4, seed=1003)
    _compare_one_step(V, meta, "fp64", TOL64, (40, 40), recon=recon, riemann="rusanov", wref=wref)
