"""GPU parity of the Roe solver for MHD (Cargo-Gallice averages, closed-form
eigenvectors of the averaged state) through the C ABI, against the
oracle: PPM characteristic tracing on a ragged box (t^n and time-centred
solves), the 2D workload with MC-linear tracing, WENO3 tracing and
MUSCL-Hancock."""
import pytest

from paper_1110_0740_amd import inputs as I
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd3d_ppm_roe_ragged_box(precision, tol):
    V, meta = I.mhd3d_fields(n=19, ng=4, seed=2011)
    # a 19^3 generator box cut to 19 x 13 x 11 interior cells: several tiles
    # along x, ragged tails along y and z
    V = V[:, :11 + 8, :13 + 8, :]
    meta = dict(meta)
    meta["box"] = I.Box((0, 0, 0), (19, 13, 11))
    _compare_one_step(V, meta, precision, tol, (19, 13, 11), recon="ppm", riemann="roe")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd2d_mc_roe(precision, tol):
    V, meta = I.mhd2d_fields(n=128, ng=4, seed=1004)
    _compare_one_step(V, meta, precision, tol, (128, 128), recon="lin_mc", riemann="roe")


def test_mhd3d_weno3_roe():
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=2012)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), recon="weno3", riemann="roe")


def test_mhd3d_muscl_hancock_roe():
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=2013)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), recon="lin_vanleer", predictor="mh", riemann="roe")


@pytest.mark.parametrize("recon,wref", [("weno3", "cw84"), ("lin_mc", "cell")])
def test_generic_variant_roe(recon, wref):
    """A reference state other than the face value selects the kernels'
    generic option variant (the tests above run the fixed-option one)."""
    V, meta = I.mhd2d_fields(n=40, ng=4, seed=1005)
    _compare_one_step(V, meta, "fp64", TOL64, (40, 40), recon=recon, riemann="roe", wref=wref)
