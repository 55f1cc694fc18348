"""GPU parity of the MT corner coupling (transverse fluxes between
normal-predictor states, runs without parabolic terms) through the C ABI,
against the oracle: the 3D PPM + characteristic tracing + HLLD workload on a
ragged box, the 2D MC workload, WENO3 with the CW84 reference state,
MUSCL-Hancock MHD with Roe, and relativistic MHD with HLLC; plus the ABI's
rejection of MT with parabolic terms."""
import pytest

from paper_1110_0740_amd import ctu
from paper_1110_0740_amd import inputs as I
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd3d_ppm_hlld_mt_ragged_box(precision, tol):
    V, meta = I.mhd3d_fields(n=19, ng=4, seed=2014)
    V = V[:, :11 + 8, :13 + 8, :]
    meta = dict(meta)
    meta["box"] = I.Box((0, 0, 0), (19, 13, 11))
    _compare_one_step(V, meta, precision, tol, (19, 13, 11), recon="ppm", riemann="hlld", corner="mt")


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd2d_mc_hlld_mt(precision, tol):
    V, meta = I.mhd2d_fields(n=128, ng=4, seed=1006)
    _compare_one_step(V, meta, precision, tol, (128, 128), recon="lin_mc", riemann="hlld", corner="mt")


@pytest.mark.gpu
def test_mhd3d_weno3_cw84_mt():
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=2015)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), recon="weno3", riemann="hll", wref="cw84", corner="mt")


@pytest.mark.gpu
def test_mhd3d_muscl_hancock_roe_mt():
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=2016)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), recon="lin_vanleer", predictor="mh", riemann="roe",
                      corner="mt")


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_rmhd_hllc_mt(precision, tol):
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="hllc", corner="mt")


def test_mt_rejections_without_gpu():
    box = [((0, 0, 0), (8, 8, 8), 0, 0)]
    with pytest.raises(ctu.CtuError, match="MT"):
        ctu.Plan(ctu.make_opts(dim=3, recon="ppm", corner="mt", parabolic_mask=1, nu=0.01), box, 4)
    with pytest.raises(ctu.CtuError, match="MT"):
        ctu.Plan(ctu.make_opts(dim=3, recon="ppm", corner="mt", shock_eps=5.0), box, 4)
    with pytest.raises(ctu.CtuError, match="nghost"):
        ctu.Plan(ctu.make_opts(dim=3, recon="lin_mc", corner="mt"), box, 2)
    bad = ctu.make_opts(dim=3, recon="ppm")
    bad.corner = 2
    with pytest.raises(ctu.CtuError, match="corner"):
        ctu.Plan(bad, box, 4)
