"""GPU parity of the parabolic fluxes (Sec. 2.1.1, Sec. 3.1, App. A) through
the C ABI, against the FP64 oracle: each term on its own (viscosity,
resistivity, classical and saturated conduction), all terms in 2D on a box
that spans several tiles of the parabolic kernels, the generic option variant
(cell reference states), and the parabolic operator alone (hyperbolic fluxes
off).  Coefficients are a few times the non-ideal workload's largest, so that
the parabolic increments are ~1e-3 of the state: a wrong term moves the result
by far more than the tolerances."""
import pytest

from paper_1110_0740_amd import inputs as I
from tests.test_gpu_parity import TOL32, TOL64, _compare_one_step

pytestmark = pytest.mark.gpu

COEF = dict(nu=2e-2, eta=1.5e-2, kappa_par=3e-2, kappa_perp=4e-3)
BOX3 = (13, 11, 9)  # ragged against the 32 x 8 tiles and 16-plane chunks


def _fields3(seed):
    return I.mhd3d_fields(n=16, ng=4, seed=seed, box=I.Box((0, 0, 0), BOX3), level_n=16, v_rms=0.5)


@pytest.mark.parametrize("mask,phi", [(1, 0.0), (2, 0.0), (4, 0.0), (4, 0.3)],
                         ids=["viscosity", "resistivity", "conduction", "saturated_conduction"])
def test_single_parabolic_terms_fp64(mask, phi):
    print(f"parabolic term mask {mask} phi {phi}: {BOX3}", flush=True)
    V, meta = _fields3(5100 + mask)
    e, _, _ = _compare_one_step(V, meta, "fp64", TOL64, BOX3, recon="ppm", riemann="hlld", parabolic_mask=mask,
                                tc_phi=phi, **COEF)
    print(f"L1 {e.max():.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_parabolic_2d_across_tiles(precision, tol):
    """2D, 300 x 20: the 256-wide rows of k_pflux and the 255-wide rows of
    k_pdiv's overlapping tiles each need two tiles per row."""
    n2 = (300, 20)
    print(f"parabolic 2D {precision}: {n2}", flush=True)
    V, meta = I.mhd2d_fields(n=384, ng=4, seed=5200, box=I.Box((0, 0, 0), (n2[0], n2[1], 1)))
    e, _, _ = _compare_one_step(V, meta, precision, tol, n2, recon="ppm", riemann="hlld", parabolic_mask=7,
                                tc_phi=0.3, **COEF)
    print(f"L1 {e.max():.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_parabolic_generic_variant(precision, tol):
    """Cell reference states select the generic sweep and t^n kernels, which
    read the parabolic options at run time."""
    print(f"parabolic generic variant {precision}: {BOX3}", flush=True)
    V, meta = _fields3(5300)
    e, _, _ = _compare_one_step(V, meta, precision, tol, BOX3, recon="ppm", riemann="hlld", wref="cell",
                                parabolic_mask=7, tc_phi=0.3, **COEF)
    print(f"L1 {e.max():.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_parabolic_operator_alone(precision, tol):
    """Hyperbolic fluxes off: the step is the unsplit parabolic update with
    the half-step state of Eq. transv."""
    print(f"parabolic operator alone {precision}: {BOX3}", flush=True)
    V, meta = _fields3(5400)
    e, _, _ = _compare_one_step(V, meta, precision, tol, BOX3, recon="ppm", riemann="hlld", hyperbolic_off=True,
                                parabolic_mask=7, tc_phi=0.3, **COEF)
    print(f"L1 {e.max():.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_parabolic_several_boxes_one_plan(precision, tol):
    """Three boxes of different extents in one plan: the parabolic kernels'
    tile tables span the boxes and each box's face slots sit at its own
    workspace offset.  Each box against the oracle's step of that box alone."""
    import numpy as np

    import oracle as O
    from paper_1110_0740_amd import ctu
    from tests.gpu_common import GpuStepper, assert_parity, gpu_opts, oracle_opts

    exts = [(13, 11, 9), (21, 7, 12), (8, 16, 10)]
    los = [(0, 0, 0), (16, 0, 0), (40, 0, 0)]
    ng = 4
    kw = dict(recon="ppm", riemann="hlld", parabolic_mask=7, tc_phi=0.3, **COEF)
    print(f"parabolic several boxes {precision}: {exts}", flush=True)
    blocks, boxes, off, rates, meta = [], [], 0, [], None
    for b, (n, lo) in enumerate(zip(exts, los)):
        V, meta = I.mhd3d_fields(n=16, ng=ng, seed=5500 + b, box=I.Box(lo, n), level_n=16, v_rms=0.5)
        oo = oracle_opts(3, meta["dx"], meta["gamma"], **kw)
        U = O.prim2cons(oo, V)
        rates.append(O.cfl_rate(oo, U, ng))
        blocks.append(U)
        boxes.append((lo, n, 0, off))
        off += U.size
    dt = 0.4 / max(rates)
    ch = 0.4 * meta["dx"][0] / dt
    oo = oracle_opts(3, meta["dx"], meta["gamma"], **kw)
    refs = [O.step(oo, U, ng, dt, ch)[0] for U in blocks]
    plan = ctu.Plan(gpu_opts(3, meta["dx"], meta["gamma"], precision=precision, **kw), boxes, ng)
    st = GpuStepper(plan, (off,), precision)
    Ucat = np.concatenate([U.reshape(-1) for U in blocks])
    if precision == "fp32":
        Ucat = Ucat.astype(np.float32).astype(np.float64)
    out, rate, dpp, fails = st.step(Ucat, dt, ch)
    assert fails == [0] * 5
    pos = 0
    for U, ref in zip(blocks, refs):
        got = out[pos:pos + U.size].reshape(U.shape)
        pos += U.size
        e, c = assert_parity(got, ref, ng, 3, ch, tol)
        print(f"L1 {e.max():.2e} cell {c.max():.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_parabolic_with_shock_flags(precision, tol):
    """With the App. B zone flags the t^n kernel and the sweeps run their
    shock-flag variants, which read the parabolic options at run time."""
    print(f"parabolic with shock flags {precision}: {BOX3}", flush=True)
    V, meta = _fields3(5600)
    e, _, _ = _compare_one_step(V, meta, precision, tol, BOX3, recon="ppm", riemann="hlld", shock_eps=0.05,
                                parabolic_mask=7, tc_phi=0.3, **COEF)
    print(f"L1 {e.max():.2e}")


@pytest.mark.parametrize("ext", [(3, 2, 5), (1, 4, 2), (5, 1, 1)])
@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_parabolic_tiny_boxes(precision, tol, ext):
    """Boxes of one to five cells per axis: the parabolic kernels' regions are
    smaller than one tile and one chunk in every direction."""
    print(f"parabolic tiny box {precision}: {ext}", flush=True)
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=5700 + sum(ext), box=I.Box((0, 0, 0), ext), level_n=16, v_rms=0.5)
    e, _, _ = _compare_one_step(V, meta, precision, tol, ext, recon="ppm", riemann="hlld", parabolic_mask=7,
                                tc_phi=0.3, **COEF)
    print(f"L1 {e.max():.2e}")
