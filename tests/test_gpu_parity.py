"""GPU parity: the HIP CTU step (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (relative L1 per conserved variable over interior cells, psi
against c_h sum|B|):
  FP64 one step from identical inputs   <= 1e-12
  FP64 ten chained steps                <= 1e-11
  FP32 one step                         <= 2e-6
  FP32 one hundred chained steps        <= 1e-5   (smooth data, oracle dt)
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1110_0740_amd import ctu, inputs as I
from tests.gpu_common import DEV, GpuStepper, assert_parity, gpu_opts, l1rel, oracle_opts, single_box_plan

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL64_CHAIN = 1e-11
TOL32 = 2e-6
TOL32_CHAIN = 1e-5


def _first_dt(oo, U, ng, cfl=0.4):
    rate = O.cfl_rate(oo, U, ng)
    dt = cfl / rate
    return dt, cfl * min(oo.dx[q] for q in range(oo.dim)) / dt


def _compare_one_step(V, meta, precision, tol, n_int, **kw):
    return _compare_one_step_ctol(V, meta, precision, tol, None, n_int, **kw)


def _compare_one_step_ctol(V, meta, precision, tol, ctol, n_int, **kw):
    dim, ng, dx, gam = meta["dim"], meta["ng"], meta["dx"], meta["gamma"]
    L0 = kw.pop("_L0", None)
    oo = oracle_opts(dim, dx, gam, **kw)
    U = O.prim2cons(oo, V)
    dt, ch = _first_dt(oo, U, ng, 0.3 if kw.get("physics") == "rmhd" else 0.4)
    if kw.get("physics") == "rmhd":
        ch = min(ch, 1.0)
    Uref, rref, dref, fref = O.step(oo, U, ng, dt, ch, L0=L0)
    go = gpu_opts(dim, dx, gam, precision=precision, **kw)
    st = GpuStepper(single_box_plan(go, n_int, ng), U.shape, precision)
    Ug = U.astype(np.float32).astype(np.float64) if precision == "fp32" else U
    out, rate, dpp, fails = st.step(Ug, dt, ch, L0=L0)
    assert fails == [0] * 5 and fref == [0] * 5, (fails, fref)
    e, c = assert_parity(out, Uref, ng, dim, ch, tol, kw.get("physics", "mhd"), ctol=ctol)
    print(f"cell {c.max():.2e}")
    assert abs(rate - rref) <= max(tol, 1e-7 if precision == "fp32" else 1e-13) * rref * 10, (rate, rref)
    return e, out, Uref


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mhd2d_128_one_step(precision, tol):
    V, meta = I.mhd2d_fields(n=128, ng=4, seed=1000)
    _compare_one_step(V, meta, precision, tol, (128, 128), recon="lin_mc", riemann="hlld")


def test_mhd2d_128_ten_chained_steps_fp64():
    """Ten chained steps of the 2D workload; both sides use the oracle's dt
    and c_h sequence; ghosts refilled periodically between steps."""
    n, ng = 128, 4
    V, meta = I.mhd2d_fields(n=n, ng=ng, seed=1000)
    oo = oracle_opts(2, meta["dx"], meta["gamma"], recon="lin_mc", riemann="hlld")
    U = O.prim2cons(oo, V)
    go = gpu_opts(2, meta["dx"], meta["gamma"], recon="lin_mc", riemann="hlld")
    st = GpuStepper(single_box_plan(go, (n, n), ng), U.shape, "fp64")
    Uo, Ug = U.copy(), U.copy()
    dt, ch = _first_dt(oo, U, ng)
    for s in range(10):
        Uo_next, rref, _, _ = O.step(oo, Uo, ng, dt, ch)
        Ug_next, rate, _, fails = st.step(Ug, dt, ch)
        assert fails == [0] * 5
        I.fill_periodic(Uo_next, ng, 2)
        I.fill_periodic(Ug_next, ng, 2)
        Uo, Ug = Uo_next, Ug_next
        dt = 0.4 / rref
        ch = 0.4 * meta["dx"][0] / dt
    assert_parity(Ug, Uo, ng, 2, ch, TOL64_CHAIN)


@pytest.mark.parametrize("n", [(24, 24, 24), (19, 13, 11), (5, 7, 6)])
def test_mhd3d_ppm_fp64_one_step(n):
    """PPM characteristic tracing + HLLD + GLM (the 3D workload's options) on
    cubic and ragged boxes."""
    ng = 4
    box = I.Box((3, 5, 7), n)
    V, meta = I.mhd3d_fields(n=max(n), ng=ng, seed=2000, box=box, level_n=32)
    _compare_one_step(V, meta, "fp64", TOL64, n, recon="ppm", riemann="hlld")


def test_mhd3d_ppm_fp32_one_step():
    V, meta = I.mhd3d_fields(n=24, ng=4, seed=2000)
    _compare_one_step(V, meta, "fp32", TOL32, (24, 24, 24), recon="ppm", riemann="hlld")


def test_mhd3d_ppm_fp32_hundred_chained_steps():
    """FP32 GPU vs FP64 oracle after 100 chained steps of the 3D workload's
    generator at 64^3 (PPM + HLLD + GLM; the oracle's dt sequence drives
    both, ghosts refilled periodically), every cell compared.

    Smooth-data settings: at the configured Mach 1 the flow steepens and the
    oracle itself reaches p < 0 by step 33 (no floors); at v_rms = 0.3 and
    CFL 0.4 the PPM run with psi damping 0.1 breaks down at step 14 (it
    survives with damping 0.8 or MC slopes), so the run uses v_rms = 0.3 at
    CFL 0.3, which stays physical over the 100 steps."""
    n, ng, cfl = 64, 4, 0.3
    V, meta = I.mhd3d_fields(n=n, ng=ng, seed=2001, v_rms=0.3)
    oo = oracle_opts(3, meta["dx"], meta["gamma"], recon="ppm", riemann="hlld")
    U = O.prim2cons(oo, V)
    go = gpu_opts(3, meta["dx"], meta["gamma"], precision="fp32", recon="ppm", riemann="hlld")
    st = GpuStepper(single_box_plan(go, (n, n, n), ng), U.shape, "fp32")
    Uo = U.copy()
    Ug = U.astype(np.float32).astype(np.float64)
    dt, ch = _first_dt(oo, U, ng, cfl)
    for s in range(100):
        Uo_next, rref, _, fref = O.step(oo, Uo, ng, dt, ch)
        Ug_next, _, _, fails = st.step(Ug, dt, ch)
        assert fails == [0] * 5 and fref == [0] * 5, (s, fails, fref)
        I.fill_periodic(Uo_next, ng, 3)
        I.fill_periodic(Ug_next, ng, 3)
        Uo, Ug = Uo_next, Ug_next
        dt = cfl / rref
        ch = cfl * meta["dx"][0] / dt
    # per cell: FP32 rounding differences grow where the flow steepens over
    # 100 steps (1.6e-3 of max|q| measured at the worst cell), well apart
    # from a wrong cell's O(1)
    e, c = assert_parity(Ug, Uo, ng, 3, ch, TOL32_CHAIN, ctol=5e-3)
    print(f"64^3 FP32 100 steps: L1 {e.max():.2e} cell {c.max():.2e}")


@pytest.mark.parametrize("recon,riemann,wref", [
    ("weno3", "hlld", "face"), ("lin_minmod", "hll", "face"), ("lin_vanleer", "hlld", "cell"),
    ("lin_vanalbada", "hlld", "cw84"), ("ppm", "hll", "cw84"), ("weno3", "hll", "cell")])
def test_scheme_variants_fp64(recon, riemann, wref):
    V, meta = I.mhd2d_fields(n=40, ng=4, seed=1002)
    _compare_one_step(V, meta, "fp64", TOL64, (40, 40), recon=recon, riemann=riemann, wref=wref)


@pytest.mark.parametrize("recon,riemann,wref", [
    ("lin_minmod", "hll", "face"), ("lin_mc", "hlld", "cw84"), ("ppm", "hlld", "cell"), ("ppm", "hll", "face")])
def test_scheme_variants_fp32(recon, riemann, wref):
    """The FP32 limiters are medians (minmod, MC and the PPM constraints of
    Sec. 3.2): the values of the FP64 selects, so parity at the FP32
    tolerance on each limiter and reference state."""
    V, meta = I.mhd2d_fields(n=40, ng=4, seed=1003)
    _compare_one_step(V, meta, "fp32", TOL32, (40, 40), recon=recon, riemann=riemann, wref=wref)


@pytest.mark.parametrize("riemann", ["hlld", "hll"])
def test_mhd_muscl_hancock_fp64(riemann):
    V, meta = I.mhd3d_fields(n=16, ng=4, seed=2002)
    _compare_one_step(V, meta, "fp64", TOL64, (16, 16, 16), recon="lin_mc", predictor="mh", riemann=riemann)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_rmhd_muscl_hancock_hll(precision, tol):
    """Relativistic jets/blobs (Lorentz factors up to 4 at this size),
    MUSCL-Hancock + MC + HLL + GLM; the inversion is FP64 on both sides."""
    V, meta = I.rmhd3d_fields(n=16, ng=4, seed=4000, gmax_cap=4.0)
    _compare_one_step(V, meta, precision, tol, (16, 16, 16), physics="rmhd", recon="lin_mc", predictor="mh",
                      riemann="hll")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_nonideal_parabolic_and_cooling(precision, tol):
    """Viscosity, resistivity, saturated anisotropic conduction as unsplit
    fluxes, plus the exact power-law cooling source with per-cell L0."""
    n, ng = 14, 4
    V, meta = I.mhd3d_fields(n=n, ng=ng, seed=5000)
    coef = I.nonideal_coeffs(5001)
    oo = oracle_opts(3, meta["dx"], meta["gamma"], recon="ppm", riemann="hlld")
    U = O.prim2cons(oo, V)
    dt0 = 0.4 / O.cfl_rate(oo, U, ng)
    X, Y, Z = I.cell_centres(meta["box"], ng, meta["dx"], 3)
    tc = I.cooling_time_field(5002, X, Y, Z, dt0)
    G = meta["gamma"]
    T = V[4] / V[0]
    L0 = V[4] / ((G - 1) * V[0] ** 2 * np.sqrt(T) * tc)
    kw = dict(recon="ppm", riemann="hlld", parabolic_mask=7, tc_phi=0.3, cooling=True, cool_beta=0.5,
              T_floor=0.1 * float(T.min()), **coef)
    if precision == "fp32":
        L0 = L0.astype(np.float32).astype(np.float64)
    kw["_L0"] = L0
    e, out, ref = _compare_one_step(V, meta, precision, tol, (n, n, n), **kw)


@pytest.mark.parametrize("precision,tol,ctol", [("fp64", TOL64, None), ("fp32", TOL32, None)])
def test_nonideal_white_noise_cooling_times(precision, tol, ctol):
    """The non-ideal workload with white-noise cooling times (t_c / dt0
    log-uniform in [1e-3, 1e3], independent per cell): the stiffest cells
    cool to the floor within the step, so neighbouring cells differ by orders
    of magnitude in their source.  The smooth case's bounds hold (measured
    FP32: L1 8e-8, largest cell 1.1e-6)."""
    n, ng = 14, 4
    V, meta = I.mhd3d_fields(n=n, ng=ng, seed=5000)
    coef = I.nonideal_coeffs(5001)
    oo = oracle_opts(3, meta["dx"], meta["gamma"], recon="ppm", riemann="hlld")
    U = O.prim2cons(oo, V)
    dt0 = 0.4 / O.cfl_rate(oo, U, ng)
    tc = I.cooling_time_white(5003, n, ng, dt0)
    G = meta["gamma"]
    T = V[4] / V[0]
    L0 = V[4] / ((G - 1) * V[0] ** 2 * np.sqrt(T) * tc)
    kw = dict(recon="ppm", riemann="hlld", parabolic_mask=7, tc_phi=0.3, cooling=True, cool_beta=0.5,
              T_floor=0.1 * float(T.min()), **coef)
    if precision == "fp32":
        L0 = L0.astype(np.float32).astype(np.float64)
    kw["_L0"] = L0
    e, out, ref = _compare_one_step_ctol(V, meta, precision, tol, ctol, (n, n, n), **kw)
    print(f"white-noise cooling {precision}: L1 {e.max():.2e}")


def test_graph_replays_match_eager():
    n, ng = 20, 4
    V, meta = I.mhd3d_fields(n=n, ng=ng, seed=2003)
    oo = oracle_opts(3, meta["dx"], meta["gamma"])
    U = O.prim2cons(oo, V)
    dt, ch = _first_dt(oo, U, ng)
    go = gpu_opts(3, meta["dx"], meta["gamma"], recon="ppm", riemann="hlld")
    st = GpuStepper(single_box_plan(go, (n, n, n), ng), U.shape, "fp64")
    eager, rate_e, _, _ = st.step(U, dt, ch)
    s = torch.cuda.Stream()
    Uin = torch.from_numpy(U.reshape(-1)).to(DEV)
    Uout = torch.zeros_like(Uin)
    params = torch.tensor([dt, ch], dtype=torch.float64, device=DEV)
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    fails = torch.zeros(5, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        st.plan.graph_capture(Uin, Uout, params, rate, fails=fails, stream=s)
    s.synchronize()
    for rep in range(3):
        Uout.zero_()
        rate.fill_(123.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            st.plan.graph_launch(stream=s)
        s.synchronize()
        got = Uout.cpu().numpy().reshape(U.shape)
        assert np.array_equal(I.interior(got, ng, 3), I.interior(eager, ng, 3))
        assert rate.item() == rate_e
        # eager work between replays
        st.step(U, dt, ch)


def test_failure_counters_count_unphysical_cells():
    """A forced negative-pressure cell is counted, not fatal (condition set
    from the host; every kernel runs to completion)."""
    n, ng = 16, 4
    V, meta = I.mhd2d_fields(n=n, ng=ng, seed=1003)
    oo = oracle_opts(2, meta["dx"], meta["gamma"], recon="lin_mc")
    U = O.prim2cons(oo, V)
    U[4, 0, ng + 5, ng + 5] = 0.0  # energy below the kinetic + magnetic part
    go = gpu_opts(2, meta["dx"], meta["gamma"], recon="lin_mc")
    st = GpuStepper(single_box_plan(go, (n, n), ng), U.shape, "fp64")
    out, rate, _, fails = st.step(U, 1e-3, 1.0)
    assert fails[1] >= 1


def test_prim_cons_maps_and_cfl_rate():
    for physics, (V, meta) in (("mhd", I.mhd3d_fields(n=12, ng=4, seed=2004)),
                               ("rmhd", I.rmhd3d_fields(n=12, ng=4, seed=4001, gmax_cap=10.0))):
        kw = dict(physics=physics, recon="lin_mc", predictor="mh" if physics == "rmhd" else "char",
                  riemann="hll" if physics == "rmhd" else "hlld")
        oo = oracle_opts(3, meta["dx"], meta["gamma"], **kw)
        Uref = O.prim2cons(oo, V)
        go = gpu_opts(3, meta["dx"], meta["gamma"], **kw)
        plan = single_box_plan(go, (12, 12, 12), 4)
        Vd = torch.from_numpy(V.reshape(-1)).to(DEV)
        Ud = torch.zeros_like(Vd)
        plan.prim_to_cons(Vd, Ud)
        V2 = torch.zeros_like(Vd)
        fails = torch.zeros(5, dtype=torch.int32, device=DEV)
        plan.cons_to_prim(Ud, V2, fails=fails)
        rate = torch.zeros(1, dtype=torch.float64, device=DEV)
        plan.cfl_rate(Ud, rate)
        torch.cuda.synchronize()
        Ug = Ud.cpu().numpy().reshape(V.shape)
        assert np.max(np.abs(Ug - Uref) / (np.abs(Uref) + 1e-300)) < 1e-13
        assert fails.sum().item() == 0
        assert np.max(np.abs(V2.cpu().numpy().reshape(V.shape) - V) / (np.abs(V) + 1.0)) < 1e-12
        rref = O.cfl_rate(oo, Uref, 4)
        assert abs(rate.item() - rref) < 1e-12 * rref


def test_bad_arguments_rejected():
    with pytest.raises(ctu.CtuError):
        ctu.Plan(ctu.make_opts(dim=3, physics="rmhd", predictor="char"), [((0, 0, 0), (8, 8, 8), 0, 0)], 4)
    with pytest.raises(ctu.CtuError):
        ctu.Plan(ctu.make_opts(dim=3, recon="ppm", predictor="mh"), [((0, 0, 0), (8, 8, 8), 0, 0)], 4)
    with pytest.raises(ctu.CtuError):
        ctu.Plan(ctu.make_opts(dim=3), [((0, 0, 0), (8, 8, 8), 0, 0)], 2)
    with pytest.raises(ctu.CtuError):
        ctu.Plan(ctu.make_opts(dim=3), [((0, 0, 0), (8, 8, 8), 0, 0), ((0, 0, 0), (8, 8, 8), 0, 9)], 4)
