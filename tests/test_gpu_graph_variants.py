"""HIP-graph replays of the widened option sets match their eager steps
bitwise, with eager work between the replays: the MT corner coupling (its
flux and difference kernels inside the graph), relativistic MHD with HLLD
(the secant iteration) and with the exact fast speeds, and the App. B
shock-adaptive hybrid (its flag kernels inside the graph)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.gpu_common import DEV, GpuStepper, gpu_opts, oracle_opts, single_box_plan
from tests.test_gpu_parity import _first_dt

pytestmark = pytest.mark.gpu

CASES = {
    "mt": dict(physics="mhd", recon="ppm", riemann="hlld", corner="mt"),
    "rmhd_hlld": dict(physics="rmhd", predictor="mh", recon="lin_mc", riemann="hlld"),
    "rmhd_exact_speeds": dict(physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", exact_speeds=True),
    "shock_hybrid": dict(physics="mhd", recon="ppm", riemann="hlld", shock_eps=0.5),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager(case, precision):
    kw = CASES[case]
    n, ng = 16, 4
    if kw["physics"] == "rmhd":
        V, meta = I.rmhd3d_fields(n=n, ng=ng, seed=4000, gmax_cap=4.0)
    else:
        V, meta = I.mhd3d_fields(n=n, ng=ng, seed=2003)
    oo = oracle_opts(3, meta["dx"], meta["gamma"], **kw)
    U = O.prim2cons(oo, V)
    dt, ch = _first_dt(oo, U, ng, 0.3)
    if kw["physics"] == "rmhd":
        ch = min(ch, 1.0)
    go = gpu_opts(3, meta["dx"], meta["gamma"], precision=precision, **kw)
    st = GpuStepper(single_box_plan(go, (n, n, n), ng), U.shape, precision)
    eager, rate_e, _, fails_e = st.step(U, dt, ch)
    assert fails_e == [0] * 5
    dtype = torch.float64 if precision == "fp64" else torch.float32
    s = torch.cuda.Stream()
    Uin = torch.from_numpy(U.reshape(-1)).to(dtype).to(DEV)
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
        got = Uout.cpu().numpy().astype(np.float64).reshape(U.shape)
        assert np.array_equal(I.interior(got, ng, 3), I.interior(eager, ng, 3)), (case, rep)
        assert rate.item() == rate_e
        assert fails.cpu().tolist() == [0] * 5
        st.step(U, dt, ch)  # eager work between replays


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager_nonideal(precision):
    """Viscosity, resistivity, saturated conduction and cooling: the parabolic
    flux kernels and the cooling source inside the graph; state, rate and
    max |dp/p| of every replay bitwise those of the eager step."""
    n, ng = 16, 4
    V, meta = I.mhd3d_fields(n=n, ng=ng, seed=5003)
    kw = dict(recon="ppm", riemann="hlld", parabolic_mask=7, tc_phi=0.3, cooling=True, cool_beta=0.5,
              nu=2e-2, eta=1.5e-2, kappa_par=3e-2, kappa_perp=4e-3)
    G = meta["gamma"]
    T = V[4] / V[0]
    kw["T_floor"] = 0.1 * float(T.min())
    oo = oracle_opts(3, meta["dx"], G, **kw)
    U = O.prim2cons(oo, V)
    dt, ch = _first_dt(oo, U, ng, 0.3)
    L0 = V[4] / ((G - 1) * V[0] ** 2 * np.sqrt(T) * (30.0 * dt))
    go = gpu_opts(3, meta["dx"], G, precision=precision, **kw)
    st = GpuStepper(single_box_plan(go, (n, n, n), ng), U.shape, precision)
    eager, rate_e, dpp_e, fails_e = st.step(U, dt, ch, L0=L0)
    assert fails_e == [0] * 5 and dpp_e > 0.0
    dtype = torch.float64 if precision == "fp64" else torch.float32
    s = torch.cuda.Stream()
    Uin = torch.from_numpy(U.reshape(-1)).to(dtype).to(DEV)
    Uout = torch.zeros_like(Uin)
    L0d = torch.from_numpy(np.ascontiguousarray(L0).reshape(-1)).to(dtype).to(DEV)
    params = torch.tensor([dt, ch], dtype=torch.float64, device=DEV)
    rate = torch.zeros(1, dtype=torch.float64, device=DEV)
    dpp = torch.zeros(1, dtype=torch.float64, device=DEV)
    fails = torch.zeros(5, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        st.plan.graph_capture(Uin, Uout, params, rate, L0=L0d, dpp=dpp, fails=fails, stream=s)
    s.synchronize()
    for rep in range(3):
        Uout.zero_()
        rate.fill_(123.0)
        dpp.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            st.plan.graph_launch(stream=s)
        s.synchronize()
        got = Uout.cpu().numpy().astype(np.float64).reshape(U.shape)
        assert np.array_equal(I.interior(got, ng, 3), I.interior(eager, ng, 3)), rep
        assert rate.item() == rate_e and dpp.item() == dpp_e, rep
        assert fails.cpu().tolist() == [0] * 5
        st.step(U, dt, ch, L0=L0)  # eager work between replays
