"""GPU parity on the degenerate MHD states where the GPU's closed-form left
eigenvectors and its HLLD degeneracy switch differ most from the oracle's
numerical inversion and FP64 threshold (PPM characteristic tracing + HLLD +
GLM, the 3D workload's options, one step, FP64 and FP32):

  * field along x only: B_t = 0 on x faces (beta_y = beta_z = 1/sqrt2 in the
    eigenvectors), B_n = 0 on y and z faces (HLLD's B_n -> 0 limit);
  * field along y only: B_n = 0 on x and z faces, B_t = 0 on y faces;
  * the triple point a = c_a with B along x and uniform rho, p (c_f = c_s =
    c_a on x faces: alpha_f = 1, alpha_s = 0), transverse velocity only;
  * B = 0: the Sod shock tube along x (hydrodynamics through the MHD
    solver: every Alfven and slow family degenerates).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1110_0740_amd import inputs as I
from tests.gpu_common import GpuStepper, assert_parity, gpu_opts, oracle_opts, single_box_plan

pytestmark = pytest.mark.gpu

NG = 4
N = (20, 12, 10)
G = 5.0 / 3.0


def smooth_fields():
    V, _ = I.mhd3d_fields(ng=NG, seed=2300, box=I.Box((0, 0, 0), N), level_n=32)
    return V


def state(case):
    if case == "sod_b0":
        V = np.zeros((9,) + tuple(n + 2 * NG for n in reversed(N)))
        x = np.arange(N[0] + 2 * NG) - NG
        left = (x < N[0] // 2)[None, None, :]
        V[0] = np.where(left, 1.0, 0.125)
        V[4] = np.where(left, 1.0, 0.1)
        return V, (2, 3)  # v_y = v_z = 0 and B = 0 stay zero: natural scale for m_y, m_z
    V = smooth_fields()
    if case == "bx_only":
        V[5], V[6], V[7] = 1.1, 0.0, 0.0
    elif case == "by_only":
        V[5], V[6], V[7] = 0.0, 0.9, 0.0
    elif case == "triple_point":
        V[0] = 1.0
        V[4] = 0.6
        V[1] = 0.0
        V[5], V[6], V[7] = math.sqrt(G * 0.6), 0.0, 0.0  # a^2 = Gamma p / rho = B_x^2 / rho
        return V, (1,)  # v_x = 0 initially
    return V, ()


@pytest.mark.parametrize("case", ["bx_only", "by_only", "triple_point", "sod_b0"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_degenerate_state_matches_oracle(case, precision, tol):
    V, natural = state(case)
    dx = (1.0 / 32,) * 3
    kw = dict(recon="ppm", riemann="hlld")
    oo = oracle_opts(3, dx, G, **kw)
    U = O.prim2cons(oo, V)
    if case == "triple_point":
        Vc, _ = O.cons2prim(oo, U)
        a2 = G * Vc[4] / Vc[0]
        ca2 = Vc[5] ** 2 / Vc[0]
        assert np.abs(a2 - ca2).max() < 1e-14
    dt = 0.3 / O.cfl_rate(oo, U, NG)
    ch = 0.3 * dx[0] / dt
    ref, rref, _, fref = O.step(oo, U, NG, dt, ch)
    st = GpuStepper(single_box_plan(gpu_opts(3, dx, G, precision=precision, **kw), N, NG), U.shape, precision)
    Ug = U.astype(np.float32).astype(np.float64) if precision == "fp32" else U
    got, rate, _, fails = st.step(Ug, dt, ch)
    assert fails == [0] * 5 and fref == [0] * 5
    assert_parity(got, ref, NG, 3, ch, tol, natural=natural, what=case)
    assert abs(rate - rref) <= (1e-13 if precision == "fp64" else 2e-6) * rref
