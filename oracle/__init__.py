"""ctypes front end of the FP64 CPU oracle (``oracle/ctu_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product library.
The shared object is compiled here with gcc (no fast-math, no FMA
contraction) when it is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ctu_oracle.c")
LIB = os.path.join(HERE, "libctu_oracle.so")

PHYS = {"mhd": 0, "rmhd": 1}
RECON = {"lin_mc": 0, "lin_minmod": 1, "lin_vanleer": 2, "lin_vanalbada": 3, "ppm": 4, "weno3": 5}
PRED = {"char": 0, "mh": 1}
WREF = {"face": 0, "cell": 1, "cw84": 2}
RIEMANN = {"hlld": 0, "hll": 1, "rusanov": 2, "hllc": 3, "roe": 4}
EOS = {"ideal": 0, "tm": 1}
CORNER = {"tn": 0, "mt": 1}  # Eq. transv with t^n fluxes, or predictor fluxes
PARAB_VISC, PARAB_RES, PARAB_TC = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile the oracle shared object with gcc.  Its independent cell and
    face loops run on OpenMP threads (set_threads); results do not depend on
    the thread count."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Opts(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("physics", C.c_int), ("recon", C.c_int), ("predictor", C.c_int),
        ("wref", C.c_int), ("riemann", C.c_int),
        ("gamma", C.c_double), ("dx", C.c_double * 3),
        ("glm", C.c_int), ("glm_alpha", C.c_double),
        ("parabolic_mask", C.c_uint), ("nu", C.c_double), ("eta", C.c_double),
        ("kappa_par", C.c_double), ("kappa_perp", C.c_double), ("tc_phi", C.c_double),
        ("cooling", C.c_int), ("cool_beta", C.c_double), ("T_floor", C.c_double),
        ("hyperbolic_off", C.c_int), ("shock_eps", C.c_double), ("eos", C.c_int), ("exact_speeds", C.c_int),
        ("corner", C.c_int),
    ]


def make_opts(dim=3, physics="mhd", recon="ppm", predictor="char", wref="face", riemann="hlld", gamma=5.0 / 3.0,
              dx=(1.0, 1.0, 1.0), glm=True, glm_alpha=0.1, parabolic_mask=0, nu=0.0, eta=0.0, kappa_par=0.0,
              kappa_perp=0.0, tc_phi=0.0, cooling=False, cool_beta=0.5, T_floor=0.0, hyperbolic_off=False,
              shock_eps=0.0, eos="ideal", exact_speeds=False, corner="tn") -> Opts:
    o = Opts()
    o.dim = dim
    o.physics = PHYS[physics]
    o.recon = RECON[recon]
    o.predictor = PRED[predictor]
    o.wref = WREF[wref]
    o.riemann = RIEMANN[riemann]
    o.eos = EOS[eos]
    o.exact_speeds = int(bool(exact_speeds))
    o.corner = CORNER[corner]
    o.gamma = gamma
    for q in range(3):
        o.dx[q] = dx[q]
    o.glm = int(bool(glm))
    o.glm_alpha = glm_alpha
    o.parabolic_mask = parabolic_mask
    o.nu, o.eta, o.kappa_par, o.kappa_perp, o.tc_phi = nu, eta, kappa_par, kappa_perp, tc_phi
    o.cooling = int(bool(cooling))
    o.cool_beta, o.T_floor = cool_beta, T_floor
    o.hyperbolic_off = int(bool(hyperbolic_off))
    o.shock_eps = shock_eps
    return o


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def configure(L):
    """Declare the argument types of a loaded oracle library (the built one,
    or a test's copy of it)."""
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [C.POINTER(Opts), C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, C.c_double,
                           C.c_double, _dp, _dp, _dp, _ip, C.POINTER(C.c_ubyte)]
    L.orc_shock_flags.restype = C.c_int
    L.orc_shock_flags.argtypes = [C.POINTER(Opts), C.c_int, C.c_int, C.c_int, C.c_int, _dp,
                                  C.POINTER(C.c_ubyte)]
    L.orc_cfl_rate.restype = C.c_double
    L.orc_cfl_rate.argtypes = [C.POINTER(Opts), C.c_int, C.c_int, C.c_int, C.c_int, _dp]
    L.orc_prim2cons.argtypes = [C.POINTER(Opts), C.c_long, _dp, _dp]
    L.orc_cons2prim.argtypes = [C.POINTER(Opts), C.c_long, _dp, _dp, _ip]
    L.orc_flux.argtypes = [C.POINTER(Opts), _dp, C.c_int, C.c_double, _dp]
    L.orc_riemann.argtypes = [C.POINTER(Opts), _dp, _dp, C.c_int, C.c_double, _dp, _dp]
    L.orc_speeds.argtypes = [C.POINTER(Opts), _dp, C.c_int, _dp, _dp]
    L.orc_eigen.argtypes = [C.POINTER(Opts), _dp, C.c_int, _dp, _dp, _dp]
    L.orc_reconstruct.argtypes = [C.c_int, _dp, C.c_double, _dp, _dp]
    L.orc_trace.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                            C.c_double, _dp, _dp]
    L.orc_predict.argtypes = [C.POINTER(Opts), _dp, _dp, C.c_int, C.c_double, C.c_double, _dp, _dp, _ip]
    L.orc_riemann_count.restype = C.c_long
    L.orc_riemann_count.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = configure(C.CDLL(build()))
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's OpenMP loops for the next calls (0: the
    OpenMP default, OMP_NUM_THREADS or every core); returns the count."""
    return int(lib().orc_set_threads(int(n)))


def riemann_count(reset: bool = True) -> int:
    """Riemann solves since the last reset (then cleared if `reset`)."""
    return int(lib().orc_riemann_count(int(bool(reset))))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def prim2cons(o: Opts, V: np.ndarray) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    U = np.empty_like(V)
    n = V.size // 9
    lib().orc_prim2cons(C.byref(o), n, _p(V), _p(U))
    return U


def cons2prim(o: Opts, U: np.ndarray):
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.empty_like(U)
    fails = (C.c_int * 5)()
    lib().orc_cons2prim(C.byref(o), U.size // 9, _p(U), _p(V), fails)
    return V, list(fails)


def flux(o: Opts, V, d: int, ch: float = 0.0) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.empty(9)
    lib().orc_flux(C.byref(o), _p(V), d, ch, _p(F))
    return F


def riemann(o: Opts, VL, VR, d: int, ch: float = 0.0):
    VL = np.ascontiguousarray(VL, dtype=np.float64)
    VR = np.ascontiguousarray(VR, dtype=np.float64)
    F = np.empty(9)
    s = np.zeros(1)
    lib().orc_riemann(C.byref(o), _p(VL), _p(VR), d, ch, _p(F), _p(s))
    return F, float(s[0])


def speeds(o: Opts, V, d: int):
    V = np.ascontiguousarray(V, dtype=np.float64)
    a = np.zeros(1)
    b = np.zeros(1)
    lib().orc_speeds(C.byref(o), _p(V), d, _p(a), _p(b))
    return float(a[0]), float(b[0])


def eigen(o: Opts, V, d: int):
    V = np.ascontiguousarray(V, dtype=np.float64)
    R = np.zeros((7, 7))
    L = np.zeros((7, 7))
    lam = np.zeros(7)
    lib().orc_eigen(C.byref(o), _p(V), d, _p(R), _p(L), _p(lam))
    return R, L, lam


def reconstruct(recon: str, w, dx: float = 1.0):
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert w.size == 5
    a = np.zeros(1)
    b = np.zeros(1)
    lib().orc_reconstruct(RECON[recon], _p(w), dx, _p(a), _p(b))
    return float(a[0]), float(b[0])


def trace(wref: str, w0, wm, wp, nu, numax=0.0, numin=0.0):
    a = np.zeros(1)
    b = np.zeros(1)
    lib().orc_trace(WREF[wref], w0, wm, wp, nu, numax, numin, _p(a), _p(b))
    return float(a[0]), float(b[0])


def predict(o: Opts, Vs, U0, d: int, dt: float, ch: float):
    Vs = np.ascontiguousarray(Vs, dtype=np.float64)
    U0 = np.ascontiguousarray(U0, dtype=np.float64)
    Vm = np.zeros(9)
    Vp = np.zeros(9)
    fails = (C.c_int * 5)()
    lib().orc_predict(C.byref(o), _p(Vs), _p(U0), d, dt, ch, _p(Vm), _p(Vp), fails)
    return Vm, Vp


def step(o: Opts, U: np.ndarray, ng: int, dt: float, ch: float, L0: np.ndarray | None = None,
         want_faces: bool = False, leaf: np.ndarray | None = None):
    """One CTU step of a ghosted box U[9, NZ, NY, NX].  Returns
    (U_out, rate, dpp, fails[, face_flux]); with `leaf` (a [NZ, NY, NX]
    mask) dpp is the maximum over the masked cells only."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    dim = o.dim
    NZ, NY, NX = U.shape[1:]
    nx, ny = NX - 2 * ng, NY - 2 * ng
    nz = NZ - 2 * ng if dim == 3 else 1
    Uo = np.empty_like(U)
    sc = np.zeros(2)
    fails = (C.c_int * 5)()
    ff = np.zeros((dim, 9) + U.shape[1:]) if want_faces else None
    L0p = _p(np.ascontiguousarray(L0, dtype=np.float64)) if L0 is not None else None
    if L0 is not None:
        L0 = np.ascontiguousarray(L0, dtype=np.float64)
        L0p = _p(L0)
    lf = None
    if leaf is not None:
        leaf = np.ascontiguousarray(leaf, dtype=np.uint8)
        lf = leaf.ctypes.data_as(C.POINTER(C.c_ubyte))
    rc = lib().orc_step(C.byref(o), nx, ny, nz, ng, _p(U), L0p, dt, ch, _p(Uo),
                        _p(ff) if ff is not None else None, _p(sc), fails, lf)
    if rc != 0:
        raise ValueError(f"orc_step rejected the options (code {rc})")
    out = (Uo, float(sc[0]), float(sc[1]), list(fails))
    return out + (ff,) if want_faces else out


def cfl_rate(o: Opts, U: np.ndarray, ng: int) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    NZ, NY, NX = U.shape[1:]
    nx, ny = NX - 2 * ng, NY - 2 * ng
    nz = NZ - 2 * ng if o.dim == 3 else 1
    return float(lib().orc_cfl_rate(C.byref(o), nx, ny, nz, ng, _p(U)))


def shock_flags(o: Opts, U: np.ndarray, ng: int) -> np.ndarray:
    """App. B flags of a ghosted box (bit 1: HLL zone, bit 2: MinMod zone)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    NZ, NY, NX = U.shape[1:]
    nx, ny = NX - 2 * ng, NY - 2 * ng
    nz = NZ - 2 * ng if o.dim == 3 else 1
    out = np.zeros((NZ, NY, NX), dtype=np.uint8)
    rc = lib().orc_shock_flags(C.byref(o), nx, ny, nz, ng, _p(U), out.ctypes.data_as(C.POINTER(C.c_ubyte)))
    if rc != 0:
        raise ValueError("orc_shock_flags rejected the options")
    return out
