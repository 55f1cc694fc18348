"""Thin ctypes binding of libctu.so (argument marshalling only).

Every entry point mirrors a function of ``include/ctu.h`` and takes torch
CUDA tensors for device buffers; the computation runs entirely in the HIP
kernels of the library.  Loading fails loudly when the shared object is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctu.so")

MHD, RMHD = 0, 1
FP64, FP32 = 0, 1
RECON = {"lin_mc": 0, "lin_minmod": 1, "lin_vanleer": 2, "lin_vanalbada": 3, "ppm": 4, "weno3": 5}
PRED = {"char": 0, "mh": 1}
WREF = {"face": 0, "cell": 1, "cw84": 2}
RIEMANN = {"hlld": 0, "hll": 1, "rusanov": 2, "hllc": 3, "roe": 4}
EOS = {"ideal": 0, "tm": 1}
CORNER = {"tn": 0, "mt": 1}
PARAB_VISC, PARAB_RES, PARAB_TC = 1, 2, 4
NFAIL = 5

# exported C symbols (kept in step with include/ctu.h)
SYMBOLS = [
    "ctu_plan_create", "ctu_plan_destroy", "ctu_plan_state_elems", "ctu_plan_workspace_bytes", "ctu_step",
    "ctu_step_graph_capture", "ctu_step_graph_launch", "ctu_cfl_rate", "ctu_prim_to_cons", "ctu_cons_to_prim",
    "ctu_plan_set_reflux", "ctu_reflux", "ctu_reflux_consume", "ctu_plan_enable_timing", "ctu_plan_read_timing",
    "ctu_last_error", "ctu_hier_create", "ctu_hier_destroy", "ctu_hier_fill_ghosts", "ctu_hier_average_down",
    "ctu_hier_advance", "ctu_hier_leaf_mask", "ctu_hier_tag", "ctu_hier_next_dt", "ctu_plan_set_leaf_mask",
    "ctu_plan_set_shape", "ctu_plan_get_shape", "ctu_plan_autotune", "ctu_tune_cache_clear",
    "ctu_plan_create_ex", "ctu_plan_set_workspace", "ctu_plan_device", "ctu_step_static",
    "ctu_static_scratch_bytes", "ctu_measure_fma", "ctu_measure_copy",
]
PLAN_CALLER_WORKSPACE = 1
PLAN_LEVEL_DT = 2
TC_LAYOUT = {"auto": 0, "tiles": 1, "flat": 2}
NSTAGE = 8
STAGES = ["prim", "tcouple", "pdiv", "pflux", "unused4", "sweep_x", "sweep_y", "sweep_z"]


class CtuOpts(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("physics", C.c_int32), ("precision", C.c_int32), ("recon", C.c_int32),
        ("predictor", C.c_int32), ("wref", C.c_int32), ("riemann", C.c_int32), ("glm", C.c_int32),
        ("gamma", C.c_double), ("dx", C.c_double * 3), ("glm_alpha", C.c_double),
        ("parabolic_mask", C.c_uint32), ("cooling", C.c_int32),
        ("nu", C.c_double), ("eta", C.c_double), ("kappa_par", C.c_double), ("kappa_perp", C.c_double),
        ("tc_phi", C.c_double), ("cool_beta", C.c_double), ("T_floor", C.c_double),
        ("hyperbolic_off", C.c_int32), ("pad", C.c_int32), ("shock_eps", C.c_double),
        ("eos", C.c_int32), ("exact_speeds", C.c_int32), ("corner", C.c_int32), ("pad2", C.c_int32),
    ]


class CtuBox(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("n", C.c_int32 * 3), ("level", C.c_int32), ("pad", C.c_int32),
                ("offset", C.c_int64)]


class CtuRegFace(C.Structure):
    _fields_ = [("box", C.c_int32), ("dir", C.c_int32), ("face", C.c_int32), ("pad", C.c_int32),
                ("tlo", C.c_int32 * 2), ("tn", C.c_int32 * 2), ("slot", C.c_int64)]


class CtuShape(C.Structure):
    _fields_ = [("tc_layout", C.c_int32), ("tc_chunk", C.c_int32), ("x_pencils", C.c_int32),
                ("xcd_order", C.c_int32), ("yz_segments", C.c_int32)]

    def as_dict(self):
        inv = {v: k for k, v in TC_LAYOUT.items()}
        return {"tc_layout": inv.get(self.tc_layout, self.tc_layout), "tc_chunk": self.tc_chunk,
                "x_pencils": self.x_pencils, "xcd_order": self.xcd_order, "yz_segments": self.yz_segments}


class CtuRefluxFace(C.Structure):
    _fields_ = [("box", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("k", C.c_int32), ("dir", C.c_int32),
                ("side", C.c_int32), ("nfine", C.c_int32), ("pad", C.c_int32), ("coarse_slot", C.c_int64),
                ("fine_slot", C.c_int64 * 4)]


_lib = None
_vp = C.c_void_p


def lib() -> C.CDLL:
    """Load libctu.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        L.ctu_plan_create.restype = C.c_int32
        L.ctu_plan_create.argtypes = [C.POINTER(CtuOpts), C.POINTER(CtuBox), C.c_int32, C.c_int32,
                                      C.POINTER(CtuRegFace), C.c_int32, C.POINTER(_vp)]
        L.ctu_plan_create_ex.restype = C.c_int32
        L.ctu_plan_create_ex.argtypes = [C.c_int32, C.c_uint32, C.POINTER(CtuOpts), C.POINTER(CtuBox), C.c_int32,
                                         C.c_int32, C.POINTER(CtuRegFace), C.c_int32, C.POINTER(CtuRefluxFace),
                                         C.c_int32, C.POINTER(_vp)]
        L.ctu_plan_set_workspace.restype = C.c_int32
        L.ctu_plan_set_workspace.argtypes = [_vp, _vp, C.c_int64]
        L.ctu_plan_device.restype = C.c_int32
        L.ctu_plan_device.argtypes = [_vp]
        L.ctu_step_static.restype = C.c_int32
        L.ctu_step_static.argtypes = [_vp] + [_vp] * 8 + [_vp]
        L.ctu_static_scratch_bytes.restype = C.c_int64
        L.ctu_static_scratch_bytes.argtypes = []
        L.ctu_measure_fma.restype = C.c_int32
        L.ctu_measure_fma.argtypes = [C.c_int32, C.c_int32, C.c_int32, _vp, C.POINTER(C.c_double)]
        L.ctu_measure_copy.restype = C.c_int32
        L.ctu_measure_copy.argtypes = [_vp, _vp, C.c_int64, C.POINTER(C.c_double)]
        L.ctu_plan_destroy.argtypes = [_vp]
        L.ctu_plan_state_elems.restype = C.c_int64
        L.ctu_plan_state_elems.argtypes = [_vp]
        L.ctu_plan_workspace_bytes.restype = C.c_int64
        L.ctu_plan_workspace_bytes.argtypes = [_vp]
        L.ctu_step.restype = C.c_int32
        L.ctu_step.argtypes = [_vp] + [_vp] * 8 + [_vp]
        L.ctu_step_graph_capture.restype = C.c_int32
        L.ctu_step_graph_capture.argtypes = [_vp] + [_vp] * 8 + [_vp]
        L.ctu_step_graph_launch.restype = C.c_int32
        L.ctu_step_graph_launch.argtypes = [_vp, _vp]
        L.ctu_cfl_rate.restype = C.c_int32
        L.ctu_cfl_rate.argtypes = [_vp, _vp, _vp, _vp]
        L.ctu_prim_to_cons.restype = C.c_int32
        L.ctu_prim_to_cons.argtypes = [_vp, _vp, _vp, _vp]
        L.ctu_cons_to_prim.restype = C.c_int32
        L.ctu_cons_to_prim.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.ctu_plan_set_reflux.restype = C.c_int32
        L.ctu_plan_set_reflux.argtypes = [_vp, C.POINTER(CtuRefluxFace), C.c_int32]
        L.ctu_reflux.restype = C.c_int32
        L.ctu_reflux.argtypes = [_vp, _vp, _vp, _vp]
        L.ctu_reflux_consume.restype = C.c_int32
        L.ctu_reflux_consume.argtypes = [_vp, _vp, _vp, _vp]
        L.ctu_hier_create.restype = C.c_int32
        L.ctu_hier_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(CtuBox),
                                      C.c_int32, C.POINTER(_vp)]
        L.ctu_hier_destroy.argtypes = [_vp]
        L.ctu_hier_fill_ghosts.restype = C.c_int32
        L.ctu_hier_fill_ghosts.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, C.c_double, _vp, _vp]
        L.ctu_hier_average_down.restype = C.c_int32
        L.ctu_hier_average_down.argtypes = [_vp, C.c_int32, _vp, _vp, _vp]
        L.ctu_hier_advance.restype = C.c_int32
        L.ctu_hier_advance.argtypes = [_vp, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(C.c_int32),
                                       C.POINTER(_vp), C.POINTER(_vp), _vp, _vp, _vp, _vp, _vp, _vp]
        L.ctu_hier_leaf_mask.restype = C.c_int32
        L.ctu_hier_leaf_mask.argtypes = [_vp, C.c_int32, _vp, _vp]
        L.ctu_hier_tag.restype = C.c_int32
        L.ctu_hier_tag.argtypes = [_vp, C.c_int32, _vp, C.c_int32, C.c_double, C.c_double, _vp, _vp, _vp]
        L.ctu_hier_next_dt.restype = C.c_int32
        L.ctu_hier_next_dt.argtypes = [_vp, _vp, _vp, C.c_double, C.c_double, C.POINTER(_vp), _vp]
        L.ctu_plan_set_leaf_mask.restype = C.c_int32
        L.ctu_plan_set_leaf_mask.argtypes = [_vp, _vp]
        L.ctu_plan_enable_timing.restype = C.c_int32
        L.ctu_plan_enable_timing.argtypes = [_vp, C.c_int32]
        L.ctu_plan_read_timing.restype = C.c_int32
        L.ctu_plan_read_timing.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.ctu_plan_set_shape.restype = C.c_int32
        L.ctu_plan_set_shape.argtypes = [_vp, C.POINTER(CtuShape)]
        L.ctu_plan_get_shape.restype = C.c_int32
        L.ctu_plan_get_shape.argtypes = [_vp, C.POINTER(CtuShape), C.POINTER(C.c_int32)]
        L.ctu_plan_autotune.restype = C.c_int32
        L.ctu_plan_autotune.argtypes = [_vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, C.POINTER(CtuShape),
                                        C.POINTER(C.c_double)]
        L.ctu_tune_cache_clear.restype = C.c_int32
        L.ctu_tune_cache_clear.argtypes = []
        L.ctu_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class CtuError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise CtuError(f"libctu error {rc}: {lib().ctu_last_error().decode()}")


def make_opts(dim=3, physics="mhd", precision="fp64", recon="ppm", predictor="char", wref="face", riemann="hlld",
              glm=True, gamma=5.0 / 3.0, dx=(1.0, 1.0, 1.0), glm_alpha=0.1, parabolic_mask=0, cooling=False,
              nu=0.0, eta=0.0, kappa_par=0.0, kappa_perp=0.0, tc_phi=0.0, cool_beta=0.5, T_floor=0.0,
              hyperbolic_off=False, shock_eps=0.0, eos="ideal", exact_speeds=False, corner="tn") -> CtuOpts:
    o = CtuOpts()
    o.dim = dim
    o.physics = {"mhd": MHD, "rmhd": RMHD}[physics]
    o.precision = {"fp64": FP64, "fp32": FP32}[precision]
    o.recon = RECON[recon]
    o.predictor = PRED[predictor]
    o.wref = WREF[wref]
    o.riemann = RIEMANN[riemann]
    o.glm = int(bool(glm))
    o.gamma = gamma
    for q in range(3):
        o.dx[q] = dx[q]
    o.glm_alpha = glm_alpha
    o.parabolic_mask = parabolic_mask
    o.cooling = int(bool(cooling))
    o.nu, o.eta, o.kappa_par, o.kappa_perp, o.tc_phi = nu, eta, kappa_par, kappa_perp, tc_phi
    o.cool_beta, o.T_floor = cool_beta, T_floor
    o.hyperbolic_off = int(bool(hyperbolic_off))
    o.shock_eps = shock_eps
    o.eos = EOS[eos]
    o.exact_speeds = int(bool(exact_speeds))
    o.corner = CORNER[corner]
    return o


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _need(name, t, dtype, numel, device, required=True, check_device=True):
    """Reject a buffer that the kernels would read or write out of range or
    misinterpret: wrong dtype, too few elements, not contiguous, not on the
    plan's device."""
    import torch

    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if check_device:
        _on_device(name, t, device)


def _on_device(name, t, device):
    if t is not None and (t.device.type != "cuda" or (device is not None and t.device.index != device)):
        raise ValueError(f"{name} must be a CUDA tensor on device {device}, got {t.device}")


def _refl_array(entries):
    n = len(entries)
    arr = (CtuRefluxFace * max(1, n))()
    for q, e in enumerate(entries):
        box, (i, j, k), d, side, cslot, fslots = e
        a = arr[q]
        a.box, a.i, a.j, a.k, a.dir, a.side = box, i, j, k, d, side
        a.nfine = len(fslots)
        a.coarse_slot = cslot
        for f, s in enumerate(fslots):
            a.fine_slot[f] = s
    return arr, n


class Plan:
    """A ctu_plan: boxes (lo, n, level, offset), ghosts, register faces,
    optionally the reflux table of this (coarse) level.  `device` is the HIP
    device (default: torch's current one); workspace="caller" leaves the
    workspace to a torch tensor that this object allocates and holds (the
    caller-owned path of the C ABI), "library" lets the library own it,
    "none" creates the plan without one (it then steps only through
    step_static).  level_dt: the boxes may lie on several levels, params
    hold the level-0 step and a level-l box steps by dt / 2^l."""

    def __init__(self, opts: CtuOpts, boxes, nghost: int, regfaces=None, reflux=None, device=None,
                 workspace="library", level_dt=False):
        L = lib()
        if workspace not in ("library", "caller", "none"):
            raise ValueError("workspace must be 'library', 'caller' or 'none'")
        if device is None:
            import torch

            # device_count() does not initialise the GPU; with none, the
            # library's option checks still run and the device is refused after
            device = torch.cuda.current_device() if torch.cuda.device_count() > 0 else 0
        nb = len(boxes)
        arr = (CtuBox * nb)()
        for q, b in enumerate(boxes):
            lo, n, level, offset = b
            for d in range(3):
                arr[q].lo[d] = lo[d]
                arr[q].n[d] = n[d]
            arr[q].level = level
            arr[q].offset = offset
        regs = regfaces or []
        rarr = (CtuRegFace * max(1, len(regs)))()
        for q, r in enumerate(regs):
            box, d, face, tlo, tn, slot = r
            rarr[q].box, rarr[q].dir, rarr[q].face = box, d, face
            rarr[q].tlo[0], rarr[q].tlo[1] = tlo
            rarr[q].tn[0], rarr[q].tn[1] = tn
            rarr[q].slot = slot
        self.opts = opts
        self.device = int(device)
        self.nslots = max([r[5] + r[4][0] * r[4][1] for r in regs], default=0)
        self._h = C.c_void_p()
        rf, nrf = _refl_array(reflux or [])
        flags = PLAN_CALLER_WORKSPACE if workspace in ("caller", "none") else 0
        if level_dt:
            flags |= PLAN_LEVEL_DT
        _check(L.ctu_plan_create_ex(self.device, flags, C.byref(opts), arr, nb, nghost, rarr if regs else None,
                                    len(regs), rf if nrf else None, nrf, C.byref(self._h)))
        self._ws = None
        if workspace == "caller":
            import torch

            nbytes = self.workspace_bytes
            # torch's allocator returns blocks aligned to at least 512 bytes
            self._ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=torch.device("cuda", self.device))
            _check(L.ctu_plan_set_workspace(self._h, C.c_void_p(self._ws.data_ptr()), self._ws.numel()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ctu_plan_destroy(h)
            self._h = None

    @property
    def state_elems(self) -> int:
        return int(lib().ctu_plan_state_elems(self._h))

    @property
    def workspace_bytes(self) -> int:
        return int(lib().ctu_plan_workspace_bytes(self._h))

    @property
    def dtype(self):
        import torch

        return torch.float32 if self.opts.precision == FP32 else torch.float64

    def _step_args(self, U_in, U_out, params, rate, L0, reg, dpp, fails, need_rate=True, need_reg=True):
        import torch

        se = self.state_elems
        dev = self.device
        args = [("U_in", U_in, self.dtype, se, True), ("U_out", U_out, self.dtype, se, True),
                ("params", params, torch.float64, 2, True), ("rate", rate, torch.float64, 1, need_rate),
                ("cool_L0", L0, self.dtype, se // 9, bool(self.opts.cooling)),
                ("reg", reg, torch.float64, 9 * self.nslots, need_reg and self.nslots > 0),
                ("dpp", dpp, torch.float64, 1, False), ("fails", fails, torch.int32, NFAIL, False)]
        for name, t, dt, n, req in args:
            _need(name, t, dt, n, dev, required=req, check_device=False)
        if U_in.data_ptr() == U_out.data_ptr():
            raise ValueError("U_out must not alias U_in")
        for name, t, _, _, _ in args:
            _on_device(name, t, dev)

    def step(self, U_in, U_out, params, rate, L0=None, reg=None, dpp=None, fails=None, stream=None):
        self._step_args(U_in, U_out, params, rate, L0, reg, dpp, fails)
        _check(lib().ctu_step(self._h, _ptr(U_in), _ptr(U_out), _ptr(params), _ptr(L0), _ptr(reg), _ptr(rate),
                              _ptr(dpp), _ptr(fails), _stream(stream)))

    def step_static(self, U_in, U_out, params, rate, L0=None, reg=None, dpp=None, fails=None, stream=None):
        """ctu_step_static: the step on the library's fixed per-GPU scratch
        array (no allocation, no plan workspace needed)."""
        self._step_args(U_in, U_out, params, rate, L0, reg, dpp, fails)
        _check(lib().ctu_step_static(self._h, _ptr(U_in), _ptr(U_out), _ptr(params), _ptr(L0), _ptr(reg),
                                     _ptr(rate), _ptr(dpp), _ptr(fails), _stream(stream)))

    def graph_capture(self, U_in, U_out, params, rate, L0=None, reg=None, dpp=None, fails=None, stream=None):
        self._step_args(U_in, U_out, params, rate, L0, reg, dpp, fails)
        self._graph_args = (U_in, U_out, params, rate, L0, reg, dpp, fails)  # kept alive for the replays
        _check(lib().ctu_step_graph_capture(self._h, _ptr(U_in), _ptr(U_out), _ptr(params), _ptr(L0), _ptr(reg),
                                            _ptr(rate), _ptr(dpp), _ptr(fails), _stream(stream)))

    def graph_launch(self, stream=None):
        _check(lib().ctu_step_graph_launch(self._h, _stream(stream)))

    def cfl_rate(self, U, rate, stream=None):
        import torch

        _need("U", U, self.dtype, self.state_elems, self.device)
        _need("rate", rate, torch.float64, 1, self.device)
        _check(lib().ctu_cfl_rate(self._h, _ptr(U), _ptr(rate), _stream(stream)))

    def prim_to_cons(self, V, U, stream=None):
        _need("V", V, self.dtype, self.state_elems, self.device)
        _need("U", U, self.dtype, self.state_elems, self.device)
        _check(lib().ctu_prim_to_cons(self._h, _ptr(V), _ptr(U), _stream(stream)))

    def cons_to_prim(self, U, V, fails=None, stream=None):
        import torch

        _need("U", U, self.dtype, self.state_elems, self.device)
        _need("V", V, self.dtype, self.state_elems, self.device)
        _need("fails", fails, torch.int32, NFAIL, self.device, required=False)
        _check(lib().ctu_cons_to_prim(self._h, _ptr(U), _ptr(V), _ptr(fails), _stream(stream)))

    def set_reflux(self, entries):
        arr, n = _refl_array(entries)
        _check(lib().ctu_plan_set_reflux(self._h, arr, n))

    def enable_timing(self, on: bool = True):
        _check(lib().ctu_plan_enable_timing(self._h, int(on)))

    def read_timing(self):
        """(total ms per stage as a dict, number of recorded steps)."""
        ms = (C.c_double * NSTAGE)()
        n = C.c_int32()
        _check(lib().ctu_plan_read_timing(self._h, ms, C.byref(n)))
        return dict(zip(STAGES, list(ms))), n.value

    def _reflux_args(self, U, reg):
        import torch

        _need("U", U, self.dtype, self.state_elems, self.device)
        # the table's slots are not known here; reg must at least be FP64 on the device
        _need("reg", reg, torch.float64, 9, self.device)

    def reflux(self, U, reg, stream=None):
        self._reflux_args(U, reg)
        _check(lib().ctu_reflux(self._h, _ptr(U), _ptr(reg), _stream(stream)))

    def reflux_consume(self, U, reg, stream=None):
        self._reflux_args(U, reg)
        _check(lib().ctu_reflux_consume(self._h, _ptr(U), _ptr(reg), _stream(stream)))

    def set_leaf_mask(self, leaf):
        """uint8 tensor in the cool_L0 layout (kept alive by the caller) or None"""
        import torch

        _need("leaf", leaf, torch.uint8, self.state_elems // 9, self.device, required=False)
        self._leaf = leaf
        _check(lib().ctu_plan_set_leaf_mask(self._h, _ptr(leaf)))

    def set_shape(self, tc_layout="auto", tc_chunk=0, x_pencils=0, xcd_order=1, yz_segments=0):
        sh = CtuShape(TC_LAYOUT[tc_layout] if isinstance(tc_layout, str) else int(tc_layout), int(tc_chunk),
                      int(x_pencils), int(xcd_order), int(yz_segments))
        _check(lib().ctu_plan_set_shape(self._h, C.byref(sh)))

    def get_shape(self):
        """(shape dict, number of boxes on the flat t^n layout)"""
        sh = CtuShape()
        nf = C.c_int32()
        _check(lib().ctu_plan_get_shape(self._h, C.byref(sh), C.byref(nf)))
        return sh.as_dict(), nf.value

    def autotune(self, U_in, U_out, params, L0=None, reps=3, stream=None):
        """Time candidate shapes on these buffers, keep the fastest; returns
        (shape dict, ms per step).  U_out is overwritten."""
        sh = CtuShape()
        ms = C.c_double()
        self._step_args(U_in, U_out, params, None, L0, None, None, None, need_rate=False, need_reg=False)
        _check(lib().ctu_plan_autotune(self._h, _ptr(U_in), _ptr(U_out), _ptr(params), _ptr(L0), int(reps),
                                       _stream(stream), C.byref(sh), C.byref(ms)))
        return sh.as_dict(), ms.value


def tune_cache_clear():
    _check(lib().ctu_tune_cache_clear())


def measure_fma(precision: str = "fp32", nblocks: int = 4096, iters: int = 256) -> float:
    """TFLOP/s of the library's FMA-chain kernel on the current device
    (ctu_measure_fma); the output buffer is a torch tensor."""
    import torch

    prec = {"fp64": FP64, "fp32": FP32}[precision]
    out = torch.empty(int(nblocks) * 256, dtype=torch.float32 if precision == "fp32" else torch.float64,
                      device="cuda")
    t = C.c_double()
    _check(lib().ctu_measure_fma(prec, int(nblocks), int(iters), _ptr(out), C.byref(t)))
    return t.value


def measure_copy(nbytes: int = 2 << 30) -> float:
    """GB/s (read + write) of the library's float4 copy kernel over two
    torch buffers of `nbytes` (ctu_measure_copy)."""
    import torch

    n = int(nbytes) // 16 * 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    g = C.c_double()
    _check(lib().ctu_measure_copy(_ptr(src), _ptr(dst), n * 4, C.byref(g)))
    return g.value


class Hier:
    """A ctu_hier: the boxes of every level of a ratio-2 hierarchy on the
    periodic cube of `base` level-0 cells; levels[l] = list of
    (lo, n, offset) in level-l indices."""

    def __init__(self, precision: str, base: int, levels, nghost: int):
        L = lib()
        flat = [(lo, n, lev, off) for lev, boxes in enumerate(levels) for (lo, n, off) in boxes]
        arr = (CtuBox * max(1, len(flat)))()
        for q, (lo, n, lev, off) in enumerate(flat):
            for d in range(3):
                arr[q].lo[d] = lo[d]
                arr[q].n[d] = n[d]
            arr[q].level = lev
            arr[q].offset = off
        nb = (C.c_int32 * len(levels))(*[len(b) for b in levels])
        self.nlev = len(levels)
        self._h = C.c_void_p()
        _check(L.ctu_hier_create({"fp64": FP64, "fp32": FP32}[precision], base, len(levels), nb, arr, nghost,
                                 C.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ctu_hier_destroy(h)
            self._h = None

    def fill_ghosts(self, level, U, Uc_old=None, Uc_new=None, alpha=0.0, missing=None, stream=None):
        _check(lib().ctu_hier_fill_ghosts(self._h, level, _ptr(U), _ptr(Uc_old), _ptr(Uc_new), float(alpha),
                                          _ptr(missing), _stream(stream)))

    def average_down(self, fine_level, U_fine, U_coarse, stream=None):
        _check(lib().ctu_hier_average_down(self._h, fine_level, _ptr(U_fine), _ptr(U_coarse), _stream(stream)))

    def advance(self, plans, U_a, U_b, cur, params, reg, rate, dpp=None, L0=None, fails=None, missing=None,
                stream=None):
        """One level-0 step with subcycling; `cur` (list of 0/1 per level) is
        updated in place to name the buffers holding the new states.  rate
        (and dpp) hold one double per level; L0 is None or a per-level list."""
        n = self.nlev
        if len(plans) != n or len(U_a) != n or len(U_b) != n or len(params) != n or len(cur) != n:
            raise ValueError("plans, U_a, U_b, params and cur need one entry per level")
        for l, p in enumerate(plans):
            _need(f"U_a[{l}]", U_a[l], p.dtype, p.state_elems, p.device)
            _need(f"U_b[{l}]", U_b[l], p.dtype, p.state_elems, p.device)
        P = (_vp * n)(*[p._h for p in plans])
        A = (_vp * n)(*[C.c_void_p(t.data_ptr()) for t in U_a])
        B = (_vp * n)(*[C.c_void_p(t.data_ptr()) for t in U_b])
        cu = (C.c_int32 * n)(*cur)
        prm = (_vp * n)(*[C.c_void_p(t.data_ptr()) for t in params])
        l0 = None if L0 is None else (_vp * n)(*[_ptr(t) for t in L0])
        _check(lib().ctu_hier_advance(self._h, P, A, B, cu, prm, l0, _ptr(reg), _ptr(rate), _ptr(dpp), _ptr(fails),
                                      _ptr(missing), _stream(stream)))
        for l in range(n):
            cur[l] = int(cu[l])

    def leaf_mask(self, level, leaf, stream=None):
        _check(lib().ctu_hier_leaf_mask(self._h, level, _ptr(leaf), _stream(stream)))

    def tag(self, level, U, var, eps, chi_r, tags, ntag=None, stream=None):
        _check(lib().ctu_hier_tag(self._h, level, _ptr(U), var, float(eps), float(chi_r), _ptr(tags), _ptr(ntag),
                                  _stream(stream)))

    def next_dt(self, rate, dpp, cfl, eps_c, params, stream=None):
        prm = (_vp * self.nlev)(*[C.c_void_p(t.data_ptr()) for t in params])
        _check(lib().ctu_hier_next_dt(self._h, _ptr(rate), _ptr(dpp), float(cfl), float(eps_c), prm, _stream(stream)))
