"""Benchmark: zone-updates/s of the CTU-GLM step on one MI355X, FP32 batched
(HIP-graph replay, autotuned launch shapes) against FP64 plain (eager
launches, default shapes), on the five workloads of the build:

  C2 (headline)  3D ideal MHD 256^3 periodic, PPM characteristic + HLLD + GLM
  C1             2D ideal MHD 128^2, MC-linear characteristic + HLLD + GLM, FP64, 10 steps
  C3             3D AMR batch, 3 levels at ratio 2, 1,457 patches of 16-32 cells (FP32
                 batched per level + reflux; FP64 one plan per patch; the subcycled cycle)
  C4             3D relativistic MHD 192^3 jets and blobs, MUSCL-Hancock + MC + HLL + GLM
  C5             3D non-ideal MHD 256^3 (viscosity, resistivity, saturated anisotropic
                 conduction, stiff cooling), PPM + HLLD + GLM

plus option-set variants of C2 and C4.  Every timed result carries its
relative L1 error (and largest single-cell error) against the FP64 oracle on
sampled sub-boxes of the same input, computed by the cpu_baseline leg, which
also times the oracle on the host cores.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-amr]
                  [--no-variants] [--legs c2,c1,c3,c4,c5] [--shape L,C,P,X[,S]]

A step is one pass of the whole hot path (primitive recovery, t^n fluxes and
corner-coupling increments, normal predictors, time-centred Riemann solves,
update, split sources, FP64 CFL reduction, FP64 flux registers on AMR
levels) over inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec per CTU step (FP32 batched vs FP64 plain) + achieved HBM GB/s"
NG = 4
# the AMR legs' ghost width: the PPM CTU stencil's minimum (the plan refuses
# fewer); on 16-32 cell patches a fourth layer would add ~30 % more ghost
# cells to fill and to recover
NG_AMR = 3

# Algorithmic FLOP per interior zone (add, mul, div, sqrt, transcendental;
# FMA = 2) of what each kernel computes, from the op-counting build of the
# FP64 oracle (profiles/oracle_opcount.md, `python oracle/opcount.py`):
# prim = primitive recovery, tcouple = the t^n Godunov fluxes with their
# increments and, with parabolic terms, the half-step state; pdiv / pflux =
# the parabolic fluxes Pi^n (with their divergence) and Pi^{n+1/2}; for
# the relativistic workload also the sweeps (MUSCL-Hancock predictor and
# coupling, time-centred solves, a third each, and the update in the last
# one).  The characteristic-tracing sweeps are not listed: the oracle's
# predictor projects with dense 7 x 7 eigenvector products where the kernels
# use the sparse closed forms, so its count is not the method's minimum; nor
# are the relativistic inversions, whose oracle form is a bisection.
ALG_FLOP = {"C1": {"prim": 20.0, "tcouple": 943.0}, "C2": {"prim": 20.0, "tcouple": 1354.0},
            "C4": {"tcouple": 1696.0, "sweep_x": 1190.0, "sweep_y": 1190.0, "sweep_z": 1351.0},
            "C5": {"prim": 20.0, "tcouple": 1520.0, "pdiv": 536.0, "pflux": 594.0}}
# HBM bytes per launch of the FP32 256^3 t^n kernel, FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (KiB x 1024): a plain 1 GiB device copy (bench.py
# --copy-calibration) reads back as 524,308 KiB of FETCH_SIZE and 1,048,576
# KiB of WRITE_SIZE, hence the factors (profiles/c2_mhd3d_256_ppm_hlld.md).
# None once the kernel has changed since the counters were taken.
TCOUPLE_TRAFFIC_BYTES = (530399 * 2 + 2085694) * 1024
# the launch shape those counters were taken with (bench.py --shape tiles,4,16,1,2)
PROFILE_SHAPE = {"tc_layout": "tiles", "tc_chunk": 4, "xcd_order": 1}
# Step parameters of the workloads (dt and c_h; C1's ten chained steps; C5's
# hyperbolic step that sets the cooling times), from the FP64 oracle's CFL
# rate of each initial state, written by tests/golden/make_refs.py: the timed
# steps and the oracle comparisons use the same values, none taken from the
# GPU.
STEP_PARAMS = os.path.join(ROOT, "tests", "golden", "step_params.json")
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3           # published FP32 vector peak (packed FP32 issue)
PEAK_FP32_UNPACKED_TFLOPS = 78.6   # one FP32 lane op per VALU lane per cycle (no packed FP32 emitted)
PEAK_FP64_TFLOPS = 78.6


_STEP = None


def step_params():
    global _STEP
    if _STEP is None:
        with open(STEP_PARAMS) as f:
            _STEP = json.load(f)
    return _STEP


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle cpu_baseline leg (and the L1 figures)")
    ap.add_argument("--no-amr", action="store_true", help="skip the AMR leg (C3)")
    ap.add_argument("--no-variants", action="store_true", help="skip the option-set variants")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes for the FP32 plans")
    ap.add_argument("--no-per-patch", action="store_true",
                    help="skip C3's FP64 one-plan-per-patch path (thousands of launches; profiling aid)")
    ap.add_argument("--legs", default="c2,c1,c3,c4,c5", help="workloads to run (profiling aid)")
    ap.add_argument("--shape", default=None,
                    help="force the launch shape of the C2 FP32 plan instead of tuning it: "
                         "LAYOUT,CHUNK,PENCILS,XCD[,YZSEGMENTS] (e.g. tiles,4,16,1,2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of 1 GiB: under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE give the scale of the HBM byte counters."""
    import torch

    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))


# ---------------------------------------------------------------------------
# timing helpers (HIP events on the launch stream)
# ---------------------------------------------------------------------------


def timed(fn, K, W, s):
    import torch

    with torch.cuda.stream(s):
        for _ in range(W):
            fn()
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record(s)
        for _ in range(K):
            fn()
        e1.record(s)
    s.synchronize()
    return e0.elapsed_time(e1) / K


class StepBufs:
    """Device buffers of one plan's step."""

    def __init__(self, dev, nslots=0):
        import torch

        self.rate = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dpp = torch.zeros(1, dtype=torch.float64, device=dev)
        self.fails = torch.zeros(5, dtype=torch.int32, device=dev)
        self.reg = torch.zeros(max(1, 9 * nslots), dtype=torch.float64, device=dev) if nslots else None


def run_plan(plan, Uin, Uout, params, b, K, W, s, L0=None, graph=True, stages=True):
    """Time K steps (graph replay or eager launches); then, with `stages`, the
    same K steps launched eagerly with HIP events around every kernel.
    Returns (ms per step, {kernel: ms per launch})."""
    if graph:
        import torch

        with torch.cuda.stream(s):
            plan.graph_capture(Uin, Uout, params, b.rate, L0=L0, reg=b.reg, dpp=b.dpp, fails=b.fails, stream=s)
        ms = timed(lambda: plan.graph_launch(stream=s), K, W, s)
    else:
        ms = timed(lambda: plan.step(Uin, Uout, params, b.rate, L0=L0, reg=b.reg, dpp=b.dpp, fails=b.fails, stream=s),
                   K, W, s)
    assert b.fails.sum().item() == 0, b.fails
    per = {}
    if stages:
        plan.enable_timing(True)
        import torch

        with torch.cuda.stream(s):
            for _ in range(K):
                plan.step(Uin, Uout, params, b.rate, L0=L0, reg=b.reg, dpp=b.dpp, fails=b.fails, stream=s)
        s.synchronize()
        st, n = plan.read_timing()
        plan.enable_timing(False)
        per = {k: v / max(n, 1) for k, v in st.items() if v > 0}
    return ms, per


def result(ms, zones, alg_bytes_zone, per=None, shape=None):
    out = {"ms_per_step": ms, "zone_updates_per_s": zones / (ms * 1e-3),
           "hbm_alg_GBs": alg_bytes_zone * zones / (ms * 1e-3) / 1e9, "alg_bytes_per_zone": alg_bytes_zone}
    out["hbm_frac"] = out["hbm_alg_GBs"] / PEAK_HBM_GBS
    if per:
        out["kernel_ms"] = per
    if shape is not None:
        out["shape"] = shape
    return out


def kernel_roofline(cfg, per, zones, dtype):
    """ALU roofline of the dominant kernel with an algorithmic FLOP count."""
    if not per:
        return None
    dom = max(per, key=per.get)
    fpz = ALG_FLOP.get(cfg, {}).get(dom)
    peak = PEAK_FP32_TFLOPS if dtype == "f32" else PEAK_FP64_TFLOPS
    r = {"bound": "alu", "kernel": dom, "avg_ms": per[dom], "peak": peak, "unit": "TFLOP/s"}
    if fpz is None:
        r.update(achieved=None, frac=None,
                 note="no algorithmic FLOP count for this kernel (see ALG_FLOP)")
        return r
    achieved = fpz * zones / (per[dom] * 1e-3) / 1e12
    r.update(achieved=achieved, frac=achieved / peak, alg_flop_per_zone=fpz)
    if dtype == "f32":
        r.update(peak_unpacked=PEAK_FP32_UNPACKED_TFLOPS, frac_unpacked=achieved / PEAK_FP32_UNPACKED_TFLOPS)
    return r


def ghost_bytes(n, esize, dim=3):
    """Algorithmic bytes per zone: read U^n on the ghosted box, write U^{n+1}."""
    return 9 * esize * ((n + 2 * NG) / n) ** dim + 9 * esize


# ---------------------------------------------------------------------------
# sampled sub-boxes for the L1 figures
# ---------------------------------------------------------------------------


def origins(n, m, dim):
    if dim == 2:
        return [(0, 0), (n - m, n - m), (n // 2 - 5, 7), (3, n // 3)]
    return [(0, 0, 0), (n - m, n - m, n - m), (n - m, 0, n // 2), (n // 2 - 3, n // 3 + 1, 0),
            (n // 4, n - m, n // 5), (7, n // 2, n - m)]


def subbox(T, N, lo, m, dim):
    """Host FP64 copy of the ghosted sub-box with interior [lo, lo + m) of a
    flat device state of one ghosted box of extent N per axis."""
    import numpy as np

    if dim == 2:
        v = T.view(9, 1, N, N)[:, :, lo[1]:lo[1] + m + 2 * NG, lo[0]:lo[0] + m + 2 * NG]
    else:
        v = T.view(9, N, N, N)[:, lo[2]:lo[2] + m + 2 * NG, lo[1]:lo[1] + m + 2 * NG, lo[0]:lo[0] + m + 2 * NG]
    return np.ascontiguousarray(v.cpu().numpy().astype(np.float64))


def subbox_cells(T, N, lo, m):
    import numpy as np

    v = T.view(N, N, N)[lo[2]:lo[2] + m + 2 * NG, lo[1]:lo[1] + m + 2 * NG, lo[0]:lo[0] + m + 2 * NG]
    return np.ascontiguousarray(v.cpu().numpy().astype(np.float64))


def parity_norms(pairs, ch, physics, dim, ng=NG):
    """(max over variables of sum|got - ref| / S_q, max over variables of
    max|got - ref| / M_q) over the interiors of (got, ref) sub-box pairs:
    S_q = sum|ref_q|, M_q = max|ref_q|; psi against c_h |B| / 3; for RMHD
    momentum against E + D and each B component against |B| / 3 where those
    are larger (the resting background makes them vanish in places)."""
    import numpy as np

    def inner(a):
        if dim == 2:
            return a[:, :, ng:-ng, ng:-ng].reshape(9, -1)
        return a[:, ng:-ng, ng:-ng, ng:-ng].reshape(9, -1)

    g = np.concatenate([inner(a) for a, _ in pairs], axis=1)
    r = np.concatenate([inner(b) for _, b in pairs], axis=1)
    d = np.abs(g - r)
    l1 = np.abs(r).sum(axis=1)
    mx = np.abs(r).max(axis=1)
    bmag = np.sqrt((r[5:8] ** 2).sum(axis=0))
    if physics == "rmhd":
        ms = np.abs(r[4]) + np.abs(r[0])
        for q in (1, 2, 3):
            l1[q], mx[q] = max(l1[q], ms.sum()), max(mx[q], ms.max())
        for q in (5, 6, 7):
            l1[q], mx[q] = max(l1[q], bmag.sum() / 3), max(mx[q], bmag.max() / 3)
    l1[8], mx[8] = max(l1[8], ch * bmag.sum() / 3), max(mx[8], ch * bmag.max() / 3)
    return float((d.sum(axis=1) / np.maximum(l1, 1e-300)).max()), float((d.max(axis=1) / np.maximum(mx, 1e-300)).max())


class Samples:
    """What the oracle needs to recompute a timed result on sub-boxes: the
    oracle options, dt, c_h, the input sub-boxes as primitive fields from the
    seeded generator (the oracle forms the conserved state itself), cooling
    coefficients, and the GPU's output on the same sub-boxes."""

    def __init__(self):
        self.items = {}

    def add(self, leg, okw, dx, dt, ch, ins, outs, L0s=None, physics="mhd", dim=3, chain=None, ng=NG):
        self.items[leg] = dict(okw=okw, dx=dx, dt=dt, ch=ch, ins=ins, outs=outs, L0s=L0s, physics=physics, dim=dim,
                               chain=chain, ng=ng)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------


def leg_c2(args, dev, s, samples):
    import torch

    from paper_1110_0740_amd import ctu, inputs as I

    n = 256
    K, W = args.steps, args.warmup
    log(f"C2: generating {n}^3 inputs on the GPU")
    V64, meta = I.mhd3d_fields_torch(n=n, ng=NG, seed=2000, device=dev)
    dx, gamma = meta["dx"], meta["gamma"]
    N, zones = n + 2 * NG, n ** 3
    box = [((0, 0, 0), (n, n, n), 0, 0)]
    okw = dict(recon="ppm", riemann="hlld")
    p64 = ctu.Plan(ctu.make_opts(dim=3, gamma=gamma, dx=dx, precision="fp64", **okw), box, NG)
    U64 = torch.empty(9 * N ** 3, dtype=torch.float64, device=dev)
    p64.prim_to_cons(V64.reshape(-1), U64)
    org = origins(n, 16, 3)
    ins = [subbox(V64.reshape(-1), N, lo, 16, 3) for lo in org]
    # the sub-boxes the cpu_baseline leg times the oracle on (C2's own input)
    timing_boxes = [subbox(V64.reshape(-1), N, lo, 48, 3) for lo in ((0, 0, 0), (100, 60, 180), (200, 200, 30))]
    del V64
    b = StepBufs(dev)
    sp = step_params()["C2"]
    dt, ch = sp["dt"], sp["ch"]
    params = torch.tensor([dt, ch], dtype=torch.float64, device=dev)
    outs = {}
    # FP32 batched: tuned shape, graph replay
    log("C2: FP32 batched (autotune, graph)")
    p32 = ctu.Plan(ctu.make_opts(dim=3, gamma=gamma, dx=dx, precision="fp32", **okw), box, NG)
    U32 = U64.to(torch.float32)
    Uo32 = torch.zeros_like(U32)
    if args.shape:
        f = args.shape.split(",")
        p32.set_shape(tc_layout=f[0], tc_chunk=int(f[1]), x_pencils=int(f[2]), xcd_order=int(f[3]),
                      yz_segments=int(f[4]) if len(f) > 4 else 0)
    elif not args.no_autotune:
        p32.autotune(U32, Uo32, params, reps=20, stream=s)
    shape, flat = p32.get_shape()
    ms, per = run_plan(p32, U32, Uo32, params, b, K, W, s)
    r32 = result(ms, zones, ghost_bytes(n, 4), per, shape)
    r32["flat_boxes"] = flat
    # FP64 plain: default shape, eager launches
    log("C2: FP64 plain (eager)")
    Uo64 = torch.zeros_like(U64)
    ms64, per64 = run_plan(p64, U64, Uo64, params, b, K, W, s, graph=False)
    r64 = result(ms64, zones, ghost_bytes(n, 8), per64)
    samples.add("c2_fp32", okw, dx, dt, ch, ins, [subbox(Uo32, N, lo, 16, 3) for lo in org])
    samples.add("c2_fp64", okw, dx, dt, ch, ins, [subbox(Uo64, N, lo, 16, 3) for lo in org])
    out = {"fp32_batched": r32, "fp64_plain": r64, "zones": zones, "dt": dt, "c_h": ch}
    out["fp32_batched"]["roofline"] = kernel_roofline("C2", per, zones, "f32")
    variants = None
    if not args.no_variants:
        variants = c2_variants(args, dev, s, U64, ins[:3], params, b, dx, gamma, samples)
    del Uo64, Uo32, U32
    return out, variants, timing_boxes, (dx, gamma, dt, ch)


def c2_variants(args, dev, s, U64, ins, params, b, dx, gamma, samples):
    """The C2 workload under the widened option sets: the App. B hybrid,
    Rusanov, HLLC and Roe solvers, the MT corner coupling (FP32, tuned,
    graph-replayed)."""
    import torch

    from paper_1110_0740_amd import ctu

    n, N = 256, 256 + 2 * NG
    K, W = args.steps, args.warmup
    box = [((0, 0, 0), (n, n, n), 0, 0)]
    out = {}
    org = origins(n, 16, 3)[:3]
    variants = {"shock_hybrid": dict(riemann="hlld", shock_eps=5.0), "rusanov": dict(riemann="rusanov"),
                "hllc": dict(riemann="hllc"), "roe": dict(riemann="roe"), "mt_corner": dict(riemann="hlld", corner="mt")}
    for name, kw in variants.items():
        log(f"C2 variant {name}")
        p = ctu.Plan(ctu.make_opts(dim=3, recon="ppm", gamma=gamma, dx=dx, precision="fp32", **kw), box, NG)
        U32 = U64.to(torch.float32)
        Uo = torch.zeros_like(U32)
        if not args.no_autotune:
            p.autotune(U32, Uo, params, reps=3, stream=s)
        ms, _ = run_plan(p, U32, Uo, params, b, K, W, s, stages=False)
        out[name] = result(ms, n ** 3, ghost_bytes(n, 4), shape=p.get_shape()[0])
        samples.add(f"c2_{name}", dict(recon="ppm", **kw), dx, float(params[0]), float(params[1]), ins,
                    [subbox(Uo, N, lo, 16, 3) for lo in org])
        del p, U32, Uo
    return out


def leg_peaks():
    """The rates this build reaches on the device (library kernels): FP32 and
    FP64 FMA chains, and a float4 device copy of 2 GiB."""
    from paper_1110_0740_amd import ctu

    log("peaks: FMA chains and device copy")
    return {"valu_fp32_fma_TFLOPs": ctu.measure_fma("fp32"), "valu_fp64_fma_TFLOPs": ctu.measure_fma("fp64"),
            "hbm_copy_GBs": ctu.measure_copy(2 << 30),
            "note": "FP32 as every kernel of this build: single-lane FMAs, no packed FP32"}


def leg_c1(args, dev, s, samples):
    """2D 128^2 FP64, 10 CTU steps at CFL 0.4: timed as repeated steps (eager
    and graph); the L1 figure compares 10 chained steps (GPU ghosts refilled
    periodically on the device between steps), both sides driven by the
    oracle's stored dt sequence."""
    import numpy as np
    import torch

    from paper_1110_0740_amd import ctu, inputs as I

    n = 128
    K, W = args.steps, args.warmup
    V, meta = I.mhd2d_fields(n=n, ng=NG, seed=1000)
    okw = dict(recon="lin_mc", riemann="hlld")
    plan = ctu.Plan(ctu.make_opts(dim=2, gamma=meta["gamma"], dx=meta["dx"], precision="fp64", **okw),
                    [((0, 0, 0), (n, n, 1), 0, 0)], NG)
    Vd = torch.from_numpy(V.reshape(-1)).to(dev)
    U = torch.empty_like(Vd)
    plan.prim_to_cons(Vd, U)
    b = StepBufs(dev)
    chain = step_params()["C1"]
    dt, ch = chain["dt"][0], chain["ch"][0]
    params = torch.tensor([dt, ch], dtype=torch.float64, device=dev)
    Uo = U.clone()
    log("C1: FP64 plain (eager, default shape), then batched (tuned shape, graph)")
    ms_e, per = run_plan(plan, U, Uo, params, b, K, W, s, graph=False)
    if not args.no_autotune:
        plan.autotune(U, Uo, params, reps=20, stream=s)
    ms_g, per_g = run_plan(plan, U, Uo, params, b, K, W, s)
    zones = n * n
    out = {"fp64_plain": result(ms_e, zones, ghost_bytes(n, 8, 2), per),
           "fp64_batched": result(ms_g, zones, ghost_bytes(n, 8, 2), per_g, plan.get_shape()[0]), "zones": zones}
    out["fp64_plain"]["roofline"] = kernel_roofline("C1", per, zones, "f64")
    out["fp64_batched"]["roofline"] = kernel_roofline("C1", per_g, zones, "f64")
    # 10 chained steps for the L1 figure, with the oracle's dt sequence
    cur, nxt = U.clone(), torch.empty_like(U)
    dts = list(zip(chain["dt"], chain["ch"]))
    for dt, ch in dts:
        params.copy_(torch.tensor([dt, ch], dtype=torch.float64))
        plan.step(cur, nxt, params, b.rate, fails=b.fails)
        g = nxt.view(9, 1, n + 2 * NG, n + 2 * NG)
        g[..., :NG, :] = g[..., n:n + NG, :]
        g[..., n + NG:, :] = g[..., NG:2 * NG, :]
        g[..., :, :NG] = g[..., :, n:n + NG]
        g[..., :, n + NG:] = g[..., :, NG:2 * NG]
        torch.cuda.synchronize()
        cur, nxt = nxt, cur
    assert b.fails.sum().item() == 0
    samples.add("c1_fp64_10steps", okw, meta["dx"], None, None, [V], [cur.cpu().numpy().reshape(V.shape)], dim=2,
                chain=dts)
    return out


def leg_c4(args, dev, s, samples):
    import torch

    from paper_1110_0740_amd import ctu, inputs as I

    n = 192
    K, W = args.steps, args.warmup
    log("C4: generating 192^3 relativistic inputs")
    V, meta = I.rmhd3d_fields(n=n, ng=NG, seed=4000)
    Vd = torch.from_numpy(V.reshape(-1)).to(dev)
    del V
    N, zones = n + 2 * NG, n ** 3
    box = [((0, 0, 0), (n, n, n), 0, 0)]
    out, variants = {}, {}
    b = StepBufs(dev)
    org = origins(n, 12, 3)[:4]
    ins = [subbox(Vd, N, lo, 12, 3) for lo in org]
    for eos, xs, rs in (("ideal", False, "hll"), ("tm", False, "hll"), ("ideal", True, "hll"),
                        ("ideal", False, "hllc"), ("ideal", False, "hlld")):
        main = (eos, xs, rs) == ("ideal", False, "hll")
        if not main and args.no_variants:
            continue
        name = f"rmhd192_{eos}" + ("_exact_speeds" if xs else "") + ("" if rs == "hll" else "_" + rs)
        log(f"C4: {name}")
        okw = dict(physics="rmhd", predictor="mh", recon="lin_mc", riemann=rs, eos=eos, exact_speeds=xs)
        kw = dict(dim=3, gamma=meta["gamma"], dx=meta["dx"], **okw)
        p64 = ctu.Plan(ctu.make_opts(precision="fp64", **kw), box, NG)
        U64 = torch.empty_like(Vd)
        p64.prim_to_cons(Vd, U64)
        sp = step_params()["C4"][name]
        dt, ch = sp["dt"], sp["ch"]
        params = torch.tensor([dt, ch], dtype=torch.float64, device=dev)
        p = ctu.Plan(ctu.make_opts(precision="fp32", **kw), box, NG)
        U32 = U64.to(torch.float32)
        Uo = torch.zeros_like(U32)
        if not args.no_autotune:
            p.autotune(U32, Uo, params, reps=3, stream=s)
        ms, per = run_plan(p, U32, Uo, params, b, K, W, s, stages=main)
        r = result(ms, zones, ghost_bytes(n, 4), per, p.get_shape()[0])
        samples.add(f"c4_{name}_fp32", okw, meta["dx"], dt, ch, ins, [subbox(Uo, N, lo, 12, 3) for lo in org],
                    physics="rmhd")
        if main:
            r["roofline"] = kernel_roofline("C4", per, zones, "f32")
            out["fp32_batched"] = r
            log("C4: FP64 plain (eager)")
            Uo64 = torch.zeros_like(U64)
            ms64, per64 = run_plan(p64, U64, Uo64, params, b, K, W, s, graph=False)
            out["fp64_plain"] = result(ms64, zones, ghost_bytes(n, 8), per64)
            samples.add(f"c4_{name}_fp64", okw, meta["dx"], dt, ch, ins, [subbox(Uo64, N, lo, 12, 3) for lo in org],
                        physics="rmhd")
            del Uo64
        else:
            variants[name] = r
        del p, p64, U32, Uo, U64
    out["zones"] = zones
    return out, variants


def leg_c5(args, dev, s, samples):
    import torch

    from paper_1110_0740_amd import ctu, inputs as I

    n = 256
    K, W = args.steps, args.warmup
    log("C5: generating 256^3 non-ideal inputs and cooling coefficients")
    V, meta = I.mhd3d_fields_torch(n=n, ng=NG, seed=5000, device=dev)
    G, dx = meta["gamma"], meta["dx"]
    N, zones = n + 2 * NG, n ** 3
    box = [((0, 0, 0), (n, n, n), 0, 0)]
    coef = I.nonideal_coeffs(5001)
    b = StepBufs(dev)
    hyp = ctu.Plan(ctu.make_opts(dim=3, gamma=G, dx=dx, precision="fp64", recon="ppm", riemann="hlld"), box, NG)
    U64 = torch.empty(9 * N ** 3, dtype=torch.float64, device=dev)
    hyp.prim_to_cons(V.reshape(-1), U64)
    org = origins(n, 16, 3)[:4]
    ins = [subbox(V.reshape(-1), N, lo, 16, 3) for lo in org]
    sp = step_params()["C5"]
    dt0 = sp["dt0"]  # the hyperbolic CFL step of U^0 sets the cooling times
    T = V[4] / V[0]
    tc = I.cooling_time_field_torch(5002, n, NG, dt0, device=dev)
    L0 = (V[4] / ((G - 1) * V[0] ** 2 * torch.sqrt(T) * tc)).reshape(-1).contiguous()
    # the white-noise variant: t_c / dt0 log-uniform in [1e-3, 1e3], independent per cell
    tcw = torch.from_numpy(I.cooling_time_white(5003, n, NG, dt0)).to(dev)
    L0w = (V[4] / ((G - 1) * V[0] ** 2 * torch.sqrt(T) * tcw)).reshape(-1).contiguous()
    Tfl = 0.1 * float(T.min())
    del V, T, tc, tcw, hyp
    okw = dict(recon="ppm", riemann="hlld", parabolic_mask=7, tc_phi=0.3, cooling=True, cool_beta=0.5,
               T_floor=Tfl, **coef)
    p64 = ctu.Plan(ctu.make_opts(dim=3, gamma=G, dx=dx, precision="fp64", **okw), box, NG)
    dt, ch = sp["dt"], sp["ch"]
    params = torch.tensor([dt, ch], dtype=torch.float64, device=dev)
    log("C5: FP32 batched (autotune, graph)")
    p32 = ctu.Plan(ctu.make_opts(dim=3, gamma=G, dx=dx, precision="fp32", **okw), box, NG)
    U32, L32 = U64.to(torch.float32), L0.to(torch.float32)
    Uo32 = torch.zeros_like(U32)
    if not args.no_autotune:
        p32.autotune(U32, Uo32, params, L0=L32, reps=5, stream=s)
    ms, per = run_plan(p32, U32, Uo32, params, b, K, W, s, L0=L32)
    abz32 = ghost_bytes(n, 4) + 4 * ((n + 2 * NG) / n) ** 3  # plus the cooling coefficients
    r32 = result(ms, zones, abz32, per, p32.get_shape()[0])
    r32["roofline"] = kernel_roofline("C5", per, zones, "f32")
    r32["max_dp_over_p"] = b.dpp.item()
    log("C5: FP32 batched, white-noise cooling times")
    L32w = L0w.to(torch.float32)
    Uo32w = torch.zeros_like(U32)
    msw, perw = run_plan(p32, U32, Uo32w, params, b, K, W, s, L0=L32w)
    r32w = result(msw, zones, abz32, perw, p32.get_shape()[0])
    r32w["max_dp_over_p"] = b.dpp.item()
    log("C5: FP64 plain (eager)")
    Uo64 = torch.zeros_like(U64)
    ms64, per64 = run_plan(p64, U64, Uo64, params, b, K, W, s, L0=L0, graph=False)
    r64 = result(ms64, zones, ghost_bytes(n, 8) + 8 * ((n + 2 * NG) / n) ** 3, per64)
    L0s64 = [subbox_cells(L0, N, lo, 16) for lo in org]
    L0s32 = [subbox_cells(L32, N, lo, 16) for lo in org]
    samples.add("c5_fp32", okw, dx, dt, ch, ins, [subbox(Uo32, N, lo, 16, 3) for lo in org], L0s=L0s32)
    samples.add("c5_fp64", okw, dx, dt, ch, ins, [subbox(Uo64, N, lo, 16, 3) for lo in org], L0s=L0s64)
    samples.add("c5_white_fp32", okw, dx, dt, ch, ins, [subbox(Uo32w, N, lo, 16, 3) for lo in org],
                L0s=[subbox_cells(L32w, N, lo, 16) for lo in org])
    return {"fp32_batched": r32, "fp32_batched_white_tc": r32w, "fp64_plain": r64, "zones": zones,
            "coefficients": coef}


def leg_c3(args, dev, s, samples):
    """AMR: 3 levels, ratio 2, 64 / 442 / 951 patches of 16-32 cells around
    eight density blobs (1,457 patches, 17.4 M zones; 3 ghosts, fields at
    each level's resolution).  One AMR batch step = one CTU step of every
    patch of every level, each by its level's step dt0 / 2^l, with FP64 flux
    registers on the coarse-fine faces, plus the consuming reflux of the two
    coarser levels (each step's registers are consumed by its reflux).
    FP32 batched: one plan over all 1,457 patches (CTU_PLAN_LEVEL_DT), its
    step captured as one graph, then one reflux launch; also timed with one
    plan and one graph per level.  FP64 plain: one plan per patch, eager
    launches.  The subcycled
    level cycle (ghost fill, prolongation, substeps, restriction, reflux)
    runs on the nested variant of the hierarchy (level-2 boxes three level-1
    cells inside their parents, 1,181 patches), as its coarse-to-fine ghost
    fill needs."""
    import numpy as np
    import torch

    from paper_1110_0740_amd import amr, ctu, inputs as I

    K, W = max(3, args.steps // 2), min(args.warmup, 2)
    okw = dict(recon="ppm", riemann="hlld")

    def level_states(h, keep_prim=False):
        """conserved FP64 level arrays (and, with keep_prim, the primitive
        ones from the generator)"""
        U64, offs, Vs = [], [], []
        for lev, L in enumerate(h.levels):
            o, off = 0, []
            for B in L:
                off.append(o)
                o += 9 * int(np.prod([x + 2 * NG_AMR for x in B.n]))
            V = I.amr_level_fields_torch(h, lev, NG_AMR, device=dev)
            assert V.numel() == o
            tmp = ctu.Plan(ctu.make_opts(dim=3, gamma=5.0 / 3.0, dx=h.dx(0), precision="fp64", **okw),
                           [(B.lo, B.n, lev, ob) for B, ob in zip(L, off)], NG_AMR)
            U = torch.empty_like(V)
            tmp.prim_to_cons(V, U)
            U64.append(U)
            offs.append(off)
            if keep_prim:
                Vs.append(V)
            del tmp, V
        torch.cuda.synchronize()
        return U64, offs, Vs

    log("C3: configured hierarchy (1,457 patches)")
    h = I.amr_hierarchy()
    tables, nslots = amr.build_tables(h.levels, h.base, NG_AMR)
    nlev = len(h.levels)
    zones_l = [int(sum(int(np.prod(B.n)) for B in L)) for L in h.levels]
    ghost_l = [int(sum(int(np.prod([x + 2 * NG_AMR for x in B.n])) for B in L)) for L in h.levels]
    zones = sum(zones_l)
    npatch = sum(len(L) for L in h.levels)
    U64, offs, V64 = level_states(h, keep_prim=True)
    dt0 = 1e-4
    ch = 0.4 * h.dx(0)[0] / dt0
    params = [torch.tensor([dt0 / (1 << lev), ch], dtype=torch.float64, device=dev) for lev in range(nlev)]
    reg = torch.zeros(9 * nslots, dtype=torch.float64, device=dev)
    b = StepBufs(dev)
    # FP32 batched: one plan per level with its register faces and reflux table
    plans, Uin, Uout, shapes = [], [], [], []
    for lev, L in enumerate(h.levels):
        p = ctu.Plan(ctu.make_opts(dim=3, gamma=5.0 / 3.0, dx=h.dx(0), precision="fp32", **okw),
                     [(B.lo, B.n, lev, ob) for B, ob in zip(L, offs[lev])], NG_AMR, regfaces=tables[lev].regfaces,
                     reflux=tables[lev].reflux or None)
        plans.append(p)
        Uin.append(U64[lev].to(torch.float32))
        Uout.append(Uin[-1].clone())
    for lev, p in enumerate(plans):
        shapes.append(p.autotune(Uin[lev], Uout[lev], params[lev], reps=5, stream=s)[0] if not args.no_autotune
                      else p.get_shape()[0])
    # per-level kernel times (eager, events), then the captured graphs
    level_kernels = []
    for lev, p in enumerate(plans):
        p.enable_timing(True)
        with torch.cuda.stream(s):
            for _ in range(K):
                p.step(Uin[lev], Uout[lev], params[lev], b.rate, reg=reg, fails=b.fails, stream=s)
        s.synchronize()
        st, nrec = p.read_timing()
        p.enable_timing(False)
        level_kernels.append({k: v / max(nrec, 1) for k, v in st.items() if v > 0})
    reg.zero_()
    with torch.cuda.stream(s):
        for lev, p in enumerate(plans):
            p.graph_capture(Uin[lev], Uout[lev], params[lev], b.rate, reg=reg, fails=b.fails, stream=s)
    s.synchronize()
    # samples of the step (before any reflux) for the L1 figure
    rng = np.random.default_rng(3131)
    sample = []
    for lev in range(nlev):
        for bi in rng.choice(len(h.levels[lev]), size=3, replace=False):
            B = h.levels[lev][int(bi)]
            shp = (9,) + tuple(x + 2 * NG_AMR for x in reversed(B.n))
            o = offs[lev][int(bi)]
            cnt = int(np.prod(shp))
            sample.append((lev, V64[lev][o:o + cnt].cpu().numpy().reshape(shp),
                           Uout[lev][o:o + cnt].cpu().numpy().astype(np.float64).reshape(shp)))
    del V64

    def amr_step32():
        for p in plans:
            p.graph_launch(stream=s)
        for lev in range(nlev - 1):
            plans[lev].reflux_consume(Uout[lev], reg, stream=s)

    log("C3: FP32 one plan per level")
    ms_pl = timed(amr_step32, K, W, s)
    assert b.fails.sum().item() == 0
    # algorithmic bytes: ghosted reads, interior writes, register slots (read + write, FP64)
    alg_bytes = 36 * sum(ghost_l) + 36 * zones + 2 * 72 * nslots
    r_pl = result(ms_pl, zones, alg_bytes / zones, shape=shapes)
    r_pl["launches_per_step"] = 6 * nlev + nlev - 1
    del plans
    # one plan over every patch of every level, one graph per step
    log("C3: FP32 one plan over all levels")
    lbase = [0]
    for lev in range(nlev):
        lbase.append(lbase[-1] + Uin[lev].numel())
    bbase = [sum(len(x) for x in h.levels[:lev]) for lev in range(nlev)]
    Ucat = torch.cat(Uin)
    Uocat = Ucat.clone()
    allb = [(B.lo, B.n, lev, lbase[lev] + ob) for lev, L in enumerate(h.levels) for B, ob in zip(L, offs[lev])]
    regs = [(bbase[lev] + bb, d, f, tlo, tn, sl) for lev in range(nlev) for (bb, d, f, tlo, tn, sl) in tables[lev].regfaces]
    refl = [(bbase[lev] + cb, loc, d, sg, cs, fs) for lev in range(nlev) for (cb, loc, d, sg, cs, fs) in tables[lev].reflux]
    one = ctu.Plan(ctu.make_opts(dim=3, gamma=5.0 / 3.0, dx=h.dx(0), precision="fp32", **okw), allb, NG_AMR,
                   regfaces=regs, reflux=refl, level_dt=True)
    p0 = params[0]
    shape1 = one.autotune(Ucat, Uocat, p0, reps=5, stream=s)[0] if not args.no_autotune else one.get_shape()[0]
    one.enable_timing(True)
    with torch.cuda.stream(s):
        for _ in range(K):
            one.step(Ucat, Uocat, p0, b.rate, reg=reg, fails=b.fails, stream=s)
    s.synchronize()
    st, nrec = one.read_timing()
    one.enable_timing(False)
    one_kernels = {k: v / max(nrec, 1) for k, v in st.items() if v > 0}
    reg.zero_()
    with torch.cuda.stream(s):
        one.graph_capture(Ucat, Uocat, p0, b.rate, reg=reg, fails=b.fails, stream=s)
    s.synchronize()

    def amr_step_one():
        one.graph_launch(stream=s)
        one.reflux_consume(Uocat, reg, stream=s)

    ms32 = timed(amr_step_one, K, W, s)
    assert b.fails.sum().item() == 0
    r32 = result(ms32, zones, alg_bytes / zones, one_kernels, shape1)
    r32["launches_per_step"] = 7
    r32["roofline"] = kernel_roofline("C2", one_kernels, zones, "f32")
    r32["levels"] = []
    for lev in range(nlev):
        rl = {"patches": len(h.levels[lev]), "zones": zones_l[lev], "kernel_ms": level_kernels[lev],
              "roofline": kernel_roofline("C2", level_kernels[lev], zones_l[lev], "f32")}
        r32["levels"].append(rl)
    r32["per_level_plans"] = r_pl
    for lev in range(nlev):
        ins = [x for (l, x, _) in sample if l == lev]
        outs_ = [y for (l, _, y) in sample if l == lev]
        samples.add(f"c3_level{lev}_fp32", okw, h.dx(lev), dt0 / (1 << lev), ch, ins, outs_, ng=NG_AMR)
    del one, Uin, Uout, Ucat, Uocat
    torch.cuda.synchronize()
    # FP64 plain, one plan per patch
    r64 = ms64 = None
    if not args.no_per_patch:
        r64, ms64 = c3_per_patch(h, U64, params, offs, okw, zones, ghost_l, npatch, b, s, K, W)
    del U64
    torch.cuda.synchronize()
    # the subcycled level cycle on the nested hierarchy
    log("C3: subcycled level cycle (nested hierarchy)")
    hn = I.amr_hierarchy(nest=3)
    tn, nsn = amr.build_tables(hn.levels, hn.base, NG_AMR)
    U64n, offsn, _ = level_states(hn)
    paramsn = [torch.tensor([dt0 / (1 << lev), ch], dtype=torch.float64, device=dev) for lev in range(nlev)]
    regn = torch.zeros(9 * nsn, dtype=torch.float64, device=dev)
    plans_n = [ctu.Plan(ctu.make_opts(dim=3, gamma=5.0 / 3.0, dx=hn.dx(0), precision="fp32", **okw),
                        [(B.lo, B.n, lev, ob) for B, ob in zip(L, offsn[lev])], NG_AMR, regfaces=tn[lev].regfaces,
                        reflux=tn[lev].reflux or None) for lev, L in enumerate(hn.levels)]
    Ua = [u.to(torch.float32) for u in U64n]
    Ub = [u.clone() for u in Ua]
    # the level plans take their tuned launch shapes, as the batched plans do
    cyc_shapes = [p.autotune(Ua[lev], Ub[lev], paramsn[lev], reps=5, stream=s)[0] if not args.no_autotune
                  else p.get_shape()[0] for lev, p in enumerate(plans_n)]
    hier = ctu.Hier("fp32", hn.base, [[(B.lo, B.n, ob) for B, ob in zip(L, offsn[lev])]
                                      for lev, L in enumerate(hn.levels)], NG_AMR)
    rate_l = torch.zeros(nlev, dtype=torch.float64, device=dev)
    fails_acc = torch.zeros(5, dtype=torch.int32, device=dev)
    missing = torch.zeros(1, dtype=torch.int32, device=dev)
    cur = [0] * nlev
    msc = timed(lambda: hier.advance(plans_n, Ua, Ub, cur, paramsn, regn, rate_l, fails=fails_acc, missing=missing,
                                     stream=s), K, W, s)
    assert fails_acc.sum().item() == 0 and missing.item() == 0
    cyc_zones = sum(int(np.prod(B.n)) << lev for lev, L in enumerate(hn.levels) for B in L)
    nsteps = sum(1 << lev for lev in range(nlev))
    cycle = {"ms_per_cycle": msc, "zone_updates_per_cycle": cyc_zones, "zone_updates_per_s": cyc_zones / (msc * 1e-3),
             "patches": sum(len(L) for L in hn.levels), "level_steps_per_cycle": nsteps, "shapes": cyc_shapes}
    return {"patches": npatch, "zones": zones, "levels": [len(L) for L in h.levels], "register_slots": nslots,
            "fp32_batched": r32, "fp64_plain_per_patch": r64,
            "batched_fp32_over_plain_fp64": ms64 / ms32 if ms64 else None,
            "fp32_cycle": cycle}


def c3_per_patch(h, U64, params, offs, okw, zones, ghost_l, npatch, b, s, K, W):
    """C3's FP64 plain path: one plan per patch, eager launches."""
    import torch

    from paper_1110_0740_amd import ctu

    log("C3: FP64 one plan per patch")
    pplans = []
    for lev, L in enumerate(h.levels):
        go = ctu.make_opts(dim=3, gamma=5.0 / 3.0, dx=h.dx(0), precision="fp64", **okw)
        for B, ob in zip(L, offs[lev]):
            pplans.append((lev, ctu.Plan(go, [(B.lo, B.n, lev, ob)], NG_AMR)))
    Uo64 = [torch.zeros_like(u) for u in U64]
    torch.cuda.synchronize()

    def amr_step64():
        for lev, p in pplans:
            p.step(U64[lev], Uo64[lev], params[lev], b.rate, fails=b.fails, stream=s)

    ms64 = timed(amr_step64, K, W, s)
    assert b.fails.sum().item() == 0
    r64 = result(ms64, zones, 2 * (36 * sum(ghost_l) + 36 * zones) / zones)
    r64["launches_per_step"] = 6 * npatch
    del pplans, Uo64
    return r64, ms64


# ---------------------------------------------------------------------------
# the oracle: host timing and the L1 figures
# ---------------------------------------------------------------------------


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(timing_boxes, c2_params, samples):
    """The FP64 oracle as it stands, timed on this host: one step of three
    48^3 sub-boxes (+4 ghosts) of the C2 input, with every core and with one,
    median of 3 runs each; then the oracle recomputes every timed result's
    sampled sub-boxes for the L1 figures."""
    import numpy as np

    import oracle as O
    from paper_1110_0740_amd import inputs as I

    dx, gamma, dt, ch = c2_params
    oo = O.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=gamma, dx=dx)
    timing_boxes = [O.prim2cons(oo, V) for V in timing_boxes]
    zones = sum(int(np.prod([x - 2 * NG for x in U.shape[1:]])) for U in timing_boxes)
    rates = {}
    for label, nt in (("all", 0), ("one", 1)):
        used = O.set_threads(nt)
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            for U in timing_boxes:
                O.step(oo, U, NG, dt, ch)
            runs.append(time.perf_counter() - t0)
        rates[label] = (zones / statistics.median(runs), used, statistics.median(runs))
    O.set_threads(0)
    base = {"value": rates["all"][0], "unit": "zone-updates/s", "cores": rates["all"][1], "kind": "oracle",
            "sample": f"one FP64 step of 3 sub-boxes of 48^3 (+4 ghosts) of the 256^3 C2 input, median of 3 runs "
                      f"({rates['all'][2]:.2f} s with {rates['all'][1]} threads, {rates['one'][2]:.2f} s with 1)",
            "one_core": {"value": rates["one"][0], "cores": 1}, "nproc": os.cpu_count(), "cpu_model": cpu_model()}
    l1 = {}
    for leg, it in samples.items.items():
        pairs = []
        if it["chain"] is not None:  # C1: chained steps on the periodic box
            o = O.make_opts(dim=it["dim"], gamma=5.0 / 3.0, dx=it["dx"], **it["okw"])
            U = O.prim2cons(o, it["ins"][0])
            for dtk, chk in it["chain"]:
                U, _, _, f = O.step(o, U, NG, dtk, chk)
                I.fill_periodic(U, NG, it["dim"])
            pairs.append((it["outs"][0], U))
            ch_last = it["chain"][-1][1]
        else:
            gam = 4.0 / 3.0 if it["physics"] == "rmhd" else 5.0 / 3.0
            o = O.make_opts(dim=3, gamma=gam, dx=it["dx"], **it["okw"])
            for k, (Vi, Ug) in enumerate(zip(it["ins"], it["outs"])):
                L0 = it["L0s"][k] if it["L0s"] else None
                ref, _, _, f = O.step(o, O.prim2cons(o, Vi), it["ng"], it["dt"], it["ch"], L0=L0)
                pairs.append((Ug, ref))
            ch_last = it["ch"]
        e, c = parity_norms(pairs, ch_last, it["physics"], it["dim"], it["ng"])
        l1[leg] = {"l1_rel": e, "cell_rel": c, "subboxes": len(pairs)}
    return base, l1


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no multi-GPU path "
              f"(boxes would shard by zone count with one halo exchange per substep; not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    legs = set(args.legs.split(","))
    samples = Samples()
    line_legs = {}
    peaks = leg_peaks()
    variants = {}
    c2 = timing_boxes = c2p = None
    if "c2" in legs:
        c2, v, timing_boxes, c2p = leg_c2(args, dev, s, samples)
        if v:
            variants.update({f"c2_{k}": x for k, x in v.items()})
        torch.cuda.empty_cache()
    if "c1" in legs:
        line_legs["c1_2d_128"] = leg_c1(args, dev, s, samples)
    if "c4" in legs:
        c4, v4 = leg_c4(args, dev, s, samples)
        line_legs["c4_rmhd_192"] = c4
        variants.update(v4)
        torch.cuda.empty_cache()
    if "c5" in legs:
        line_legs["c5_nonideal_256"] = leg_c5(args, dev, s, samples)
        torch.cuda.empty_cache()
    if "c3" in legs and not args.no_amr:
        line_legs["c3_amr"] = leg_c3(args, dev, s, samples)
        torch.cuda.empty_cache()
    if c2 is None:
        print(json.dumps({"legs": line_legs, "variants": variants, "measured_peaks": peaks}), flush=True)
        return
    res = c2["fp32_batched"]
    K, W = args.steps, args.warmup
    roof = dict(res["roofline"]) if res.get("roofline") else None
    if roof is not None:
        same = res.get("shape") and res.get("flat_boxes", 0) == 0 and all(
            res["shape"][f] == PROFILE_SHAPE[f] for f in PROFILE_SHAPE)
        roof["traffic"] = TCOUPLE_TRAFFIC_BYTES if (same and roof["kernel"] == "tcouple") else None
        roof["shape"] = res.get("shape")
        if roof.get("achieved"):
            roof["frac_of_measured_fma"] = roof["achieved"] / peaks["valu_fp32_fma_TFLOPs"]
    line = {
        "metric": METRIC,
        "value": res["zone_updates_per_s"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D ideal MHD 256^3 periodic, PPM characteristic tracing + HLLD + GLM, Gamma 5/3, "
                               "CFL 0.4, seeded smooth random modes (beta~1, Mach~1), 20 steps",
                   "zones": c2["zones"], "nghost": NG, "path": "fp32_batched"},
        "hbm_step": {"bound": "hbm", "achieved": res["hbm_alg_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": res["hbm_frac"], "alg_bytes_per_zone": res["alg_bytes_per_zone"],
                     "frac_of_measured_copy": res["hbm_alg_GBs"] / peaks["hbm_copy_GBs"]},
        "roofline": roof,
        "measured_peaks": peaks,
        "paths": {"fp32_batched": res, "fp64_plain": c2["fp64_plain"]},
        "fp32_over_fp64": res["zone_updates_per_s"] / c2["fp64_plain"]["zone_updates_per_s"],
        "legs": line_legs,
    }
    if variants:
        line["variants"] = variants
    if not args.no_cpu:
        log("oracle cpu_baseline and L1 figures")
        base, l1 = cpu_baseline(timing_boxes, c2p, samples)
        line["cpu_baseline"] = base
        attach_l1(line, l1)
    print(json.dumps(line), flush=True)


def attach_l1(line, l1):
    """Put each L1 figure beside the timed result it checks."""
    where = {"c2_fp32": line["paths"]["fp32_batched"], "c2_fp64": line["paths"]["fp64_plain"]}
    legs = line["legs"]
    if "c1_2d_128" in legs:
        where["c1_fp64_10steps"] = legs["c1_2d_128"]["fp64_batched"]
    if "c4_rmhd_192" in legs:
        where["c4_rmhd192_ideal_fp32"] = legs["c4_rmhd_192"]["fp32_batched"]
        where["c4_rmhd192_ideal_fp64"] = legs["c4_rmhd_192"]["fp64_plain"]
    if "c5_nonideal_256" in legs:
        where["c5_fp32"] = legs["c5_nonideal_256"]["fp32_batched"]
        where["c5_white_fp32"] = legs["c5_nonideal_256"]["fp32_batched_white_tc"]
        where["c5_fp64"] = legs["c5_nonideal_256"]["fp64_plain"]
    if "c3_amr" in legs:
        for lev, rl in enumerate(legs["c3_amr"]["fp32_batched"]["levels"]):
            where[f"c3_level{lev}_fp32"] = rl
    for k, v in line.get("variants", {}).items():
        where[k if k.startswith("c2_") else f"c4_{k}_fp32"] = v
    for k, v in l1.items():
        if k in where:
            where[k]["vs_oracle"] = v


if __name__ == "__main__":
    main()
