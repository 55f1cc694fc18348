"""Benchmark: zone-updates/s of one CTU-GLM step on the 3D ideal-MHD workload
(256^3 periodic, PPM characteristic tracing + HLLD + GLM, Gamma = 5/3,
CFL 0.4), FP32 batched (HIP-graph replay) vs FP64 plain (eager launches),
on one MI355X.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--no-cpu]

A step is one pass of the whole hot path (primitive recovery, t^n Godunov
fluxes, predictors, corner coupling, final Riemann solves, update, split
sources, FP64 CFL reduction) over the resident 256^3 state.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec per CTU step (FP32 batched vs FP64 plain) + achieved HBM GB/s"

# Algorithmic FP32 floating-point operations per interior zone of each
# kernel of the FP32 step (256^3, PPM + HLLD + GLM), counted by rocprofv3
# (SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes / 16,777,216 zones, which equals
# 64 x (ADD + MUL + 2 FMA + TRANS) wave instructions) with the commands in
# profiles/ctu_step_fp32_256cube_counters.md.  t^n: the run with one chunk
# per tile column (--shape tiles,4096,16,1), which recomputes no marching
# face (4-plane chunks execute 1558); x sweep: 64 pencils per block, the
# least per-block setup (16 pencils execute 1403).  They include the ~1 %
# of items computed for the pencil ends and the region's halo faces.
KERNEL_FLOPS_PER_ZONE = {"prim": 37.0, "tcouple": 1455.0, "sweep_x": 1389.0, "sweep_y": 1387.0,
                         "sweep_z": 1386.0}
# HBM bytes per launch, FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB x 1024): a
# plain 1 GiB device copy (bench.py --copy-calibration) reads back as
# 524,308 KiB of FETCH_SIZE and 1,048,576 KiB of WRITE_SIZE, hence the
# factors.  Same profile file; set an entry to None when its kernel changes
# after the counter runs.
KERNEL_TRAFFIC_BYTES = {"prim": (327952 * 2 + 646866) * 1024, "tcouple": (471996 * 2 + 1987027) * 1024,
                        "sweep_x": (949173 * 2 + 638239) * 1024, "sweep_y": (1014995 * 2 + 632507) * 1024,
                        "sweep_z": (1005719 * 2 + 629251) * 1024}
# The launch shape of the single-box FP32 plan the counters above were taken
# with (bench.py --shape tiles,4,16,1,2).  A kernel's traffic depends on the
# shape fields that change its tiles (the t^n layout -- no box of the 256^3
# plan can take the flat one -- and chunk, the x-sweep pencils, the launch
# order, the y / z sweep segments), so the roofline reports it only when the tuned shape agrees on
# those fields.
PROFILE_SHAPE = {"tc_layout": "tiles", "tc_chunk": 4, "x_pencils": 16, "xcd_order": 1, "yz_segments": 2}
SHAPE_FIELDS = {"prim": (), "tcouple": ("tc_chunk", "xcd_order"), "sweep_x": ("x_pencils", "xcd_order"),
                "sweep_y": ("xcd_order", "yz_segments"), "sweep_z": ("xcd_order", "yz_segments")}


def same_profiled_shape(kernel, res):
    shape = res.get("shape")
    if shape is None or res.get("flat_boxes", 0) != 0:
        return False
    return all(shape[f] == PROFILE_SHAPE[f] for f in SHAPE_FIELDS.get(kernel, ("?",)))
# Algorithmic HBM bytes per zone of a whole step (read U^n on the ghosted box,
# write U^{n+1}): 36 B x (264/256)^3 + 36 B in FP32, twice that in FP64.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3           # published FP32 vector peak (packed FP32 issue)
PEAK_FP32_UNPACKED_TFLOPS = 78.6   # one FP32 lane op per VALU lane per cycle (this build emits no packed FP32)
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle cpu_baseline leg")
    ap.add_argument("--precision", default="both", choices=["both", "fp32", "fp64"])
    ap.add_argument("--no-amr", action="store_true", help="skip the AMR batch leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of tuning the FP32 plans first")
    ap.add_argument("--only-amr", action="store_true",
                    help="run the AMR batch leg alone and print it (profiling aid; not the bench line)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the shock-hybrid and Rusanov variants of the FP32 step")
    ap.add_argument("--shape", default=None,
                    help="force the launch shape of the single-box FP32 plan instead of tuning it: "
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


def cpu_baseline(Vfull, ng, dx, gamma, sub=96, nsub=3):
    """The FP64 oracle, single-threaded, on `nsub` sub-boxes of sub^3 cut from
    the same input (ghosts included), one step each."""
    import numpy as np

    import oracle as O
    from paper_1110_0740_amd import inputs as I

    oo = O.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=gamma, dx=dx)
    n = Vfull.shape[-1] - 2 * ng
    origins = [(0, 0, 0), (n - sub, n // 2 - sub // 2, 17), (n // 3, n - sub, n - sub)][:nsub]
    zones = 0
    elapsed = 0.0
    for lo in origins:
        Vs = I.sub_box(Vfull, lo, (sub, sub, sub), ng, 3)
        U = O.prim2cons(oo, Vs)
        rate = O.cfl_rate(oo, U, ng)
        dt = 0.4 / rate
        ch = 0.4 * dx[0] / dt
        t0 = time.perf_counter()
        O.step(oo, U, ng, dt, ch)
        elapsed += time.perf_counter() - t0
        zones += sub ** 3
    return {"value": zones / elapsed, "unit": "zone-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsub} sub-boxes of {sub}^3 (+4 ghosts) of the {n}^3 input, one FP64 step each, "
                      f"{elapsed:.1f} s single-threaded"}


def amr_leg(K, W, dev, s, tune=True):
    """AMR batch: 3 levels, ratio 2, ~1200 patches of 16^3-32^3 around density
    blobs (4 ghosts, fields evaluated at each level's resolution; level-2
    boxes 3 parent cells inside their parents).  One AMR step = one CTU step
    of every patch of every level plus the two reflux launches.  FP32
    batched: one plan and one captured graph per level.  FP64 plain: one
    plan per patch, eager launches, no graph.  FP32 cycle: one level-0 step
    of the subcycled level cycle (ctu_hier_advance)."""
    import numpy as np
    import torch

    from paper_1110_0740_amd import amr, ctu, inputs as I

    ng = 4
    h = I.amr_hierarchy(nest=3)
    tables, nslots = amr.build_tables(h.levels, h.base, ng)
    zones = int(sum(int(np.prod(B.n)) for L in h.levels for B in L))
    npatch = sum(len(L) for L in h.levels)
    dt0 = 1e-4
    ch = 0.4 * h.dx(0)[0] / dt0
    reg = torch.zeros(9 * nslots, dtype=torch.float64, device=dev)
    rate = torch.zeros(1, dtype=torch.float64, device=dev)
    fails = torch.zeros(5, dtype=torch.int32, device=dev)
    # conserved states per level, FP64, packed in box order
    U64, offs = [], []
    for lev, L in enumerate(h.levels):
        o, off = 0, []
        for B in L:
            off.append(o)
            o += 9 * int(np.prod([n + 2 * ng for n in B.n]))
        U = torch.empty(o, dtype=torch.float64, device=dev)
        go = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=5.0 / 3.0, dx=h.dx(0), precision="fp64")
        boxes = [(B.lo, B.n, lev, ob) for B, ob in zip(L, off)]
        tmp = ctu.Plan(go, boxes, ng)
        for B, ob in zip(L, off):
            V = I.amr_fields_torch(h, B, ng, device=dev).reshape(-1)
            U[ob:ob + V.numel()] = V
        Uc = torch.empty_like(U)
        tmp.prim_to_cons(U, Uc)
        U64.append(Uc)
        offs.append(off)
        del tmp, U
    torch.cuda.synchronize()
    params = [torch.tensor([dt0 / (1 << lev), ch], dtype=torch.float64, device=dev) for lev in range(len(h.levels))]
    out = {"patches": npatch, "zones": zones, "levels": [len(L) for L in h.levels], "register_slots": nslots}

    # FP32 batched
    plans, Uin, Uout = [], [], []
    for lev, L in enumerate(h.levels):
        go = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=5.0 / 3.0, dx=h.dx(0), precision="fp32")
        p = ctu.Plan(go, [(B.lo, B.n, lev, ob) for B, ob in zip(L, offs[lev])], ng, regfaces=tables[lev].regfaces)
        if tables[lev].reflux:
            p.set_reflux(tables[lev].reflux)
        plans.append(p)
        Uin.append(U64[lev].to(torch.float32))
        Uout.append(torch.empty_like(Uin[-1]))
    torch.cuda.synchronize()
    # launch shapes: measured per level plan (untimed setup), then captured
    shapes = []
    for lev, p in enumerate(plans):
        if tune:
            shapes.append(p.autotune(Uin[lev], Uout[lev], params[lev], reps=5, stream=s)[0])
        else:
            shapes.append(p.get_shape()[0])
    with torch.cuda.stream(s):
        for lev, p in enumerate(plans):
            p.graph_capture(Uin[lev], Uout[lev], params[lev], rate, reg=reg, fails=fails, stream=s)

    def amr_step32():
        for p in plans:
            p.graph_launch(stream=s)
        for lev in range(len(plans) - 1):
            plans[lev].reflux(Uout[lev], reg, stream=s)

    with torch.cuda.stream(s):
        for _ in range(W):
            amr_step32()
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record(s)
        for _ in range(K):
            amr_step32()
        e1.record(s)
    s.synchronize()
    ms32 = e0.elapsed_time(e1) / K
    assert fails.sum().item() == 0, fails
    out["fp32_batched"] = {"ms_per_step": ms32, "zone_updates_per_s": zones / (ms32 * 1e-3),
                           "launches_per_step": len(plans) + len(plans) - 1, "shapes": shapes}

    # FP32 level cycle: one level-0 step with ratio-2 subcycling (ghost fill
    # and prolongation, steps, restriction, refluxing), eager launches
    nlev = len(h.levels)
    hier = ctu.Hier("fp32", h.base, [[(B.lo, B.n, ob) for B, ob in zip(L, offs[lev])]
                                     for lev, L in enumerate(h.levels)], ng)
    rate_l = torch.zeros(nlev, dtype=torch.float64, device=dev)
    fails_acc = torch.zeros(5, dtype=torch.int32, device=dev)
    missing = torch.zeros(1, dtype=torch.int32, device=dev)
    reg.zero_()
    cur = [0] * nlev

    def amr_cycle32():
        hier.advance(plans, Uin, Uout, cur, params, reg, rate_l, fails=fails_acc, missing=missing, stream=s)

    with torch.cuda.stream(s):
        for _ in range(W):
            amr_cycle32()
    s.synchronize()
    with torch.cuda.stream(s):
        e0.record(s)
        for _ in range(K):
            amr_cycle32()
        e1.record(s)
    s.synchronize()
    msc = e0.elapsed_time(e1) / K
    assert fails_acc.sum().item() == 0 and missing.item() == 0, (fails_acc, missing)
    cyc_zones = sum(int(np.prod(B.n)) << lev for lev, L in enumerate(h.levels) for B in L)
    nsteps = sum(1 << lev for lev in range(nlev))
    out["fp32_cycle"] = {"ms_per_cycle": msc, "zone_updates_per_cycle": cyc_zones,
                         "zone_updates_per_s": cyc_zones / (msc * 1e-3), "level_steps_per_cycle": nsteps,
                         "launches_per_cycle": 8 * nsteps + 2 * sum(1 << lev for lev in range(nlev - 1))}
    del plans, Uin, Uout, hier
    torch.cuda.synchronize()

    # FP64 plain, one plan per patch
    pplans = []
    for lev, L in enumerate(h.levels):
        go = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=5.0 / 3.0, dx=h.dx(0), precision="fp64")
        for B, ob in zip(L, offs[lev]):
            pplans.append((lev, ctu.Plan(go, [(B.lo, B.n, lev, ob)], ng)))
    Uo64 = [torch.empty_like(u) for u in U64]
    torch.cuda.synchronize()

    def amr_step64():
        for lev, p in pplans:
            p.step(U64[lev], Uo64[lev], params[lev], rate, fails=fails, stream=s)

    with torch.cuda.stream(s):
        for _ in range(W):
            amr_step64()
    s.synchronize()
    with torch.cuda.stream(s):
        e0.record(s)
        for _ in range(K):
            amr_step64()
        e1.record(s)
    s.synchronize()
    ms64 = e0.elapsed_time(e1) / K
    assert fails.sum().item() == 0, fails
    out["fp64_plain_per_patch"] = {"ms_per_step": ms64, "zone_updates_per_s": zones / (ms64 * 1e-3),
                                   "launches_per_step": 6 * npatch}
    out["batched_fp32_over_plain_fp64"] = ms64 / ms32
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no multi-GPU path "
              f"(boxes would shard by zone count with one halo exchange per substep; not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1110_0740_amd import ctu, inputs as I

    dev = torch.device("cuda:0")
    n, ng = args.n, 4
    K, W = args.steps, args.warmup
    if args.only_amr:
        # the AMR batch leg alone (for profiling its kernels); not the bench line
        print(json.dumps({"amr": amr_leg(max(3, K // 2), min(W, 2), dev, torch.cuda.Stream(),
                                         tune=not args.no_autotune)}), flush=True)
        return
    print(f"[bench] generating {n}^3 inputs on the GPU", file=sys.stderr, flush=True)
    V64, meta = I.mhd3d_fields_torch(n=n, ng=ng, seed=2000, device=dev)
    dx, gamma = meta["dx"], meta["gamma"]
    N = n + 2 * ng
    zones = n ** 3
    box = [((0, 0, 0), (n, n, n), 0, 0)]
    s = torch.cuda.Stream()

    o64 = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=gamma, dx=dx, precision="fp64")
    p64 = ctu.Plan(o64, box, ng)
    U64 = torch.empty(9 * N ** 3, dtype=torch.float64, device=dev)
    p64.prim_to_cons(V64.reshape(-1), U64)
    rate = torch.zeros(1, dtype=torch.float64, device=dev)
    p64.cfl_rate(U64, rate)
    torch.cuda.synchronize()
    dt = 0.4 / rate.item()
    ch = 0.4 * dx[0] / dt
    params = torch.tensor([dt, ch], dtype=torch.float64, device=dev)
    fails = torch.zeros(5, dtype=torch.int32, device=dev)
    Vhost = None
    if not args.no_cpu:
        Vhost = V64.cpu().numpy()
    del V64

    result = {}

    def run_fp64():
        Uo = torch.empty_like(U64)
        with torch.cuda.stream(s):
            for _ in range(W):
                p64.step(U64, Uo, params, rate, fails=fails, stream=s)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            e0.record(s)
            for _ in range(K):
                p64.step(U64, Uo, params, rate, fails=fails, stream=s)
            e1.record(s)
        s.synchronize()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        assert fails.sum().item() == 0, fails
        result["fp64_plain"] = {"ms_per_step": ms, "zone_updates_per_s": zones / (ms * 1e-3)}
        del Uo

    def run_fp32():
        o32 = ctu.make_opts(dim=3, recon="ppm", riemann="hlld", gamma=gamma, dx=dx, precision="fp32")
        p32 = ctu.Plan(o32, box, ng)
        U32 = U64.to(torch.float32)
        Uo = torch.empty_like(U32)
        torch.cuda.synchronize()
        if args.shape:
            f = args.shape.split(",")
            p32.set_shape(tc_layout=f[0], tc_chunk=int(f[1]), x_pencils=int(f[2]), xcd_order=int(f[3]),
                          yz_segments=int(f[4]) if len(f) > 4 else 0)
        elif not args.no_autotune:
            p32.autotune(U32, Uo, params, reps=20, stream=s)
        shape, flat_boxes = p32.get_shape()
        with torch.cuda.stream(s):
            p32.graph_capture(U32, Uo, params, rate, fails=fails, stream=s)
            for _ in range(W):
                p32.graph_launch(stream=s)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            e0.record(s)
            for _ in range(K):
                p32.graph_launch(stream=s)
            e1.record(s)
        s.synchronize()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        assert fails.sum().item() == 0, fails
        # per-kernel durations: the same K steps launched eagerly with HIP
        # events around every kernel, on the same stream
        p32.enable_timing(True)
        with torch.cuda.stream(s):
            for _ in range(K):
                p32.step(U32, Uo, params, rate, fails=fails, stream=s)
        s.synchronize()
        stage_ms, nrec = p32.read_timing()
        p32.enable_timing(False)
        result["fp32_batched"] = {"ms_per_step": ms, "zone_updates_per_s": zones / (ms * 1e-3), "shape": shape,
                                  "flat_boxes": flat_boxes,
                                  "stage_ms": {k: v / max(nrec, 1) for k, v in stage_ms.items() if v > 0}}
        del Uo, U32, p32

    def run_variants():
        """The same FP32 workload under the option sets of the widened rows:
        the App. B shock-adaptive hybrid (flags from V^n every step, HLL and
        MinMod where flagged), the Rusanov, HLLC and Roe solvers, the MT corner coupling; and the relativistic
        workload under both equations of state.  Tuned, graph-replayed."""
        out = {}
        variants = {"shock_hybrid": dict(riemann="hlld", shock_eps=5.0), "rusanov": dict(riemann="rusanov"),
                    "hllc": dict(riemann="hllc"), "roe": dict(riemann="roe"),
                    "mt_corner": dict(riemann="hlld", corner="mt")}
        for name, kw in variants.items():
            o = ctu.make_opts(dim=3, recon="ppm", gamma=gamma, dx=dx, precision="fp32", **kw)
            p = ctu.Plan(o, box, ng)
            U32 = U64.to(torch.float32)
            Uo = torch.empty_like(U32)
            torch.cuda.synchronize()
            if not args.no_autotune:
                p.autotune(U32, Uo, params, reps=3, stream=s)
            with torch.cuda.stream(s):
                p.graph_capture(U32, Uo, params, rate, fails=fails, stream=s)
                for _ in range(W):
                    p.graph_launch(stream=s)
            s.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(s):
                e0.record(s)
                for _ in range(K):
                    p.graph_launch(stream=s)
                e1.record(s)
            s.synchronize()
            ms = e0.elapsed_time(e1) / K
            assert fails.sum().item() == 0, (name, fails)
            out[name] = {"ms_per_step": ms, "zone_updates_per_s": zones / (ms * 1e-3), "shape": p.get_shape()[0]}
            del p, U32, Uo
        # relativistic MHD, 192^3 jets and blobs (Lorentz factors up to 10),
        # MUSCL-Hancock + MC + HLL + GLM, FP32 fluxes with the FP64 inversion,
        # under the ideal EOS (Gamma = 4/3) and the Taub-Matthews EOS, and
        # with the exact fast speeds instead of the isotropic bound
        nr = 192
        Vr, mr = I.rmhd3d_fields(n=nr, ng=ng, seed=4000)
        Vr = torch.from_numpy(Vr.reshape(-1)).to(dev)
        zr = nr ** 3
        boxr = [((0, 0, 0), (nr, nr, nr), 0, 0)]
        for eos, xs, rs in (("ideal", False, "hll"), ("tm", False, "hll"), ("ideal", True, "hll"),
                            ("ideal", False, "hllc"), ("ideal", False, "hlld")):
            kw = dict(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", riemann=rs, gamma=mr["gamma"],
                      dx=mr["dx"], eos=eos, exact_speeds=xs)
            p64 = ctu.Plan(ctu.make_opts(precision="fp64", **kw), boxr, ng)
            Ur64 = torch.empty_like(Vr)
            p64.prim_to_cons(Vr, Ur64)
            p64.cfl_rate(Ur64, rate)
            torch.cuda.synchronize()
            dtr = 0.3 / rate.item()
            pr = torch.tensor([dtr, min(0.3 * mr["dx"][0] / dtr, 1.0)], dtype=torch.float64, device=dev)
            p = ctu.Plan(ctu.make_opts(precision="fp32", **kw), boxr, ng)
            U32 = Ur64.to(torch.float32)
            Uo = torch.empty_like(U32)
            del p64, Ur64
            if not args.no_autotune:
                p.autotune(U32, Uo, pr, reps=3, stream=s)
            with torch.cuda.stream(s):
                p.graph_capture(U32, Uo, pr, rate, fails=fails, stream=s)
                for _ in range(W):
                    p.graph_launch(stream=s)
            s.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(s):
                e0.record(s)
                for _ in range(K):
                    p.graph_launch(stream=s)
                e1.record(s)
            s.synchronize()
            ms = e0.elapsed_time(e1) / K
            assert fails.sum().item() == 0, ("rmhd", eos, fails)
            out[f"rmhd192_{eos}" + ("_exact_speeds" if xs else "") + ("" if rs == "hll" else "_" + rs)] = {
                "ms_per_step": ms, "zone_updates_per_s": zr / (ms * 1e-3), "shape": p.get_shape()[0]}
            del p, U32, Uo
        del Vr
        return out

    print(f"[bench] timing {K} steps after {W} warm-up steps", file=sys.stderr, flush=True)
    if args.precision in ("both", "fp32"):
        run_fp32()
    if args.precision in ("both", "fp64"):
        run_fp64()
    variants = run_variants() if args.precision in ("both", "fp32") and not args.no_variants else None

    main_key = "fp32_batched" if "fp32_batched" in result else "fp64_plain"
    res = result[main_key]
    esize = 4 if main_key == "fp32_batched" else 8
    alg_bytes_zone = 9 * esize * ((n + 2 * ng) / n) ** 3 + 9 * esize
    hbm_gbs = alg_bytes_zone * zones / (res["ms_per_step"] * 1e-3) / 1e9
    roofline = None
    if "stage_ms" in res:
        dom = max(res["stage_ms"], key=res["stage_ms"].get)
        dom_ms = res["stage_ms"][dom]
        fpz = KERNEL_FLOPS_PER_ZONE.get(dom) if main_key == "fp32_batched" and n == 256 else None
        if fpz is not None:
            achieved = fpz * zones / (dom_ms * 1e-3) / 1e12
            roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                        "traffic": (KERNEL_TRAFFIC_BYTES.get(dom) if same_profiled_shape(dom, res) else None),
                        "avg_ms": dom_ms, "shape": res.get("shape"),
                        "flop_per_zone": fpz, "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
                        "frac_unpacked": achieved / PEAK_FP32_UNPACKED_TFLOPS}
        else:
            roofline = {"bound": "alu", "kernel": dom, "achieved": None, "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": None, "traffic": None, "avg_ms": dom_ms}
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
        "dtype": "f32" if main_key == "fp32_batched" else "f64",
        "data": "synthetic",
        "config": {"workload": f"3D ideal MHD {n}^3 periodic, PPM characteristic tracing + HLLD + GLM, "
                               f"Gamma 5/3, CFL 0.4, seeded smooth random modes (beta~1, Mach~1)",
                   "zones": zones, "nghost": ng, "path": main_key},
        "hbm_step": {"bound": "hbm", "achieved": hbm_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": hbm_gbs / PEAK_HBM_GBS, "alg_bytes_per_zone": alg_bytes_zone},
        "roofline": roofline,
        "paths": result,
    }
    if variants:
        line["variants"] = variants
    if "fp64_plain" in result and "fp32_batched" in result:
        line["fp32_over_fp64"] = result["fp32_batched"]["zone_updates_per_s"] / result["fp64_plain"][
            "zone_updates_per_s"]
    if not args.no_amr:
        print("[bench] AMR batch leg", file=sys.stderr, flush=True)
        del U64
        torch.cuda.empty_cache()
        line["amr"] = amr_leg(max(3, K // 2), min(W, 2), dev, s, tune=not args.no_autotune)
    if not args.no_cpu:
        print("[bench] oracle cpu_baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(Vhost, ng, dx, gamma)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
