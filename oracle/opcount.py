"""Algorithmic operation counts per zone of the CTU step, from the op-counting
build of the oracle (oracle/opcount.cpp).

MEASUREMENT INFRASTRUCTURE, like the oracle itself: never imported by the
product library.  Writes profiles/oracle_opcount.md; the benchmark's
algorithmic FLOP figures are copied from there.

For each workload, one step of the oracle on a sub-box of the workload's own
fields (a box of 32^3 zones at the workload's resolution; 2D: 64^2) is
counted stage by stage (orc_step's ORC_STAGE hooks).  Each stage's count is
divided by the units of work the oracle does in it on that ghosted box and
multiplied by the units the method needs per interior zone, so the halo
work of the oracle's box does not enter:
  1 primitive recovery         per ghosted cell   -> 1 per zone
  2 t^n fluxes + increments    per face solved    -> dim per zone
  3 predictors + coupling      per predicted cell -> dim per zone
  4 time-centred solves        per face           -> dim per zone
  5 half-step state V^{n+1/2}  per ghosted cell   -> 1 per zone (parabolic)
  6 half-step parabolic flux   per face           -> dim per zone (parabolic)
  7 update, sources, rate      per zone           -> 1 per zone
With parabolic terms the t^n stage also evaluates Pi^n; the step is counted
a second time on the same fields with the parabolic terms and cooling off,
and the difference of the two t^n stages is listed as Pi^n (the GPU computes
it in a kernel of its own, k_pdiv; Pi^{n+1/2} likewise in k_pflux).
FLOPs are additions / subtractions, multiplications, divisions, square roots
and transcendental calls (exp, log, pow, cbrt), each one (a fused
multiply-add is two); comparisons and min / max / abs are listed apart.
The oracle's numerical inversion of the eigenvector matrix (which the
method, and the GPU, replaces by closed-form left eigenvectors) is listed
apart and not counted; so is its relativistic conserved-to-primitive
inversion, a bisection to machine precision where the GPU runs a few Newton
steps: its count per inversion says nothing about the method's, so only the
number of inversions per zone is given.

Run:  python oracle/opcount.py
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1110_0740_amd import inputs as I  # noqa: E402

SRC = os.path.join(HERE, "opcount.cpp")
LIB = os.path.join(HERE, "libctu_opcount.so")
CATS = ["add", "mul", "div", "sqrt", "trans", "cmp", "minmax"]
NG = 4


def build() -> str:
    deps = [SRC, O.SRC]
    if not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(d) for d in deps):
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fpermissive", "-w", "-fno-fast-math",
                               "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC], cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def counted_step(o, U, L0, dt, ch):
    """Counter rows (10 x 7) of one oracle step in the op-counting build."""
    lib = O.configure(C.CDLL(build()))
    lib.opc_read.argtypes = [C.POINTER(C.c_uint64)]
    saved = O.lib()
    O._lib = lib
    try:
        lib.opc_reset()
        out = O.step(o, U, NG, dt, ch, L0=L0)
        buf = (C.c_uint64 * 78)()
        lib.opc_read(buf)
    finally:
        O._lib = saved
    assert out[3] == [0] * 5
    rows = np.array(buf[:77], dtype=np.float64).reshape(11, 7)
    rows = np.vstack([rows, np.full((1, 7), float(buf[77]))])
    # a stage the option set skips keeps a zero row: carry the previous one
    for k in range(1, 8):
        if not rows[k].any():
            rows[k] = rows[k - 1]
    return rows


def per_zone(rows, n, dim, par):
    """Per-zone counts per stage (7 x 7) from the stage rows of a box with
    interior n (tuple of dim extents)."""
    N = [x + 2 * NG for x in n]
    nc = float(np.prod(N))
    faces_all = sum((N[d] - 1) * np.prod([N[e] for e in range(dim) if e != d]) for d in range(dim))
    pred = sum((n[d] + 2) * np.prod([n[e] for e in range(dim) if e != d]) for d in range(dim))
    faces_int = sum((n[d] + 1) * np.prod([n[e] for e in range(dim) if e != d]) for d in range(dim))
    zones = float(np.prod(n))
    units = [nc, faces_all, pred, faces_int, nc, faces_int, zones]   # work units of the box, per stage
    per = [1, dim, dim, dim, 1, dim, 1]                              # units the method needs per zone
    delta = np.diff(rows[0:8], axis=0)  # stage k = rows[k] - rows[k-1]
    out = np.zeros((7, 7))
    for k in range(7):
        if k in (4, 5) and not par:
            continue
        out[k] = delta[k] / units[k] * per[k]
    return out


def flops(v):
    return float(v[0] + v[1] + v[2] + v[3] + v[4])


def workload(name):
    if name == "C1":
        n = (64, 64)
        V, meta = I.mhd2d_fields(n=128, ng=NG, seed=1000, box=I.Box((0, 0, 0), (64, 64, 1)))
        o = O.make_opts(dim=2, recon="lin_mc", riemann="hlld", gamma=meta["gamma"], dx=meta["dx"])
        return o, V, None, n, 2, None, 0.4, 1.0
    if name in ("C2", "C5"):
        seed = 2000 if name == "C2" else 5000
        n = (32, 32, 32)
        V, meta = I.mhd3d_fields(ng=NG, seed=seed, box=I.Box((0, 0, 0), n), level_n=256)
        kw = dict(recon="ppm", riemann="hlld")
        L0 = None
        if name == "C5":
            coef = I.nonideal_coeffs(5001)
            T = V[4] / V[0]
            kw.update(parabolic_mask=7, tc_phi=0.3, cooling=True, cool_beta=0.5, T_floor=0.1 * float(T.min()),
                      **coef)
            L0 = V[4] / ((meta["gamma"] - 1) * V[0] ** 2 * np.sqrt(T) * 1e-3)
        o = O.make_opts(dim=3, gamma=meta["gamma"], dx=meta["dx"], **kw)
        o_hyp = O.make_opts(dim=3, gamma=meta["gamma"], dx=meta["dx"], recon="ppm", riemann="hlld")
        return o, V, L0, n, 3, (o_hyp if name == "C5" else None), 0.4, 1.0
    if name == "C4":
        n = (32, 32, 32)
        V, meta = I.rmhd3d_fields(n=192, ng=NG, seed=4000, box=I.Box((80, 80, 80), n))
        o = O.make_opts(dim=3, physics="rmhd", predictor="mh", recon="lin_mc", riemann="hll", gamma=meta["gamma"],
                        dx=meta["dx"])
        return o, V, None, n, 3, None, 0.3, 1.0
    raise KeyError(name)


DESC = {"C1": "2D ideal MHD 128^2, MC-linear characteristic + HLLD + GLM (FP64)",
        "C2": "3D ideal MHD 256^3, PPM characteristic + HLLD + GLM (also the AMR patches' options)",
        "C4": "3D RMHD 192^3, MUSCL-Hancock + MC + HLL + GLM, ideal EOS 4/3",
        "C5": "3D non-ideal MHD 256^3, PPM + HLLD + GLM + viscosity, resistivity, saturated conduction, cooling"}
STAGES = ["prim recovery", "t^n fluxes", "predict+couple", "final solves", "V^{n+1/2}", "Pi^{n+1/2}",
          "update+sources"]
KERNELS = {"prim": [0], "tcouple": [1, 4], "sweeps": [2, 3, 5, 6]}
# parabolic runs: row 7 = the t^n stage without parabolic terms, row 8 = Pi^n
KERNELS_PAR = {"prim": [0], "tcouple": [7, 4], "pdiv": [8], "pflux": [5], "sweeps": [2, 3, 6]}


def main():
    lines = ["# Algorithmic operations per zone (op-counting build of the FP64 oracle)", "",
             "Command: `python oracle/opcount.py` (builds `oracle/libctu_opcount.so` from `oracle/opcount.cpp`,",
             "which compiles `oracle/ctu_oracle.c` unchanged with a counting double).", "",
             "Per stage: the oracle's count on a 32^3 (2D: 64^2) sub-box of the workload's fields, per unit of",
             "work in that stage, times the units the method needs per interior zone (see the script's",
             "docstring). FLOP = add + mul + div + sqrt + transcendental; FMA counts 2.", ""]
    result = {}
    for name in ("C1", "C2", "C4", "C5"):
        o, V, L0, n, dim, o_hyp, cfl, _ = workload(name)
        par = o_hyp is not None
        U = O.prim2cons(o, V)
        dt = cfl / O.cfl_rate(o, U, NG)
        ch = cfl * o.dx[0] / dt
        if o.physics == 1:
            ch = min(ch, 1.0)
        rows = counted_step(o, U, L0, dt, ch)
        pz = per_zone(rows, n, dim, par)
        kernels = KERNELS
        if par:
            tn_hyp = per_zone(counted_step(o_hyp, U, None, dt, ch), n, dim, False)[1]
            pz = np.vstack([pz, tn_hyp, pz[1] - tn_hyp])
            kernels = KERNELS_PAR
        side = rows[9] / float(np.prod(n))
        ninv = rows[11][0] / float(np.prod(n))
        kflops = {k: sum(flops(pz[s]) for s in v) for k, v in kernels.items()}
        total = sum(kflops.values())
        result[name] = (pz, kflops, total, side)
        lines.append(f"## {name}: {DESC[name]}")
        lines.append("")
        lines.append("| stage | " + " | ".join(CATS) + " | FLOP |")
        lines.append("|---|" + "---|" * (len(CATS) + 1))
        for s in range(7):
            if s in (4, 5) and not par:
                continue
            lines.append(f"| {STAGES[s]} | " + " | ".join(f"{x:.1f}" for x in pz[s]) + f" | {flops(pz[s]):.1f} |")
        if par:
            for s, lab in ((7, "(t^n fluxes without parabolic terms)"), (8, "(of which Pi^n)")):
                lines.append(f"| {lab} | " + " | ".join(f"{x:.1f}" for x in pz[s]) + f" | {flops(pz[s]):.1f} |")
        lines.append("")
        lines.append("FLOP per zone by kernel: " + ", ".join(f"{k} {v:.0f}" for k, v in kflops.items()) +
                     f"; step {total:.0f}.")
        if side.any():
            lines.append(f"Numerical eigenvector inversions (not counted): {flops(side):.0f} FLOP per zone.")
        if ninv:
            lines.append(f"Relativistic inversions (not counted): {ninv:.1f} per zone of the oracle's box "
                         f"(bisection: {flops(rows[10]) / rows[11][0]:.0f} FLOP each).")
        lines.append("")
    out = os.path.join(ROOT, "profiles", "oracle_opcount.md")
    with open(out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))
    return result


if __name__ == "__main__":
    main()
