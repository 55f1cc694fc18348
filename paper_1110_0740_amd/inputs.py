"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method itself: it draws random mode
parameters with a counter-free SplitMix64 stream, evaluates smooth periodic
fields (sums of Fourier modes, analytic curls, compact blob profiles) at cell
centres, and copies ghost zones by index wrapping.  Primitive fields come out
as float64 arrays ``V[9, NZ, NY, NX]`` over the ghosted box, in the order
(rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi); each side converts them to
conserved variables with its own routines.

Workload recipes (Sec. 5 / Sec. 6 style smooth MHD and RMHD states):
  * 2D ideal MHD, 128^2, Gamma = 5/3  -> :func:`mhd2d_fields`
  * 3D ideal MHD, 256^3 (beta ~ 1, Mach ~ 1) -> :func:`mhd3d_fields`
  * 3D relativistic MHD jets/blobs, Gamma = 4/3 -> :func:`rmhd3d_fields`
  * 3D non-ideal MHD with per-cell cooling times -> :func:`mhd3d_fields` +
    :func:`cooling_time_field`
  * 3D AMR patch hierarchy around density blobs -> :func:`amr_hierarchy`
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
NVAR = 9
RHO, VX1, VX2, VX3, PRS, BX1, BX2, BX3, PSI = range(9)


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood 2014): state += golden gamma, then a
    two-round xor-shift-multiply finaliser."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform on [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + int(self.uniform() * (hi - lo + 1))

    def normal(self) -> float:
        u1 = max(self.uniform(), 1e-300)
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


@dataclass
class Modes:
    """A sum of ``len(k)`` cosine modes with weights ``amp``:
    S(x) = sum_m amp_m cos(2 pi k_m . x + phi_m)."""

    k: np.ndarray  # (M, 3) integers
    phi: np.ndarray  # (M,)
    amp: np.ndarray  # (M,)

    def rms(self) -> float:
        return float(math.sqrt(0.5 * float(np.sum(self.amp ** 2))))


def draw_modes(rng: SplitMix64, dim: int, nmodes: int = 8, kmax: float = 4.0) -> Modes:
    """Integer wave vectors with 0 < |k| <= kmax (k_z = 0 in 2D), uniform
    phases, equal weights 1/nmodes so that |S| <= 1."""
    ks, phis = [], []
    kr = int(math.floor(kmax))
    while len(ks) < nmodes:
        k = [rng.randint(-kr, kr), rng.randint(-kr, kr), rng.randint(-kr, kr) if dim == 3 else 0]
        n2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
        if n2 == 0 or n2 > kmax * kmax:
            continue
        ks.append(k)
        phis.append(2.0 * math.pi * rng.uniform())
    return Modes(np.array(ks, dtype=np.int64), np.array(phis), np.full(nmodes, 1.0 / nmodes))


def mode_sum(m: Modes, X, Y, Z):
    out = np.zeros(np.broadcast(X, Y, Z).shape)
    for k, ph, a in zip(m.k, m.phi, m.amp):
        out += a * np.cos(2.0 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
    return out


def mode_grad(m: Modes, X, Y, Z):
    """Analytic gradient (dS/dx, dS/dy, dS/dz)."""
    shape = np.broadcast(X, Y, Z).shape
    g = [np.zeros(shape), np.zeros(shape), np.zeros(shape)]
    for k, ph, a in zip(m.k, m.phi, m.amp):
        s = np.sin(2.0 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        for c in range(3):
            g[c] -= a * 2.0 * math.pi * k[c] * s
    return g


def curl_rms(A: list[Modes]) -> float:
    """Analytic rms of curl(A) for A = (Ax, Ay, Az) mode sums, counting each
    mode's mean square independently."""
    tot = 0.0
    for c, m in enumerate(A):
        if m is None:
            continue
        for k, a in zip(m.k, m.amp):
            kk = (2.0 * math.pi) ** 2 * (float(np.dot(k, k)) - float(k[c]) ** 2)
            tot += 0.5 * a * a * kk
    return math.sqrt(tot)


@dataclass
class Box:
    """Interior index box on one level: lo (global cell index), n (extent)."""

    lo: tuple
    n: tuple
    level: int = 0


def cell_centres(box: Box, ng: int, dx: tuple, dim: int):
    """Cell-centre coordinates of the ghosted box (periodic unit domain,
    cell i covers [i dx, (i+1) dx))."""
    gz = ng if dim == 3 else 0
    ax = []
    for d in range(3):
        g = ng if d < dim else gz
        if d >= dim:
            ax.append(np.array([0.5 * dx[d]]))
            continue
        idx = np.arange(box.lo[d] - g, box.lo[d] + box.n[d] + g)
        ax.append((idx + 0.5) * dx[d])
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------


def mhd2d_fields(n: int = 128, ng: int = 4, seed: int = 1000, box: Box | None = None):
    """2D ideal MHD, Gamma = 5/3, periodic unit square: rho = 1 + 0.2 S,
    p = 1 + 0.2 S', each velocity component 0.5 S, B_z = 0.5 S, and
    (B_x, B_y) = 0.5 curl(A_z z) / bound, where bound majorises |curl A_z|."""
    rng = SplitMix64(seed)
    dim = 2
    m = {name: draw_modes(rng, dim) for name in ("rho", "p", "vx", "vy", "vz", "Az", "Bz")}
    if box is None:
        box = Box((0, 0, 0), (n, n, 1))
    dx = (1.0 / n, 1.0 / n, 1.0)
    X, Y, Z = cell_centres(box, ng, dx, dim)
    V = np.zeros((NVAR,) + X.shape)
    V[RHO] = 1.0 + 0.2 * mode_sum(m["rho"], X, Y, Z)
    V[PRS] = 1.0 + 0.2 * mode_sum(m["p"], X, Y, Z)
    V[VX1] = 0.5 * mode_sum(m["vx"], X, Y, Z)
    V[VX2] = 0.5 * mode_sum(m["vy"], X, Y, Z)
    V[VX3] = 0.5 * mode_sum(m["vz"], X, Y, Z)
    gAx, gAy, _ = mode_grad(m["Az"], X, Y, Z)
    bound = sum(a * 2.0 * math.pi * math.sqrt(float(np.dot(k, k))) for k, a in zip(m["Az"].k, m["Az"].amp))
    V[BX1] = 0.5 * gAy / bound
    V[BX2] = -0.5 * gAx / bound
    V[BX3] = 0.5 * mode_sum(m["Bz"], X, Y, Z)
    return V, dict(dim=2, gamma=5.0 / 3.0, dx=dx, box=box, ng=ng)


def mhd3d_fields(n: int = 256, ng: int = 4, seed: int = 2000, box: Box | None = None, level_n: int | None = None,
                 v_rms: float = 1.0, b_rms: float | None = None):
    """3D ideal MHD, Gamma = 5/3, periodic unit cube: rho = 1 + 0.5 S in
    [0.5, 1.5], p = 0.6 (1 + 0.2 S'), velocity components scaled to a total
    rms of v_rms (Mach ~ 1 for v_rms = 1, c_s ~ 1), B = curl A scaled to
    rms sqrt(2 * 0.6) (plasma beta ~ 1)."""
    rng = SplitMix64(seed)
    dim = 3
    m = {name: draw_modes(rng, dim) for name in ("rho", "p", "vx", "vy", "vz", "Ax", "Ay", "Az")}
    N = level_n if level_n is not None else n
    if box is None:
        box = Box((0, 0, 0), (n, n, n))
    dx = (1.0 / N, 1.0 / N, 1.0 / N)
    X, Y, Z = cell_centres(box, ng, dx, dim)
    V = np.zeros((NVAR,) + X.shape)
    V[RHO] = 1.0 + 0.5 * mode_sum(m["rho"], X, Y, Z)
    V[PRS] = 0.6 * (1.0 + 0.2 * mode_sum(m["p"], X, Y, Z))
    for c, name in enumerate(("vx", "vy", "vz")):
        V[VX1 + c] = (v_rms / math.sqrt(3.0)) / m[name].rms() * mode_sum(m[name], X, Y, Z)
    A = [m["Ax"], m["Ay"], m["Az"]]
    if b_rms is None:
        b_rms = math.sqrt(2.0 * 0.6)
    scale = b_rms / curl_rms(A)
    g = [mode_grad(a, X, Y, Z) for a in A]
    V[BX1] = scale * (g[2][1] - g[1][2])
    V[BX2] = scale * (g[0][2] - g[2][0])
    V[BX3] = scale * (g[1][0] - g[0][1])
    return V, dict(dim=3, gamma=5.0 / 3.0, dx=dx, box=box, ng=ng)


def cooling_time_field(seed: int, X, Y, Z, dt0: float, dim: int = 3):
    """Per-cell cooling time t_c = dt0 * 10^(3 S_c) (t_c / dt0 in [1e-3, 1e3])."""
    rng = SplitMix64(seed)
    m = draw_modes(rng, dim)
    return dt0 * 10.0 ** (3.0 * mode_sum(m, X, Y, Z))


def nonideal_coeffs(seed: int):
    """nu, eta, kappa_par, kappa_perp ~ log-uniform on [1e-4, 1e-2], with
    kappa_perp <= kappa_par."""
    rng = SplitMix64(seed)
    draw = lambda: 10.0 ** (-4.0 + 2.0 * rng.uniform())
    nu, eta, k1, k2 = draw(), draw(), draw(), draw()
    return dict(nu=nu, eta=eta, kappa_par=max(k1, k2), kappa_perp=min(k1, k2))


def rmhd3d_fields(n: int = 192, ng: int = 4, seed: int = 4000, box: Box | None = None, gmax_cap: float = 10.0):
    """3D relativistic MHD, Gamma = 4/3, periodic unit cube.  Background
    rho = 1, p = 0.1.  Two periodic cylindrical jets along seeded axes and six
    spherical blobs, each with the C^1 profile P = (1 - (r/R)^2)^2, radius
    R in [0.05, 0.12], central density in [0.1, 1] and central Lorentz
    factor g_max in [2, 10] (the first equal to the cap): log(rho) and the
    spatial 4-velocity sqrt(g_max^2 - 1) P d (d the object's direction) add
    over overlapping objects.  B = uniform + mode sum, scaled so that max b^2/w = 1 would hold
    at the background state."""
    rng = SplitMix64(seed)
    dim = 3
    if box is None:
        box = Box((0, 0, 0), (n, n, n))
    dx = (1.0 / n, 1.0 / n, 1.0 / n)
    X, Y, Z = cell_centres(box, ng, dx, dim)
    shape = X.shape
    prs = np.full(shape, 0.1)
    objs = []
    for j in range(8):
        kind = "jet" if j < 2 else "blob"
        c = np.array([rng.uniform(), rng.uniform(), rng.uniform()])
        R = 0.05 + 0.07 * rng.uniform()
        dens = 0.1 + 0.9 * rng.uniform()
        gmax = gmax_cap if j == 0 else 2.0 + (gmax_cap - 2.0) * rng.uniform()
        axis = rng.randint(0, 2)
        # direction of motion: along the jet axis, random for blobs
        if kind == "jet":
            dvec = np.zeros(3)
            dvec[axis] = 1.0 if rng.uniform() < 0.5 else -1.0
        else:
            dvec = np.array([rng.normal(), rng.normal(), rng.normal()])
            dvec /= np.linalg.norm(dvec)
        objs.append((kind, c, R, dens, gmax, axis, dvec))
    # smooth superposition: log-density and spatial 4-velocity u = gamma v
    # add up the objects' profiles, so the fields stay C^1 where they overlap
    logrho = np.zeros(shape)
    u = np.zeros((3,) + shape)
    for kind, c, R, dens, gmax, axis, dvec in objs:
        d = []
        for q, Q in enumerate((X, Y, Z)):
            t = Q - c[q]
            t = t - np.round(t)  # periodic minimum image
            d.append(t)
        if kind == "jet":
            r2 = sum(d[q] ** 2 for q in range(3) if q != axis)
        else:
            r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
        x = np.clip(r2 / (R * R), 0.0, 1.0)
        prof = (1.0 - x) ** 2
        logrho += math.log(dens) * prof
        umax = math.sqrt(gmax * gmax - 1.0)
        for q in range(3):
            u[q] += umax * prof * dvec[q]
    umag = np.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    ucap = math.sqrt(gmax_cap * gmax_cap - 1.0)
    fac = np.where(umag > ucap, ucap / np.maximum(umag, 1e-300), 1.0)
    u *= fac
    lor = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    rho = np.exp(logrho)
    vel = u / lor
    V = np.zeros((NVAR,) + shape)
    V[RHO] = rho
    V[PRS] = prs
    V[VX1:VX1 + 3] = vel
    # magnetic field: uniform part + divergence-free mode sum, magnetization <= 1
    G = 4.0 / 3.0
    w_bg = 1.0 + G * 0.1 / (G - 1.0)
    b0 = math.sqrt(0.5 * w_bg)
    th = math.acos(2.0 * rng.uniform() - 1.0)
    ph = 2.0 * math.pi * rng.uniform()
    B0 = b0 * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    A = [draw_modes(rng, dim) for _ in range(3)]
    scale = 0.5 * b0 / curl_rms(A)
    g = [mode_grad(a, X, Y, Z) for a in A]
    V[BX1] = B0[0] + scale * (g[2][1] - g[1][2])
    V[BX2] = B0[1] + scale * (g[0][2] - g[2][0])
    V[BX3] = B0[2] + scale * (g[1][0] - g[0][1])
    return V, dict(dim=3, gamma=G, dx=dx, box=box, ng=ng)


# --------------------------------------------------------------------------
# Ghost zones (pure index copies)
# --------------------------------------------------------------------------


def fill_periodic(U: np.ndarray, ng: int, dim: int) -> None:
    """Copy periodic images into the ghost zones of one ghosted box in place
    (arrays shaped [..., NZ, NY, NX])."""
    axes = [-1, -2, -3][:dim]
    for ax in axes:
        n = U.shape[ax] - 2 * ng
        sl = [slice(None)] * U.ndim
        src = [slice(None)] * U.ndim
        sl[ax] = slice(0, ng)
        src[ax] = slice(n, n + ng)
        U[tuple(sl)] = U[tuple(src)]
        sl[ax] = slice(n + ng, n + 2 * ng)
        src[ax] = slice(ng, 2 * ng)
        U[tuple(sl)] = U[tuple(src)]


def fill_outflow(U: np.ndarray, ng: int, dim: int) -> None:
    """Zero-gradient ghost zones (copy of the nearest interior cell)."""
    axes = [-1, -2, -3][:dim]
    for ax in axes:
        n = U.shape[ax] - 2 * ng
        for g in range(ng):
            sl = [slice(None)] * U.ndim
            src = [slice(None)] * U.ndim
            sl[ax] = slice(g, g + 1)
            src[ax] = slice(ng, ng + 1)
            U[tuple(sl)] = U[tuple(src)]
            sl[ax] = slice(n + ng + g, n + ng + g + 1)
            src[ax] = slice(n + ng - 1, n + ng)
            U[tuple(sl)] = U[tuple(src)]


def interior(a: np.ndarray, ng: int, dim: int) -> np.ndarray:
    sl = [slice(None)] * a.ndim
    for q, ax in enumerate([-1, -2, -3]):
        if q < dim:
            sl[ax] = slice(ng, a.shape[ax] - ng)
    return a[tuple(sl)]


def sub_box(a: np.ndarray, lo: tuple, n: tuple, ng: int, dim: int) -> np.ndarray:
    """Extract the ghosted sub-box whose interior starts at interior index lo
    (relative to the big box's interior) with extent n, from a ghosted array."""
    sl = [slice(None)] * a.ndim
    for q, ax in enumerate([-1, -2, -3]):
        if q < dim:
            s = lo[q]
            sl[ax] = slice(s, s + n[q] + 2 * ng)
    return np.ascontiguousarray(a[tuple(sl)])


# --------------------------------------------------------------------------
# Device-side evaluation of the same recipes (torch), for full-size runs
# --------------------------------------------------------------------------


def _axis_phases(torch, box: Box, ng: int, dx: tuple, dim: int, device):
    """exp(2 pi i x) factors per axis at ghosted cell centres, as a list of
    functions k -> complex 1D tensor (separable form of cos(2 pi k.x + phi))."""
    cache = []
    for d in range(3):
        if d >= dim:
            x = torch.tensor([0.5 * dx[d]], dtype=torch.float64, device=device)
        else:
            idx = torch.arange(box.lo[d] - ng, box.lo[d] + box.n[d] + ng, dtype=torch.float64, device=device)
            x = (idx + 0.5) * dx[d]
        cache.append(x)
    return cache


def _mode_terms(torch, m: Modes, axes):
    """Complex field sum_m a_m exp(i (2 pi k_m . x + phi_m)) as [NZ, NY, NX]."""
    x, y, z = axes
    out = None
    for k, ph, a in zip(m.k, m.phi, m.amp):
        ex = torch.exp(2j * math.pi * float(k[0]) * x.to(torch.complex128))
        ey = torch.exp(2j * math.pi * float(k[1]) * y.to(torch.complex128))
        ez = torch.exp(2j * math.pi * float(k[2]) * z.to(torch.complex128)) * complex(math.cos(ph), math.sin(ph))
        term = (a * ez)[:, None, None] * ey[None, :, None] * ex[None, None, :]
        out = term if out is None else out + term
    return out


def _mode_sum_t(torch, m, axes):
    return _mode_terms(torch, m, axes).real


def _mode_grad_t(torch, m, axes):
    """Analytic gradient of the mode sum: d/dx_c cos(theta) = Re(2 pi i k_c e^{i theta})."""
    x, y, z = axes
    g = [None, None, None]
    for k, ph, a in zip(m.k, m.phi, m.amp):
        ex = torch.exp(2j * math.pi * float(k[0]) * x.to(torch.complex128))
        ey = torch.exp(2j * math.pi * float(k[1]) * y.to(torch.complex128))
        ez = torch.exp(2j * math.pi * float(k[2]) * z.to(torch.complex128)) * complex(math.cos(ph), math.sin(ph))
        base = (a * ez)[:, None, None] * ey[None, :, None] * ex[None, None, :]
        for c in range(3):
            t = (2j * math.pi * float(k[c]) * base).real
            g[c] = t if g[c] is None else g[c] + t
    return g


def mhd3d_fields_torch(n: int = 256, ng: int = 4, seed: int = 2000, device="cuda", v_rms: float = 1.0):
    """:func:`mhd3d_fields` evaluated with torch on `device` (float64,
    ghosted [9, NZ, NY, NX]); same modes, same recipe."""
    import torch

    rng = SplitMix64(seed)
    dim = 3
    m = {name: draw_modes(rng, dim) for name in ("rho", "p", "vx", "vy", "vz", "Ax", "Ay", "Az")}
    box = Box((0, 0, 0), (n, n, n))
    dx = (1.0 / n, 1.0 / n, 1.0 / n)
    axes = _axis_phases(torch, box, ng, dx, dim, device)
    N = n + 2 * ng
    V = torch.zeros((NVAR, N, N, N), dtype=torch.float64, device=device)
    V[RHO] = 1.0 + 0.5 * _mode_sum_t(torch, m["rho"], axes)
    V[PRS] = 0.6 * (1.0 + 0.2 * _mode_sum_t(torch, m["p"], axes))
    for c, name in enumerate(("vx", "vy", "vz")):
        V[VX1 + c] = (v_rms / math.sqrt(3.0)) / m[name].rms() * _mode_sum_t(torch, m[name], axes)
    A = [m["Ax"], m["Ay"], m["Az"]]
    scale = math.sqrt(2.0 * 0.6) / curl_rms(A)
    g0 = _mode_grad_t(torch, A[0], axes)
    g1 = _mode_grad_t(torch, A[1], axes)
    g2 = _mode_grad_t(torch, A[2], axes)
    V[BX1] = scale * (g2[1] - g1[2])
    V[BX2] = scale * (g0[2] - g2[0])
    V[BX3] = scale * (g1[0] - g0[1])
    return V, dict(dim=3, gamma=5.0 / 3.0, dx=dx, box=box, ng=ng)


def splitmix64_uniform(seed: int, counters: np.ndarray) -> np.ndarray:
    """The (c + 1)-th uniform draw of SplitMix64(seed) for every counter c
    (vectorised: the state after c + 1 steps is seed + (c + 1) gamma)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + (counters.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def cooling_time_white(seed: int, n: int, ng: int, dt0: float, box: Box | None = None, level_n: int | None = None):
    """White-noise cooling times on a ghosted box of the periodic level of
    level_n cells per side (default: the n^3 box itself): t_c = dt0 *
    10^(3 (2u - 1)) in [1e-3, 1e3] dt0, u uniform and independent per cell,
    drawn by SplitMix64 at the cell's periodic index (so ghosts repeat
    their images).  [NZ, NY, NX] float64."""
    N = level_n if level_n is not None else n
    if box is None:
        box = Box((0, 0, 0), (n, n, n))
    idx = [np.arange(box.lo[d] - ng, box.lo[d] + box.n[d] + ng) % N for d in range(3)]
    K, J, Iq = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    c = (K.astype(np.int64) * N + J) * N + Iq
    u = splitmix64_uniform(seed, c)
    return dt0 * 10.0 ** (3.0 * (2.0 * u - 1.0))


def cooling_time_field_torch(seed: int, n: int, ng: int, dt0: float, device="cuda"):
    """:func:`cooling_time_field` on the ghosted n^3 periodic box, with torch
    on `device` (float64, [NZ, NY, NX])."""
    import torch

    rng = SplitMix64(seed)
    m = draw_modes(rng, 3)
    box = Box((0, 0, 0), (n, n, n))
    axes = _axis_phases(torch, box, ng, (1.0 / n,) * 3, 3, device)
    return dt0 * 10.0 ** (3.0 * _mode_sum_t(torch, m, axes))


# --------------------------------------------------------------------------
# AMR hierarchy around density blobs (3 levels, refinement ratio 2)
# --------------------------------------------------------------------------


@dataclass
class Hierarchy:
    base: int                      # level-0 cells per side of the periodic unit cube
    levels: list                   # levels[l] = list of Box (level-l global indices)
    blobs: list                    # (centre (3,), radius)
    seed: int
    modes: dict = field(default_factory=dict)

    def dx(self, level: int):
        h = 1.0 / (self.base * (1 << level))
        return (h, h, h)


def _blob_bump(blobs, x, widen=1.0):
    v = 0.0
    for c, r in blobs:
        d = np.asarray(x) - c
        d = d - np.round(d)
        v = max(v, math.exp(-float(np.dot(d, d)) / (widen * r) ** 2))
    return v


def amr_hierarchy(seed: int = 3000, base: int = 128, base_box: int = 32, lattice: int = 32,
                  size_range=(16, 32), nblobs: int = 8, p1=(0.75, 1.0), p2=(0.35, 1.2), nest: int = 1) -> Hierarchy:
    """Level 0 tiles the base^3 domain with base_box^3 boxes.  Level 1 (2x)
    places at most one box per lattice^3 cell of a jittered lattice, with
    probability p1[0] + p1[1] * bump, bump = max_b exp(-|x - c_b|^2/(3 r_b)^2)
    at the lattice-cell centre; sizes are even and uniform in size_range per
    axis, origins even, one level-1 cell of margin from the domain boundary.
    Level 2 (4x) refines a level-1 box with probability p2[0] + p2[1] * bump
    (width 2 r_b) into 1 or 2 children per axis inside the parent shrunk by
    `nest` level-1 cells (2 nest level-2 cells), sizes even in size_range.
    Boxes are therefore disjoint per level and properly nested by
    construction; nest = 3 keeps the coarse stencil of every level-2 ghost
    cell (2 coarse cells deep, plus 1 for the slopes) inside the parent, as
    the coarse-to-fine ghost fill needs."""
    rng = SplitMix64(seed)
    blobs = []
    for _ in range(nblobs):
        c = np.array([0.15 + 0.7 * rng.uniform() for _ in range(3)])
        r = 0.03 + 0.05 * rng.uniform()
        blobs.append((c, r))
    levels = [[Box((i, j, k), (base_box,) * 3, 0) for k in range(0, base, base_box)
               for j in range(0, base, base_box) for i in range(0, base, base_box)]]
    lo_s, hi_s = size_range
    # level 1
    N1 = base * 2
    L1 = []
    for k in range(0, N1, lattice):
        for j in range(0, N1, lattice):
            for i in range(0, N1, lattice):
                org = (i, j, k)
                ctr = np.array([(org[q] + 0.5 * lattice) / N1 for q in range(3)])
                prob = p1[0] + p1[1] * _blob_bump(blobs, ctr, 3.0)
                if rng.uniform() >= prob:
                    continue
                lo, n = [], []
                for q in range(3):
                    a0 = max(org[q], 2)
                    a1 = min(org[q] + lattice, N1 - 2)
                    span = a1 - a0
                    nq = min(2 * rng.randint(lo_s // 2, hi_s // 2), span - span % 2)
                    off = 2 * rng.randint(0, (span - nq) // 2)
                    lo.append(a0 + off)
                    n.append(nq)
                L1.append(Box(tuple(lo), tuple(n), 1))
    levels.append(L1)
    # level 2
    L2 = []
    for P in L1:
        ctr = np.array([(P.lo[q] + 0.5 * P.n[q]) / N1 for q in range(3)])
        prob = p2[0] + p2[1] * _blob_bump(blobs, ctr, 2.0)
        if rng.uniform() >= prob:
            continue
        segs = []
        for q in range(3):
            u0 = 2 * P.lo[q] + 2 * nest
            u1 = 2 * (P.lo[q] + P.n[q]) - 2 * nest
            usable = u1 - u0
            parts = 2 if (usable >= 2 * lo_s and rng.uniform() < 0.75) else 1
            width = usable // parts
            axis = []
            for pidx in range(parts):
                s0 = u0 + pidx * width
                nq = min(2 * rng.randint(lo_s // 2, hi_s // 2), width - width % 2)
                off = 2 * rng.randint(0, (width - nq) // 2)
                axis.append((s0 + off, nq))
            segs.append(axis)
        for (x0, nx) in segs[0]:
            for (y0, ny) in segs[1]:
                for (z0, nz) in segs[2]:
                    L2.append(Box((x0, y0, z0), (nx, ny, nz), 2))
    levels.append(L2)
    return Hierarchy(base=base, levels=levels, blobs=blobs, seed=seed)


def amr_fields(h: Hierarchy, box: Box, ng: int = 4, v_rms: float = 0.5, b_rms: float = 0.5):
    """Primitive fields of the AMR workload on one ghosted box at its level:
    rho = 1 + 9 max_b exp(-|x - c_b|^2 / r_b^2) (periodic minimum image,
    contrast 10), p = 0.6, velocity and B as the 3D MHD recipe with rms
    v_rms and b_rms; Gamma = 5/3."""
    if not h.modes:
        rng = SplitMix64(h.seed + 17)
        h.modes = {name: draw_modes(rng, 3) for name in ("vx", "vy", "vz", "Ax", "Ay", "Az")}
    m = h.modes
    dx = h.dx(box.level)
    X, Y, Z = cell_centres(box, ng, dx, 3)
    V = np.zeros((NVAR,) + X.shape)
    bump = np.zeros(X.shape)
    for c, r in h.blobs:
        d2 = np.zeros(X.shape)
        for q, Q in enumerate((X, Y, Z)):
            t = Q - c[q]
            t = t - np.round(t)
            d2 += t * t
        bump = np.maximum(bump, np.exp(-d2 / (r * r)))
    V[RHO] = 1.0 + 9.0 * bump
    V[PRS] = 0.6
    for c, name in enumerate(("vx", "vy", "vz")):
        V[VX1 + c] = (v_rms / math.sqrt(3.0)) / m[name].rms() * mode_sum(m[name], X, Y, Z)
    A = [m["Ax"], m["Ay"], m["Az"]]
    scale = b_rms / curl_rms(A)
    g = [mode_grad(a, X, Y, Z) for a in A]
    V[BX1] = scale * (g[2][1] - g[1][2])
    V[BX2] = scale * (g[0][2] - g[2][0])
    V[BX3] = scale * (g[1][0] - g[0][1])
    return V


def amr_level_fields_torch(h: Hierarchy, level: int, ng: int = 4, device="cuda", v_rms: float = 0.5,
                           b_rms: float = 0.5):
    """:func:`amr_fields` of every box of one level at once, evaluated with
    torch on `device` (float64) over the flat list of the level's ghosted
    cells: the boxes' ghosted [9, NZ, NY, NX] blocks packed one after
    another in box order, as one 1D tensor.  A few hundred vector operations
    per level instead of a thousand per box."""
    import torch

    if not h.modes:
        rng = SplitMix64(h.seed + 17)
        h.modes = {name: draw_modes(rng, 3) for name in ("vx", "vy", "vz", "Ax", "Ay", "Az")}
    m = h.modes
    L = h.levels[level]
    dx = h.dx(level)
    idx, sizes = [[], [], []], []
    for B in L:
        ax = [np.arange(B.lo[d] - ng, B.lo[d] + B.n[d] + ng) for d in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        for d, Q in enumerate((X, Y, Z)):
            idx[d].append(Q.ravel())
        sizes.append(X.size)
    ncell = int(sum(sizes))
    xs = [(torch.from_numpy(np.concatenate(idx[d]) if sizes else np.zeros(0, np.int64)).to(device=device,
                                                                                              dtype=torch.float64)
           + 0.5) * dx[d] for d in range(3)]
    x, y, z = xs

    def modesum(mm):
        out = torch.zeros(ncell, dtype=torch.float64, device=device)
        for k, ph, a in zip(mm.k, mm.phi, mm.amp):
            out += a * torch.cos(2.0 * math.pi * (float(k[0]) * x + float(k[1]) * y + float(k[2]) * z) + ph)
        return out

    def modegrad(mm):
        g = [torch.zeros(ncell, dtype=torch.float64, device=device) for _ in range(3)]
        for k, ph, a in zip(mm.k, mm.phi, mm.amp):
            sn = torch.sin(2.0 * math.pi * (float(k[0]) * x + float(k[1]) * y + float(k[2]) * z) + ph)
            for c in range(3):
                g[c] -= a * 2.0 * math.pi * float(k[c]) * sn
        return g

    F = torch.empty((NVAR, ncell), dtype=torch.float64, device=device)
    bump = torch.zeros(ncell, dtype=torch.float64, device=device)
    for c, r in h.blobs:
        d2 = torch.zeros(ncell, dtype=torch.float64, device=device)
        for q, Q in enumerate(xs):
            t = Q - float(c[q])
            t = t - torch.round(t)
            d2 += t * t
        bump = torch.maximum(bump, torch.exp(-d2 / (r * r)))
    F[RHO] = 1.0 + 9.0 * bump
    F[PRS] = 0.6
    for c, name in enumerate(("vx", "vy", "vz")):
        F[VX1 + c] = (v_rms / math.sqrt(3.0)) / m[name].rms() * modesum(m[name])
    A = [m["Ax"], m["Ay"], m["Az"]]
    scale = b_rms / curl_rms(A)
    g = [modegrad(a) for a in A]
    F[BX1] = scale * (g[2][1] - g[1][2])
    F[BX2] = scale * (g[0][2] - g[2][0])
    F[BX3] = scale * (g[1][0] - g[0][1])
    F[PSI] = 0.0
    out = torch.empty(NVAR * ncell, dtype=torch.float64, device=device)
    s0 = 0
    for n in sizes:
        out[NVAR * s0:NVAR * (s0 + n)].view(NVAR, n).copy_(F[:, s0:s0 + n])
        s0 += n
    return out


def amr_fields_torch(h: Hierarchy, box: Box, ng: int = 4, device="cuda", v_rms: float = 0.5, b_rms: float = 0.5):
    """:func:`amr_fields` evaluated with torch on `device` (float64)."""
    import torch

    if not h.modes:
        rng = SplitMix64(h.seed + 17)
        h.modes = {name: draw_modes(rng, 3) for name in ("vx", "vy", "vz", "Ax", "Ay", "Az")}
    m = h.modes
    dx = h.dx(box.level)
    axes = _axis_phases(torch, box, ng, dx, 3, device)
    x, y, z = axes
    shape = (z.numel(), y.numel(), x.numel())
    V = torch.zeros((NVAR,) + shape, dtype=torch.float64, device=device)
    bump = torch.zeros(shape, dtype=torch.float64, device=device)
    for c, r in h.blobs:
        tx = x - c[0]
        tx = tx - torch.round(tx)
        ty = y - c[1]
        ty = ty - torch.round(ty)
        tz = z - c[2]
        tz = tz - torch.round(tz)
        d2 = tz[:, None, None] ** 2 + ty[None, :, None] ** 2 + tx[None, None, :] ** 2
        bump = torch.maximum(bump, torch.exp(-d2 / (r * r)))
    V[RHO] = 1.0 + 9.0 * bump
    V[PRS] = 0.6
    for c, name in enumerate(("vx", "vy", "vz")):
        V[VX1 + c] = (v_rms / math.sqrt(3.0)) / m[name].rms() * _mode_sum_t(torch, m[name], axes)
    A = [m["Ax"], m["Ay"], m["Az"]]
    scale = b_rms / curl_rms(A)
    g0 = _mode_grad_t(torch, A[0], axes)
    g1 = _mode_grad_t(torch, A[1], axes)
    g2 = _mode_grad_t(torch, A[2], axes)
    V[BX1] = scale * (g2[1] - g1[2])
    V[BX2] = scale * (g0[2] - g2[0])
    V[BX3] = scale * (g1[0] - g0[1])
    return V
