// ctu_kernels.hpp -- HIP kernels of the CTU-GLM step (Sec. 3.1) for gfx950.
//
// One step of a batch of ghosted boxes is a short chain of launches:
//   k_reset      zero the rate / dpp / failure outputs (graph-safe, no memset)
//   k_cons2prim  V = V(U) on every ghosted cell                       (a1)
//   k_shock_hll, k_shock_mm
//                App. B zone flags (shock-adaptive runs only)
//   k_pdiv       parabolic runs: the parabolic fluxes Pi^n of V^n on
//                every face of the region [g-1, g+n], differenced per cell (a3)
//   k_tcouple    first-order fluxes R(V_j, V_{j+1}) at t^n on those
//                faces, differenced into the per-cell increments T_d of
//                Eq. transv (plus the Pi^n divergence); with parabolic
//                terms also the cell-centred V^{n+1/2}       (a2, a3, a5, a7)
//   k_pflux      parabolic runs: Pi^{n+1/2} of V^{n+1/2} on the faces
//                g .. g+n of the sweeps                                (a8)
//   k_mtflux<D>, k_mtT
//                instead of k_tcouple with the MT corner coupling: the
//                transverse fluxes between normal-predictor states and their
//                differences T_d
//   k_sweep<D>   for direction D: normal predictor, corner coupling
//                (Eq. transv), final Riemann solve (Eq. ctu_flux), flux
//                registers, and the conservative update of U^{n+1}; the
//                last sweep also applies the split sources and reduces the
//                CFL rate of Eq. Ca                                    (a4-a10)
// Work is described by tables of tiles (box, range) so that boxes of any
// size and level run in one launch per kernel.
#pragma once
#include <type_traits>

#include "ctu_device.hpp"

namespace ctu {

constexpr int NT = 256;  // threads per block

// Block index in an XCD-contiguous order for launches whose consecutive
// blocks touch neighbouring data: the dispatcher sends block b to XCD b % 8
// (each XCD with its own L2), so block b works on item x * q + min(x, r) +
// b / 8 of the n blocks' list, x = b % 8, q = n / 8, r = n % 8: every XCD
// takes a contiguous run (the order the host gives the tile tables).
__device__ __forceinline__ int xcd_block(int b, int n)
{
    if (n < 16) return b;
    const int x = b & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

struct KBox {
    int N[3];      // ghosted extents (N[2] = 1 in 2D)
    int n[3];      // interior extents
    int g[3];      // ghost widths (g[2] = 0 in 2D)
    int lo[3];     // level-global index of the first interior cell
    long long uoff;  // element offset of the box block in caller arrays
    long long woff;  // element offset of the box block in workspace arrays
    long long cells; // N0*N1*N2
    double dx[3];
    int reg0, reg1;  // register entries [reg0, reg1), sorted by (dir, face)
    // per direction d: offset of this box's face index in the register face
    // table: entries [t[f], t[f + 1]) lie on the face lo[d] + f, f = 0..n[d]
    int rface[3];
    int lshift;  // the box's level when the plan's dt is the level-0 step (one plan over
                 // several levels); 0 otherwise.  The box steps by dt / 2^lshift and
                 // reports its rate times 2^-lshift (the level-0 rate of its CFL number)
};

// the step of a box: the plan's dt, halved per level of a multi-level plan
// (exact: a power-of-two scaling)
__device__ __forceinline__ double box_dt(const KBox &bx, const double *params)
{
    return ldexp(params[0], -bx.lshift);
}

struct KTile {
    int box, a, b, c;
};

struct KReg {
    int dir, face, tlo0, tlo1, tn0, tn1, pad0, pad1;
    long long slot;
};

// cell offset inside one box block (a box block of nine planes is below 4 GiB,
// checked at plan creation, so 32-bit offsets address every variable)
__device__ __forceinline__ int cidx(const KBox &bx, int i, int j, int k)
{
    return (k * bx.N[1] + j) * bx.N[0] + i;
}

// Raw-buffer view of one box's block of an array: NV variable planes of
// `cells` elements each.  An access takes the plane start in a scalar
// register and the cell's byte offset in a 32-bit vector register, so no
// 64-bit address arithmetic is done per element.  The block's byte size
// (below 4 GiB, checked at plan creation) is the hardware range limit:
// loads past it read 0 and stores past it are dropped.
template <typename R> struct Blk {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t pb;  // bytes per variable plane

    __device__ __forceinline__ Blk(const R *base, long long cells)
        : rs(__builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(uint32_t)(NV * cells * sizeof(R)),
                                               0x00020000)),
          pb((uint32_t)(cells * sizeof(R)))
    {
    }
    // element e >= 0 of variable plane q
    __device__ __forceinline__ R ld(int q, int e) const
    {
        const int vo = (int)((uint32_t)e * (uint32_t)sizeof(R)), so = (int)((uint32_t)q * pb);
        if constexpr (sizeof(R) == 4)
            return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
        else
            return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
    }
    __device__ __forceinline__ void st(int q, int e, R v) const
    {
        const int vo = (int)((uint32_t)e * (uint32_t)sizeof(R)), so = (int)((uint32_t)q * pb);
        if constexpr (sizeof(R) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, vo, so, 0);
        } else {
            using W = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, v), rs, vo, so, 0);
        }
    }
};

template <int D> __device__ __forceinline__ void unit(int &di, int &dj, int &dk)
{
    di = (D == 0);
    dj = (D == 1);
    dk = (D == 2);
}

__device__ __forceinline__ void count_fails(int f, int *fails)
{
    if (f && fails) {
        if (f & F_RHO) atomicAdd(&fails[0], 1);
        if (f & F_PRS) atomicAdd(&fails[1], 1);
        if (f & F_INV) atomicAdd(&fails[2], 1);
        if (f & F_VEL) atomicAdd(&fails[3], 1);
        if (f & F_NAN) atomicAdd(&fails[4], 1);
    }
}

// non-negative doubles order like their bit patterns
__device__ __forceinline__ void atomic_max_pos(double *addr, double v)
{
    atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double block_max(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int q = 1; q < NT / 64; q++) r = fmax(r, red[q]);
    __syncthreads();
    return r;
}

template <int Z = 0> __global__ void k_reset(double *rate, double *dpp, int *fails)
{
    int t = threadIdx.x;
    if (t == 0 && rate) rate[0] = 0.0;
    if (t == 1 && dpp) dpp[0] = 0.0;
    if (t >= 2 && t < 2 + 5 && fails) fails[t - 2] = 0;
}

// ---------------------------------------------------------------------------
// elementwise maps: tile = (box, first cell); one cell per thread
// ---------------------------------------------------------------------------

template <int PHYS, typename R>
__global__ __launch_bounds__(NT) void k_cons2prim(const KBox *boxes, const KTile *tiles, const R *U, R *V,
                                                  int *fails, R gam, int out_ws)
{
    KTile tl = tiles[blockIdx.x];
    const KBox &bx = boxes[tl.box];
    long long c = tl.a + threadIdx.x;
    if (c >= bx.cells) return;
    R u[NV], v[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) u[q] = U[bx.uoff + q * bx.cells + c];
    int f = c2p<PHYS>(u, v, gam);
    count_fails(f, fails);
    long long o = out_ws ? bx.woff : bx.uoff;
#pragma unroll
    for (int q = 0; q < NV; q++) V[o + q * bx.cells + c] = v[q];
}

template <int PHYS, typename R>
__global__ __launch_bounds__(NT) void k_prim2cons(const KBox *boxes, const KTile *tiles, const R *V, R *U, R gam)
{
    KTile tl = tiles[blockIdx.x];
    const KBox &bx = boxes[tl.box];
    long long c = tl.a + threadIdx.x;
    if (c >= bx.cells) return;
    R u[NV], v[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = V[bx.uoff + q * bx.cells + c];
    p2c<PHYS>(v, u, gam);
#pragma unroll
    for (int q = 0; q < NV; q++) U[bx.uoff + q * bx.cells + c] = u[q];
}

// ---------------------------------------------------------------------------
// Kernel variants of the t^n kernel and the sweeps: generic (every option
// read at run time), shock (App. B flags in use), fast: the common option
// set (face-value reference states, GLM on, hyperbolic fluxes on, no
// parabolic terms, no cooling) fixed at compile time, so that the code of the
// other options folds away (about half the instructions and registers of the
// generic sweep), and par: the same fixed set with parabolic terms and
// cooling read at run time (non-ideal runs).
// ---------------------------------------------------------------------------
constexpr int VAR_GENERIC = 0, VAR_SHOCK = 1, VAR_FAST = 2, VAR_PAR = 3;

template <int VAR> __device__ __forceinline__ KOpts variant_opts(const KOpts &in)
{
    KOpts o = in;
    if constexpr (VAR == VAR_FAST || VAR == VAR_PAR) {
        o.wref = WREF_FACE;
        o.glm = 1;
        o.hyp_off = 0;
    }
    if constexpr (VAR == VAR_FAST) {
        o.parab = 0;
        o.cooling = 0;
    }
    return o;
}

// ---------------------------------------------------------------------------
// App. B shock flags from V^n (workspace layout; one byte per cell at
// woff / NV): pass 1 marks FLAG_HLL where sum_d |p_{+1} - p_{-1}| /
// min(p_{+1}, p_{-1}) > eps_q and div v < 0 (central differences, FP64
// arithmetic on the stored values), on cells with both neighbours along
// every axis; pass 2 adds FLAG_MINMOD to every cell within the
// reconstruction radius of a FLAG_HLL cell along an axis.
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(NT) void k_shock_hll(const KBox *boxes, const KTile *tiles, const R *V,
                                                  unsigned char *flag, double eps, int dim)
{
    KTile tl = tiles[blockIdx.x];
    const KBox &bx = boxes[tl.box];
    const int c = tl.a + threadIdx.x;
    if (c >= bx.cells) return;
    const int i = c % bx.N[0], j = (c / bx.N[0]) % bx.N[1], k = c / (bx.N[0] * bx.N[1]);
    const int ci[3] = { i, j, k };
    const int cs = (int)bx.cells;
    const R *Vb = V + bx.woff;
    bool inside = true;
    for (int d = 0; d < dim; d++)
        if (ci[d] < 1 || ci[d] > bx.N[d] - 2) inside = false;
    unsigned char f = 0;
    if (inside) {
        double gradp = 0.0, divv = 0.0;
        for (int d = 0; d < dim; d++) {
            const int st = (d == 0) ? 1 : (d == 1 ? bx.N[0] : bx.N[0] * bx.N[1]);
            const double pp = (double)Vb[PRS * cs + c + st], pm = (double)Vb[PRS * cs + c - st];
            gradp += fabs(pp - pm) / fmin(pp, pm);
            divv += ((double)Vb[(MX1 + d) * cs + c + st] - (double)Vb[(MX1 + d) * cs + c - st]) / (2.0 * bx.dx[d]);
        }
        if (gradp > eps && divv < 0.0) f = FLAG_HLL;
    }
    flag[bx.woff / NV + c] = f;
}

template <int Z = 0>
__global__ __launch_bounds__(NT) void k_shock_mm(const KBox *boxes, const KTile *tiles, unsigned char *flag, int rad,
                                                 int dim)
{
    KTile tl = tiles[blockIdx.x];
    const KBox &bx = boxes[tl.box];
    const int c = tl.a + threadIdx.x;
    if (c >= bx.cells) return;
    const int i = c % bx.N[0], j = (c / bx.N[0]) % bx.N[1], k = c / (bx.N[0] * bx.N[1]);
    const int ci[3] = { i, j, k };
    unsigned char *fb = flag + bx.woff / NV;
    bool mm = false;
    for (int d = 0; d < dim && !mm; d++) {
        const int st = (d == 0) ? 1 : (d == 1 ? bx.N[0] : bx.N[0] * bx.N[1]);
        for (int s = -rad; s <= rad; s++) {
            const int e = ci[d] + s;
            if (e < 0 || e >= bx.N[d]) continue;
            if (fb[c + s * st] & FLAG_HLL) {
                mm = true;
                break;
            }
        }
    }
    if (mm) fb[c] |= FLAG_MINMOD;
}

// A vector store reads its data registers after issue, and the compiler
// waits for the store to complete before an instruction overwrites them.
// Values stored from short-lived temporaries make the next instructions that
// reuse those registers wait for the stores; keep(v) marks the registers of
// stored values as still in use at a later point (the next store of the same
// values), so that no other value takes them in between.
template <typename R> __device__ __forceinline__ void keep(const R &v) { asm volatile("" ::"v"(v)); }

// ---------------------------------------------------------------------------
// Parabolic face fluxes (Sec. 2.1.1, Sec. 3.1, App. A).
//
// Two kernels evaluate them from a primitive state.  On the D-face between
// cells A = c - e_D and B = c the face coefficients use the average of the
// states of A and B (the velocity density-weighted), gradients along D the
// two-point difference and the transverse gradients the four-point average
// of App. A.  The saturation of the conduction flux (Eq. tc_flux) is
// upwinded by the sign of the classical flux's normal component with the
// face's Riemann states:
//  * Pi^n (k_pdiv, from V^n): those states are the cells' own, so the kernel
//    saturates and differences the fluxes into the per-cell divergence that
//    the t^n kernel adds;
//  * Pi^{n+1/2} (k_pflux, from V^{n+1/2}): the states are the final face
//    states of the sweeps, so the classical flux is stored as its normal
//    component and magnitude in eight slots per face and the sweep
//    saturates (parab_face).
// A block owns TX x TY in-plane cells (3D: x, y; 2D: x) and marches along
// the last axis over a chunk of planes, with three planes of the eight
// staged fields (rho, v, B, T = p / rho) and a one-cell in-plane halo in LDS.
// ---------------------------------------------------------------------------

constexpr int NPF = 8;  // slots per face
constexpr int PF_M = 0;   // viscous momentum flux, three components
constexpr int PF_BT = 3;  // resistive flux of the transverse field B_t
constexpr int PF_BB = 4;  // ... and of the binormal field B_b
constexpr int PF_E = 5;   // viscous and resistive energy flux
constexpr int PF_FN = 6;  // classical conduction flux: normal component
constexpr int PF_FM = 7;  // ... and magnitude

template <int DIM> struct PTile {
    static constexpr int TX = (DIM == 3) ? 32 : NT;
    static constexpr int TY = (DIM == 3) ? 8 : 1;
    static constexpr int HX = TX + 2, HY = (DIM == 3) ? TY + 2 : 1, HP = HX * HY;
    // planes per block along the marching axis (measured at 256^3: k_pflux
    // 0.76 / 0.82 / 0.88 ms with 4 / 8 / 16, k_pdiv 0.77 / 0.73 / 0.73)
    static constexpr int LM_FLUX = 4, LM_DIV = 8;
};

template <typename R> struct PArgs {
    const KBox *boxes;
    const KTile *tiles;  // (box, x offset, y offset, marching offset) from g-1+s
    const R *V;          // primitive state (workspace)
    R *PF;               // face slots (workspace): NPF * DIM planes per cell
    KOpts o;
};

// the energy slot plus the conduction flux of normal component Fn and
// magnitude Fm, saturated (Eq. tc_flux) with the pressure upwinded by the
// sign of Fn (Eq. sat_flux)
template <typename R>
__device__ __forceinline__ R pf_energy(R E, R Fn, R Fm, const KOpts &o, R pL, R pR, R rL, R rR)
{
    if (o.parab & PB_TC) {
        if (o.phi > 0.0 && Fm > R(0)) {
            R pu = (Fn < R(0)) ? pL : pR;
            R q = R(5.0 * o.phi) * pu * sqrt(pu) / sqrt(R(0.5) * (rL + rR));
            Fn = q / (Fm + q) * Fn;
        }
        E += Fn;
    }
    return E;
}

// slots of the D-face below the lane's cell from the three staged planes
// (P[0], P[1], P[2] = planes m-1, m, m+1, field f at f * HP); l is the
// lane's in-plane slot
template <int DIM, int D, typename R>
__device__ __forceinline__ void pflux_face(const R *const *P, int l, const KBox &bx, const KOpts &o, R *out)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    constexpr int HP = PTile<DIM>::HP, HX = PTile<DIM>::HX;
    // plane and in-plane offsets of the unit step along axis e
    auto dm_of = [](int e) { return e == DIM - 1 ? 1 : 0; };
    auto dl_of = [](int e) { return e == DIM - 1 ? 0 : (e == 0 ? 1 : HX); };
    // field f of the cell at (dm, dl) from the lane's cell
    auto val = [&](int f, int dm, int dl) -> R { return P[1 + dm][f * HP + l + dl]; };
    const int aM = -dm_of(D), aL = -dl_of(D);  // cell A
    const R rA = val(0, aM, aL), rB = val(0, 0, 0);
    const R irs = R(1) / (rA + rB);
    const R rhof = R(0.5) * (rA + rB);
    R vf[3], Bf[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        vf[c] = (rA * val(1 + c, aM, aL) + rB * val(1 + c, 0, 0)) * irs;
        Bf[c] = R(0.5) * (val(4 + c, aM, aL) + val(4 + c, 0, 0));
    }
    // gradients of (v_x, v_y, v_z, B_x, B_y, B_z, T) at the face
    R g[7][3];
#pragma unroll
    for (int f = 0; f < 7; f++) {
        g[f][D] = (val(1 + f, 0, 0) - val(1 + f, aM, aL)) / R(bx.dx[D]);
#pragma unroll
        for (int e = 0; e < 3; e++) {
            if (e == D) continue;
            if (e >= DIM) {
                g[f][e] = R(0);
                continue;
            }
            const int em = dm_of(e), el = dl_of(e);
            R up = val(1 + f, em, el) + val(1 + f, aM + em, aL + el);
            R dn = val(1 + f, -em, -el) + val(1 + f, aM - em, aL - el);
            g[f][e] = (up - dn) / (R(4) * R(bx.dx[e]));
        }
    }
#pragma unroll
    for (int q = 0; q < NPF; q++) out[q] = R(0);
    if (o.parab & PB_VISC) {
        R divv = g[0][0] + g[1][1] + g[2][2];
        R mu = rhof * R(o.nu);
        R tau[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            tau[c] = mu * (g[c][n] + g[n][c] - (c == n ? R(2.0 / 3.0) * divv : R(0)));
            out[PF_M + c] = tau[c];
        }
        out[PF_E] += vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2];
    }
    if (o.parab & PB_RES) {
        R J[3];
        J[0] = g[5][1] - g[4][2];
        J[1] = g[3][2] - g[5][0];
        J[2] = g[4][0] - g[3][1];
        R eta = R(o.eta);
        out[PF_BT] = eta * J[b];
        out[PF_BB] = -(eta * J[t]);
        out[PF_E] -= eta * (J[t] * Bf[b] - J[b] * Bf[t]);
    }
    if (o.parab & PB_TC) {
        R B2 = Bf[0] * Bf[0] + Bf[1] * Bf[1] + Bf[2] * Bf[2];
        R bh[3] = { R(0), R(0), R(0) };
        if (B2 > R(0)) {
            R ib = R(1) / sqrt(B2);
#pragma unroll
            for (int c = 0; c < 3; c++) bh[c] = Bf[c] * ib;
        }
        R bg = bh[0] * g[6][0] + bh[1] * g[6][1] + bh[2] * g[6][2];
        R Fc[3];
#pragma unroll
        for (int c = 0; c < 3; c++) Fc[c] = R(o.kpar) * bh[c] * bg + R(o.kperp) * (g[6][c] - bh[c] * bg);
        out[PF_FN] = Fc[n];
        out[PF_FM] = sqrt(Fc[0] * Fc[0] + Fc[1] * Fc[1] + Fc[2] * Fc[2]);
    }
}

// stage plane m of V (rho, v, B, T = p / rho) over the tile's cells and a
// one-cell in-plane halo into S (field f at f * HP), cells of the load range
// [lo, hi] only
template <int DIM, typename R>
__device__ __forceinline__ void pf_stage(R *S, const R *Vb, const KBox &bx, const int *lo, const int *hi, int x0,
                                         int y0, int m)
{
    using PT = PTile<DIM>;
    constexpr int AM = DIM - 1;
    if (m < lo[AM] || m > hi[AM]) return;
    const int cs = (int)bx.cells;
    for (int h = threadIdx.x; h < PT::HP; h += NT) {
        const int hx = h % PT::HX, hy = h / PT::HX;
        const int xx = x0 - 1 + hx, yy = y0 - 1 + hy;
        if (xx < lo[0] || xx > hi[0]) continue;
        if (DIM == 3 && (yy < lo[1] || yy > hi[1])) continue;
        const int c = (DIM == 3) ? cidx(bx, xx, yy, m) : cidx(bx, xx, m, 0);
        const R rho = Vb[RHO * cs + c];
        R *d = S + h;
        d[0] = rho;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            d[(1 + q) * PT::HP] = Vb[(MX1 + q) * cs + c];
            d[(4 + q) * PT::HP] = Vb[(BX1 + q) * cs + c];
        }
        d[7 * PT::HP] = Vb[PRS * cs + c] / rho;
    }
}

// Pi^{n+1/2} face slots of the sweeps (all eight, conduction unsaturated):
// faces below cells g .. g+n along D at positions g .. g+n-1 across it,
// reading cells g-1 .. g+n, where V^{n+1/2} is defined
template <int DIM, typename R>
__global__ __launch_bounds__(NT) void k_pflux(PArgs<R> a)
{
    using PT = PTile<DIM>;
    constexpr int AM = DIM - 1;  // marching axis
    __shared__ R S[3][8 * PT::HP];
    const int tid = threadIdx.x;
    const KTile tl = a.tiles[blockIdx.x];
    const KBox bx = a.boxes[tl.box];
    const KOpts &o = a.o;
    const int cs = (int)bx.cells;
    const R *Vb = a.V + bx.woff;
    R *Pb = a.PF + (bx.woff / NV) * (NPF * DIM);
    // load range [lo, hi] per axis (x, y, marching in 3D; x, marching in 2D)
    int lo[3] = { 0, 0, 0 }, hi[3] = { 0, 0, 0 };
#pragma unroll
    for (int e = 0; e < DIM; e++) {
        lo[e] = bx.g[e] - 1;
        hi[e] = bx.g[e] + bx.n[e];
    }
    const int x0 = lo[0] + 1 + tl.a, y0 = (DIM == 3) ? lo[1] + 1 + tl.b : 0;
    const int tx = tid % PT::TX, ty = tid / PT::TX;
    const int x = x0 + tx, y = y0 + ty;
    const int l = (DIM == 3) ? (ty + 1) * PT::HX + tx + 1 : tx + 1;
    // the faces of this lane's position (per plane, the marching bounds below)
    const bool inx = x <= hi[0] - 1, iny = DIM == 2 || y <= hi[1] - 1;
    const bool fx = x <= hi[0] && iny;
    const bool fy = DIM == 3 && inx && y <= hi[1];
    const bool fm = inx && iny;
    const int m0 = lo[AM] + 1 + tl.c, m1 = min(m0 + PT::LM_FLUX - 1, hi[AM]);

    int r0 = 0, r1 = 1, r2 = 2;  // ring slots of planes m-1, m, m+1
    pf_stage<DIM>(&S[r0][0], Vb, bx, lo, hi, x0, y0, m0 - 1);
    pf_stage<DIM>(&S[r1][0], Vb, bx, lo, hi, x0, y0, m0);
    for (int m = m0; m <= m1; m++) {
        pf_stage<DIM>(&S[r2][0], Vb, bx, lo, hi, x0, y0, m + 1);
        __syncthreads();
        const R *P[3] = { &S[r0][0], &S[r1][0], &S[r2][0] };
        const int c = (DIM == 3) ? cidx(bx, x, y, m) : cidx(bx, x, m, 0);
        R out[NPF];
        const bool inm = m <= hi[AM] - 1;  // the in-plane faces' marching bound
        auto face = [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            pflux_face<DIM, D>(P, l, bx, o, out);
            R *dst = Pb + D * NPF * cs + c;
#pragma unroll
            for (int q = 0; q < NPF; q++) dst[q * cs] = out[q];
        };
        if (fx && inm) face(std::integral_constant<int, 0>());
        if constexpr (DIM == 3)
            if (fy && inm) face(std::integral_constant<int, 1>());
        if (fm) face(std::integral_constant<int, AM>());
        __syncthreads();
        const int rt = r0;
        r0 = r1;
        r1 = r2;
        r2 = rt;
    }
}

// (Pi_{D,+} - Pi_{D,-}) * idx of the saturated slots Fl (face below) and Fh
// (face above), added into the nine-component P
template <int D, typename R> __device__ __forceinline__ void pdiv_add(const R *Fl, const R *Fh, R idx, R *P)
{
    constexpr int t = Ax<D>::t, b = Ax<D>::b;
#pragma unroll
    for (int q = 0; q < 3; q++) P[MX1 + q] += (Fh[PF_M + q] - Fl[PF_M + q]) * idx;
    P[BX1 + t] += (Fh[PF_BT] - Fl[PF_BT]) * idx;
    P[BX1 + b] += (Fh[PF_BB] - Fl[PF_BB]) * idx;
    P[ENG] += (Fh[PF_E] - Fl[PF_E]) * idx;
}

// k_pdiv: the divergence P = sum_d (Pi_{d,+} - Pi_{d,-}) / dx_d of Pi^n on
// the cells of the t^n region [g-1, g+n], the conduction flux saturated with
// the two cells' own states (the t^n Riemann inputs).  Stored per cell as the
// seven components MX1 .. BX3 (planes 0 .. 6 of the box's face slots).
// The tiles overlap by one column (and row): every lane solves the low faces
// of its cell and the lanes of all but the last column (and row) difference
// them with their neighbours' (3D: x from the next lane of the wave by a
// cross-lane shuffle, y through LDS; 2D: x through LDS); the marching faces
// are carried from plane to plane, so each cell is finished one plane later.
template <int DIM, typename R>
__global__ __launch_bounds__(NT) void k_pdiv(PArgs<R> a)
{
    using PT = PTile<DIM>;
    constexpr int AM = DIM - 1;
    constexpr int NS = PF_E + 1;  // saturated slots
    static_assert(DIM == 2 || (PT::TX <= 64 && 64 % PT::TX == 0), "a tile row must lie within one wave");
    __shared__ R S[3][8 * PT::HP];
    __shared__ R Fy[(DIM == 3) ? NS : 1][(DIM == 3) ? NT : 1];
    __shared__ R Fx2[(DIM == 2) ? NS : 1][(DIM == 2) ? NT : 1];
    const int tid = threadIdx.x;
    const KTile tl = a.tiles[blockIdx.x];
    const KBox bx = a.boxes[tl.box];
    const KOpts &o = a.o;
    const int cs = (int)bx.cells;
    const R *Vb = a.V + bx.woff;
    R *Pb = a.PF + (bx.woff / NV) * (NPF * DIM);
    int lo[3] = { 0, 0, 0 }, hi[3] = { 0, 0, 0 };
#pragma unroll
    for (int e = 0; e < DIM; e++) {
        lo[e] = bx.g[e] - 2;
        hi[e] = bx.g[e] + bx.n[e] + 1;
    }
    const int x0 = lo[0] + 1 + tl.a, y0 = (DIM == 3) ? lo[1] + 1 + tl.b : 0;
    const int tx = tid % PT::TX, ty = tid / PT::TX;
    const int x = x0 + tx, y = y0 + ty;
    const int l = (DIM == 3) ? (ty + 1) * PT::HX + tx + 1 : tx + 1;
    const bool iny = DIM == 2 || y <= hi[1] - 1;
    const bool fx = x <= hi[0] && iny;
    const bool fy = DIM == 3 && x <= hi[0] - 1 && y <= hi[1];
    const bool fm = x <= hi[0] - 1 && iny;
    const bool own = fm && tx < PT::TX - 1 && (DIM == 2 || ty < PT::TY - 1);
    const int m0 = lo[AM] + 1 + tl.c, m1 = min(m0 + PT::LM_DIV - 1, hi[AM] - 1);
    const int sM = (DIM == 3) ? bx.N[0] * bx.N[1] : bx.N[0];
    const R ix = R(1.0 / bx.dx[0]), iy = R(1.0 / bx.dx[1]), iz = R(1.0 / bx.dx[2]);

    int r0 = 0, r1 = 1, r2 = 2;  // ring slots of planes m-1, m, m+1
    pf_stage<DIM>(&S[r0][0], Vb, bx, lo, hi, x0, y0, m0 - 1);
    pf_stage<DIM>(&S[r1][0], Vb, bx, lo, hi, x0, y0, m0);
    R Fm_prev[NS], Pin[NV], Fx[NS];
#pragma unroll
    for (int q = 0; q < NS; q++) Fx[q] = R(0);
    for (int m = m0; m <= m1 + 1; m++) {
        pf_stage<DIM>(&S[r2][0], Vb, bx, lo, hi, x0, y0, m + 1);
        __syncthreads();
        const R *P[3] = { &S[r0][0], &S[r1][0], &S[r2][0] };
        const int c = (DIM == 3) ? cidx(bx, x, y, m) : cidx(bx, x, m, 0);
        R out[NPF];
        // the D-face below the lane's cell, saturated with the states of its
        // two cells
        auto face = [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            pflux_face<DIM, D>(P, l, bx, o, out);
            const int sD = (D == 0) ? 1 : (D == 1 ? bx.N[0] : bx.N[0] * bx.N[1]);
            const R rA = P[(D == AM) ? 0 : 1][l - ((D == AM) ? 0 : (D == 0 ? 1 : PT::HX))];
            const R rB = P[1][l];
            out[PF_E] = pf_energy(out[PF_E], out[PF_FN], out[PF_FM], o, Vb[PRS * cs + c - sD], Vb[PRS * cs + c], rA, rB);
        };
        if (m <= m1) {
            if (fx) {
                face(std::integral_constant<int, 0>());
#pragma unroll
                for (int q = 0; q < NS; q++) {
                    Fx[q] = out[q];
                    if constexpr (DIM == 2) Fx2[q][tid] = out[q];
                }
            }
            if constexpr (DIM == 3) {
                if (fy) {
                    face(std::integral_constant<int, 1>());
#pragma unroll
                    for (int q = 0; q < NS; q++) Fy[q][tid] = out[q];
                }
            }
        }
        R Fm[NS];
        if (fm) {
            face(std::integral_constant<int, AM>());
#pragma unroll
            for (int q = 0; q < NS; q++) Fm[q] = out[q];
        }
        // 3D: the x-face above the lane's cell is the next lane's (same row,
        // same wave for the lanes that use it)
        R Fxh[NS];
        if constexpr (DIM == 3) {
#pragma unroll
            for (int q = 0; q < NS; q++) Fxh[q] = __shfl_down(Fx[q], 1);
        }
        __syncthreads();
        if (own) {
            // finish cell (x, y, m-1): its high marching face is Fm
            if (m > m0) {
                R Pc[NV];
#pragma unroll
                for (int q = 0; q < NV; q++) Pc[q] = Pin[q];
                pdiv_add<AM>(Fm_prev, Fm, (DIM == 3) ? iz : iy, Pc);
#pragma unroll
                for (int q = 0; q < 7; q++) Pb[q * cs + c - sM] = Pc[MX1 + q];
            }
            // in-plane part of this plane's cell
            if (m <= m1) {
#pragma unroll
                for (int q = 0; q < NV; q++) Pin[q] = R(0);
                if constexpr (DIM == 2) {
#pragma unroll
                    for (int q = 0; q < NS; q++) Fxh[q] = Fx2[q][tid + 1];
                }
                pdiv_add<0>(Fx, Fxh, ix, Pin);
                if constexpr (DIM == 3) {
                    R Fl[NS], Fh[NS];
#pragma unroll
                    for (int q = 0; q < NS; q++) {
                        Fl[q] = Fy[q][tid];
                        Fh[q] = Fy[q][tid + PT::TX];
                    }
                    pdiv_add<1>(Fl, Fh, iy, Pin);
                }
            }
#pragma unroll
            for (int q = 0; q < NS; q++) Fm_prev[q] = Fm[q];
        }
        const int rt = r0;
        r0 = r1;
        r1 = r2;
        r2 = rt;
    }
}

// Pi on the D-face below cell c from its slots (Pf: the box's slots), the
// saturated conduction flux upwinded with the face states (pL, rL), (pR, rR)
template <int D, typename R>
__device__ __forceinline__ void parab_face(const R *Pf, int cs, int c, const KOpts &o, R pL, R pR, R rL, R rR, R *Pi)
{
    constexpr int t = Ax<D>::t, b = Ax<D>::b;
    const R *f = Pf + D * NPF * cs + c;
#pragma unroll
    for (int q = 0; q < NV; q++) Pi[q] = R(0);
#pragma unroll
    for (int q = 0; q < 3; q++) Pi[MX1 + q] = f[(PF_M + q) * cs];
    Pi[BX1 + t] = f[PF_BT * cs];
    Pi[BX1 + b] = f[PF_BB * cs];
    const bool tc = (o.parab & PB_TC) != 0;
    Pi[ENG] = pf_energy(f[PF_E * cs], tc ? f[PF_FN * cs] : R(0), tc ? f[PF_FM * cs] : R(0), o, pL, pR, rL, rR);
}


// x^y for x > 0: in FP32 as 2^(y log2 x) with the hardware log2 and exp2
// (the FP32 path's approximate-transcendental convention), in FP64 pow
template <typename R> __device__ __forceinline__ R powp(R x, R y)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
    else return pow(x, y);
}

template <typename R> __device__ __forceinline__ R diff_coeff(const KOpts &o, R rho, R gam)
{
    R D = R(0);
    if (o.parab & PB_VISC) D = fmax(D, R(o.nu));
    if (o.parab & PB_RES) D = fmax(D, R(o.eta));
    if (o.parab & PB_TC) D = fmax(D, (gam - R(1)) * R(fmax(o.kpar, o.kperp)) / rho);
    return D;
}

// ---------------------------------------------------------------------------
// k_tcouple: the t^n part of the step in one marching kernel.
//
// A block owns 256 in-plane positions of the region [g-1, g+n] (x, y in 3D;
// x in 2D) and marches along the last axis over a chunk of its planes.  For
// each plane it solves the first-order Riemann problems R(V_j, V_{j+1}) on
// the low faces of its positions plus the faces above its last ones, hands
// them over through LDS, and forms per cell the increments
// L_d = -(F_{d,+} - F_{d,-})/dx_d.  The marching-axis faces of one plane are
// the high faces of the previous one, so each cell is finished one plane
// later.  With parabolic terms the cell also takes the divergence
// P = sum_d (Pi_{d,+} - Pi_{d,-})/dx_d of the Pi^n face slots.  Outputs,
// per cell:
//   T_d = sum_{d' != d} L_{d'} + P   (the Eq. transv increment of sweep d:
//                                     sum_{d' != d} (L_{d'} + Lp_{d'}) + Lp_d)
//   V^{n+1/2} = V(U^n + dt/2 (sum_d L_d + P))   (parabolic runs only)
//
// Two in-plane layouts, chosen per tile on the host:
//  * tile (b >= 0): a TX x TY rectangle at (a, b); the TY faces right of it
//    and the TX faces above it are the extra faces;
//  * strip (3D, b <= -2): the last SW = W - a <= 2 positions of rows
//    -2 - b .. -2 - b + SH - 1 (a 258-position row is eight rectangles and
//    one strip instead of a ninth rectangle with 2 of its 32 columns
//    active); its extra faces are solved by the two waves that hold no
//    position;
//  * flat (3D, b == -1): positions a .. a+255 of the extended plane of
//    (W+1) x (H+1) positions, W x H the region's extent, row by row; a
//    position with x = W or y = H only solves the face below it.  The extra
//    faces are the x face below position a+256 and the y faces below a+256 ..
//    a+256+W, so W + 2 <= 64 is required (and W + 1 <= MAXW1 for the LDS
//    slots).  On the 16-32 cell patches of an
//    AMR level this uses ~78 % of the lanes against ~61 % for 32 x 8 tiles.
// ---------------------------------------------------------------------------

template <int DIM> struct TTile {
    static constexpr int TX = (DIM == 3) ? 32 : NT;
    static constexpr int TY = (DIM == 3) ? 8 : 1;
    static constexpr int LM = 16;   // default planes per block along the marching axis
    // strip tiles (3D): the last SW <= 2 positions of each row of the region
    // when its width leaves that many beyond the TX-wide rectangles, SH rows
    // per block (positions on the first two waves, the strip's extra faces
    // on the other two)
    static constexpr int SWMAX = 2;
    static constexpr int SH = 64;
    // flat layout: at most 40 positions per row (boxes up to 37 cells wide),
    // which keeps the face planes of four FP64 blocks within 160 KiB of LDS
    static constexpr int MAXW1 = 40;
    // LDS face slots: the larger of the two layouts (flat: 256 + 1 and
    // 256 + MAXW1 + 1)
    static constexpr int GXS = (DIM == 3) ? ((TY * (TX + 1) > 257) ? TY * (TX + 1) : 257) : TY * (TX + 1);
    static constexpr int GYS = (DIM == 3) ? (((TY + 1) * TX > 256 + MAXW1 + 1) ? (TY + 1) * TX : 256 + MAXW1 + 1) : 1;
    static_assert(DIM == 2 || (SH * (SWMAX + 1) <= GXS && (SH + 1) * SWMAX <= GYS), "strip face slots exceed LDS");
    static_assert(SWMAX * SH <= 2 * 64 && SH + SWMAX <= NT - 2 * 64, "strip positions / extra faces exceed their waves");
};

template <typename R> struct TArgs {
    const KBox *boxes;
    const KTile *tiles;
    const R *U;       // U^n (caller layout)
    const R *V;       // V^n (workspace)
    R *T[3];          // transverse increments (workspace)
    R *Vh;            // V^{n+1/2} (workspace) or null
    const R *PF;      // divergence of Pi^n per cell, 7 planes (workspace) or null
    const unsigned char *flag;  // App. B zone flags (workspace) or null
    const double *params;
    KOpts o;
    int lm;           // planes per chunk along the marching axis (>= 1)
};

// the nine primitive variables of cell c
template <typename R> __device__ __forceinline__ void ld_cell(const Blk<R> &bV, int c, R *V)
{
#pragma unroll
    for (int q = 0; q < NV; q++) V[q] = bV.ld(q, c);
}

// one face: the first-order flux G = F on the D-face below cell (i,j,k),
// from states already in registers: VL of the cell below the face, VR of
// cell (i,j,k).  Both are copied (the solver overwrites B_n) through an
// empty register barrier: a cell's state is shared by its three faces, and
// without the barrier the compiler would share and contract their
// arithmetic differently from a face solved alone, so the same face would
// round differently under another launch shape
template <int D, int PHYS, int RS, int SHK, typename R>
__device__ __forceinline__ void tface_s(const R *VL_in, const R *VR_in, const KBox &bx, int i, int j, int k,
                                        const KOpts &o, R gam, R ch, R *G, const unsigned char *fb)
{
    bool hl = false;
    if constexpr (SHK) {
        int di, dj, dk;
        unit<D>(di, dj, dk);
        hl = ((fb[cidx(bx, i - di, j - dj, k - dk)] | fb[cidx(bx, i, j, k)]) & FLAG_HLL) != 0;
    }
    R VL[NV], VR[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        VL[q] = VL_in[q];
        VR[q] = VR_in[q];
        asm volatile("" : "+v"(VL[q]));
        asm volatile("" : "+v"(VR[q]));
    }
    if (!o.hyp_off) {
        R sm;
        if (SHK && hl) riemann<D, PHYS, RS_HLL>(VL, VR, G, sm, gam, ch, o.glm, o.xspeeds);
        else riemann<D, PHYS, RS>(VL, VR, G, sm, gam, ch, o.glm, o.xspeeds);
    } else {
#pragma unroll
        for (int q = 0; q < NV; q++) G[q] = R(0);
    }
}

#ifndef CTU_TC_WAVES_PAR_F32
#define CTU_TC_WAVES_PAR_F32 1
#endif
// the FP64 parabolic kernel at two waves (12 bytes of spills, without the
// U^n / P prefetch) runs 15 % faster than at one wave with it
#ifndef CTU_TC_WAVES_PAR_F64
#define CTU_TC_WAVES_PAR_F64 2
#endif
template <int PAR, typename R> constexpr int tc_waves()
{
    return PAR ? (sizeof(R) == 4 ? CTU_TC_WAVES_PAR_F32 : CTU_TC_WAVES_PAR_F64) : 1;
}

template <int DIM, int PHYS, int RS, int PAR, int VAR, typename R>
__global__ __launch_bounds__(NT, (tc_waves<PAR, R>())) void k_tcouple(TArgs<R> a)
{
    constexpr int SHK = (VAR == VAR_SHOCK);
    constexpr int TX = TTile<DIM>::TX, TY = TTile<DIM>::TY;
    constexpr int GXS = TTile<DIM>::GXS, GYS = TTile<DIM>::GYS;
    constexpr int AM = DIM - 1;                 // marching axis
    __shared__ R Gx[NV][GXS];
    __shared__ R Gy[(DIM == 3) ? NV : 1][GYS];

    const int tid = threadIdx.x;
    // lane in the wave that solves the extra faces; consecutive blocks go to
    // the eight XCDs in turn, so the choice mixes in the block's place within
    // its XCD, and over the blocks resident on a compute unit the extra
    // solves spread over its four SIMDs
    const int et = tid - 64 * (int)((blockIdx.x ^ (blockIdx.x >> 3)) & (NT / 64 - 1));
    const KTile tl = a.tiles[blockIdx.x];
    const KBox bx = a.boxes[tl.box];
    const KOpts o = variant_opts<VAR>(a.o);
    const R gam = R(o.gamma), ch = R(a.params[1]);
    const R hdt = R(0.5 * box_dt(bx, a.params));
    const int cs = (int)bx.cells;
    const R *Vb = a.V + bx.woff;
    const R *Pf = PAR ? a.PF + (bx.woff / NV) * (NPF * DIM) : nullptr;
    const Blk<R> bV(Vb, bx.cells);
    const unsigned char *fb = SHK ? a.flag + bx.woff / NV : nullptr;
    const Blk<R> bT0(a.T[0] + bx.woff, bx.cells), bT1(a.T[1] + bx.woff, bx.cells), bT2(DIM == 3 ? a.T[2] + bx.woff : Vb, bx.cells);
    const R ix = R(1.0 / bx.dx[0]), iy = R(1.0 / bx.dx[1]), iz = R(1.0 / bx.dx[2]);
    const int hi0 = bx.g[0] + bx.n[0];                       // last region cell along x
    const int hi1 = (DIM == 3) ? bx.g[1] + bx.n[1] : 0;

    // this lane's in-plane position (ghosted coordinates), the faces it
    // solves, whether it finishes a cell, and its LDS slots: the x / y face
    // below it sits at lx / ly, the faces above it at lx + 1 / ly + sy
    int i, j, lx, ly, sy;
    bool xf, yf, inplane;
    // the extra face of this lane (if any): below position (ei, ej), along
    // x (ed = 0) or y (ed = 1), into slot es
    int ei = 0, ej = 0, ed = -1, es = 0;
    if (DIM == 3 && tl.b == -1) {
        const int W1 = bx.n[0] + 3, H1 = bx.n[1] + 3, P = W1 * H1;
        const int p = tl.a + tid, x = p % W1, y = p / W1;
        i = bx.g[0] - 1 + x;
        j = bx.g[1] - 1 + y;
        xf = p < P && y < H1 - 1;
        yf = p < P && x < W1 - 1;
        inplane = xf && yf;
        lx = ly = tid;
        sy = W1;
        if (et >= 0 && et <= W1) {
            const int q = tl.a + NT + (et < W1 ? et : 0), qx = q % W1, qy = q / W1;
            ei = bx.g[0] - 1 + qx;
            ej = bx.g[1] - 1 + qy;
            if (et < W1) {
                if (q < P && qx < W1 - 1) ed = 1;
                es = NT + et;
            } else {
                if (q < P && qy < H1 - 1) ed = 0;
                es = NT;
            }
        }
    } else {
        // rectangle (tw x th = TX x TY) or strip (tw = W - a, th = SH)
        const bool strip = DIM == 3 && tl.b <= -2;
        const int tw = strip ? bx.n[0] + 2 - tl.a : TX, th = strip ? TTile<DIM>::SH : TY;
        const int y0 = strip ? -2 - tl.b : tl.b;
        const int e = strip ? tid - 2 * 64 : et;
        const bool pos = !strip || tid < tw * th;
        const int tx = tid % tw, ty = tid / tw;
        i = bx.g[0] - 1 + tl.a + tx;
        j = (DIM == 3) ? bx.g[1] - 1 + y0 + ty : 0;
        xf = pos && (i <= hi0 + 1) && (DIM == 2 || j <= hi1);
        yf = pos && (DIM == 3) && (i <= hi0) && (j <= hi1 + 1);
        inplane = pos && (i <= hi0) && (DIM == 2 || j <= hi1);
        lx = ty * (tw + 1) + tx;
        ly = ty * tw + tx;
        sy = tw;
        if (e >= 0 && e < th) {
            ei = bx.g[0] - 1 + tl.a + tw;
            ej = (DIM == 3) ? bx.g[1] - 1 + y0 + e : 0;
            if (ei <= hi0 + 1 && (DIM == 2 || ej <= hi1)) ed = 0;
            es = e * (tw + 1) + tw;
        } else if (DIM == 3 && e >= th && e < th + tw) {
            ei = bx.g[0] - 1 + tl.a + (e - th);
            ej = bx.g[1] - 1 + y0 + th;
            if (ei <= hi0 && ej <= hi1 + 1) ed = 1;
            es = th * tw + (e - th);
        }
    }
    // this block's chunk of the region [g-1, g+n] along the marching axis;
    // its first marching faces are recomputed, not shared with the chunk below
    const int m0 = bx.g[AM] - 1 + tl.c;
    const int m1 = min(m0 + a.lm - 1, bx.g[AM] + bx.n[AM]);

    // the lane's cell state on this plane (the right state of its three
    // faces) and on the previous one (the left state of the marching face),
    // loaded once and carried from plane to plane
    R Vc[NV], Vp[NV];
    if (inplane) ld_cell(bV, cidx(bx, i, (DIM == 3) ? j : m0 - 1, (DIM == 3) ? m0 - 1 : 0), Vp);
    R Gm_prev[NV], Lx_prev[NV], Ly_prev[NV];
    // the stored T_d and V^{n+1/2} values of the last finished cell, held
    // until the next cell's stores (see keep): FP32 parabolic runs, whose
    // two waves per SIMD leave the registers (6 % faster there; in the
    // three-wave kernels the extra registers cost a wave)
    constexpr bool KEEPT = PAR && sizeof(R) == 4;
    // FP32 parabolic runs load U^n and P of the cell to finish ahead of the
    // plane's face solves; FP64 loads them where they are used (the held
    // registers would cost its second wave per SIMD)
    constexpr bool PRE = PAR && sizeof(R) == 4;
    constexpr int NKT = KEEPT ? (DIM + (PAR ? 1 : 0)) * NV : 1;
    R Tk[NKT];
#pragma unroll
    for (int q = 0; q < NKT; q++) Tk[q] = R(0);
    for (int m = m0; m <= m1 + 1; m++) {
        const int cj = (DIM == 3) ? j : m, ck = (DIM == 3) ? m : 0;
        // U^n and P of the cell this plane finishes, loaded ahead of the face
        // solves that hide their latency (PRE)
        R Upre[NV], Ppre[7];
        if constexpr (PRE) {
            if (inplane && m > m0) {
                const int pc = cidx(bx, i, (DIM == 3) ? j : m - 1, (DIM == 3) ? m - 1 : 0);
#pragma unroll
                for (int q = 0; q < NV; q++) Upre[q] = Blk<R>(a.U + bx.uoff, bx.cells).ld(q, pc);
#pragma unroll
                for (int q = 0; q < 7; q++) Ppre[q] = Pf[q * cs + pc];
            }
        }
        // in FP32 every state this plane's faces read is loaded together, so
        // that one wait covers the three loads; in FP64 the two neighbour
        // states are loaded at their faces (held across the marching face
        // they would take the registers of the second wave per SIMD)
        constexpr bool GROUP = sizeof(R) == 4;
        constexpr bool GROUP_E = GROUP && !SHK && RS != RS_ROE;
        R VLx[NV], VLy[NV], VLe[NV], VRe[NV];
        if (inplane || (m <= m1 && (xf || yf))) ld_cell(bV, cidx(bx, i, cj, ck), Vc);
        if constexpr (GROUP) {
            if (m <= m1 && xf) ld_cell(bV, cidx(bx, i - 1, cj, ck), VLx);
            if constexpr (DIM == 3)
                if (m <= m1 && yf) ld_cell(bV, cidx(bx, i, j - 1, ck), VLy);
            // and the two states of the lane's extra face, where the registers
            // they take keep three waves per SIMD (not with shock flags or the
            // Roe solver)
            if constexpr (GROUP_E) {
                if (m <= m1 && ed == 0) {
                    const int ej2 = (DIM == 3) ? ej : m;
                    ld_cell(bV, cidx(bx, ei - 1, ej2, ck), VLe);
                    ld_cell(bV, cidx(bx, ei, ej2, ck), VRe);
                } else if (DIM == 3 && m <= m1 && ed == 1) {
                    ld_cell(bV, cidx(bx, ei, ej - 1, m), VLe);
                    ld_cell(bV, cidx(bx, ei, ej, m), VRe);
                }
            }
        }
        // ---- faces of this plane: the marching face below each region cell,
        // and the in-plane low faces of every position whose face borders the
        // region ----
        R Gm[NV];
        if (inplane) tface_s<AM, PHYS, RS, SHK>(Vp, Vc, bx, i, cj, ck, o, gam, ch, Gm, fb);
        if (m <= m1) {
            R G[NV];
            if (xf) {
                if constexpr (!GROUP) ld_cell(bV, cidx(bx, i - 1, cj, ck), VLx);
                tface_s<0, PHYS, RS, SHK>(VLx, Vc, bx, i, cj, ck, o, gam, ch, G, fb);
#pragma unroll
                for (int q = 0; q < NV; q++) Gx[q][lx] = G[q];
            }
            if constexpr (DIM == 3) {
                if (yf) {
                    if constexpr (!GROUP) ld_cell(bV, cidx(bx, i, j - 1, ck), VLy);
                    tface_s<1, PHYS, RS, SHK>(VLy, Vc, bx, i, cj, ck, o, gam, ch, G, fb);
#pragma unroll
                    for (int q = 0; q < NV; q++) Gy[q][ly] = G[q];
                }
            }
            // the extra faces
            if (ed == 0) {
                const int ej2 = (DIM == 3) ? ej : m;
                if constexpr (!GROUP_E) {
                    ld_cell(bV, cidx(bx, ei - 1, ej2, ck), VLe);
                    ld_cell(bV, cidx(bx, ei, ej2, ck), VRe);
                }
                tface_s<0, PHYS, RS, SHK>(VLe, VRe, bx, ei, ej2, ck, o, gam, ch, G, fb);
#pragma unroll
                for (int q = 0; q < NV; q++) Gx[q][es] = G[q];
            } else if (DIM == 3 && ed == 1) {
                if constexpr (!GROUP_E) {
                    ld_cell(bV, cidx(bx, ei, ej - 1, m), VLe);
                    ld_cell(bV, cidx(bx, ei, ej, m), VRe);
                }
                tface_s<(DIM == 3 ? 1 : 0), PHYS, RS, SHK>(VLe, VRe, bx, ei, ej, m, o, gam, ch, G, fb);
#pragma unroll
                for (int q = 0; q < NV; q++) Gy[q][es] = G[q];
            }
        }
        __syncthreads();
        if (inplane) {
            // ---- finish the previous plane (its high marching face is Gm) ----
            if (m > m0) {
                const int pj = (DIM == 3) ? j : m - 1, pk = (DIM == 3) ? m - 1 : 0;
                const int c = cidx(bx, i, pj, pk);
                const R im = (DIM == 3) ? iz : iy;
                // parabolic runs: the divergence P of Pi^n (k_pdiv), which
                // enters every T_d and the half step in full (Eq. transv: the
                // bracket's sum over d' != d of L_H plus the sum of L_P over
                // all d)
                R Pd[NV];
                if constexpr (PAR) {
                    Pd[RHO] = R(0);
                    Pd[PSI] = R(0);
#pragma unroll
                    for (int q = 0; q < 7; q++) Pd[MX1 + q] = PRE ? Ppre[q] : Pf[q * cs + c];
                }
                auto addp = [&](R x, int q) -> R {
                    if constexpr (PAR) return x + Pd[q];
                    else return x;
                };
                if constexpr (KEEPT) {
#pragma unroll
                    for (int q = 0; q < NKT; q++) keep(Tk[q]);
                }
                R Lm[NV], S[NV];
#pragma unroll
                for (int q = 0; q < NV; q++) {
                    Lm[q] = -(Gm[q] - Gm_prev[q]) * im;
                    R t0, t1, t2 = R(0);
                    if constexpr (DIM == 3) {
                        t0 = addp(Ly_prev[q] + Lm[q], q);
                        t1 = addp(Lx_prev[q] + Lm[q], q);
                        t2 = addp(Lx_prev[q] + Ly_prev[q], q);
                        S[q] = addp(Lx_prev[q] + Ly_prev[q] + Lm[q], q);
                    } else {
                        t0 = addp(Lm[q], q);
                        t1 = addp(Lx_prev[q], q);
                        S[q] = addp(Lx_prev[q] + Lm[q], q);
                    }
                    if constexpr (KEEPT) {
                        Tk[q] = t0;
                        Tk[NV + q] = t1;
                        if constexpr (DIM == 3) Tk[2 * NV + q] = t2;
                    }
                    bT0.st(q, c, t0);
                    bT1.st(q, c, t1);
                    if constexpr (DIM == 3) bT2.st(q, c, t2);
                }
                if constexpr (PAR) {
                    R u[NV], v[NV];
#pragma unroll
                    for (int q = 0; q < NV; q++) u[q] = (PRE ? Upre[q] : Blk<R>(a.U + bx.uoff, bx.cells).ld(q, c)) + hdt * S[q];
                    c2p<PHYS_MHD>(u, v, gam);
#pragma unroll
                    for (int q = 0; q < NV; q++) {
                        if constexpr (KEEPT) Tk[DIM * NV + q] = v[q];
                        Blk<R>(a.Vh + bx.woff, bx.cells).st(q, c, v[q]);
                    }
                }
            }
            // ---- in-plane increments of this plane, kept for one plane ----
            if (m <= m1) {
#pragma unroll
                for (int q = 0; q < NV; q++) {
                    Lx_prev[q] = -(Gx[q][lx + 1] - Gx[q][lx]) * ix;
                    if constexpr (DIM == 3) Ly_prev[q] = -(Gy[q][ly + sy] - Gy[q][ly]) * iy;
                }
            }
#pragma unroll
            for (int q = 0; q < NV; q++) {
                Gm_prev[q] = Gm[q];
                Vp[q] = Vc[q];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// MT corner coupling (runs without parabolic terms): the transverse fluxes of
// Eq. transv are Riemann fluxes between the normal-predictor states of the
// two cells of a face instead of first-order t^n fluxes.
//   k_mtflux<D>  the Riemann fluxes of the D-faces g..g+n at transverse
//                positions g-1..g+n between the normal-predictor states (the
//                sweep's own predictor) of their two cells, stored on the
//                face below each cell; MT tiles of 4 x 64 cells;
//   k_mtT        T_d = sum_{e != d} -(F_e(c + e) - F_e(c)) / dx_e on the cells
//                the sweep of d reads (d-layer g-1..g+n, interior across d).
// ---------------------------------------------------------------------------

template <typename R> struct MtArgs {
    const KBox *boxes;
    const KTile *tiles;   // k_mtflux: MT tiles of its direction; k_mtT: cell tiles
    const R *U;           // U^n (caller layout)
    const R *V;           // V^n (workspace)
    R *F[3];              // predictor fluxes per direction (workspace)
    R *T[3];              // transverse increments (workspace)
    const double *params;
    KOpts o;
};

// normal predictor (the sweep's) of the cell at c along D
template <int D, int PHYS, int PRED, int RK, typename R>
__device__ __forceinline__ void mt_predict(const Blk<R> &bV, const R *Ub, const KBox &bx, int c, int sD,
                                           const KOpts &o, R gam, R dtdx, R dxD, R ch, R *Vm, R *Vp)
{
    R Vs[5][NV];
    constexpr int l0 = (RK == RK_PPM) ? 0 : 1, l1 = (RK == RK_PPM) ? 5 : 4;
#pragma unroll
    for (int l = l0; l < l1; l++) ld_cell(bV, c + (l - 2) * sD, Vs[l]);
    if constexpr (PRED == PRED_CHAR) {
        predict_char<D, RK>(Vs, o, gam, dtdx, dxD, ch, Vm, Vp, o.limiter);
    } else {
        R U0[NV];
        ld_cell(Blk<R>(Ub + bx.uoff, bx.cells), c, U0);
        (void)predict_mh<D, PHYS>(Vs, U0, o, gam, dtdx, ch, Vm, Vp, o.limiter);
    }
}

// One block = 4 rows of 64 lanes (see the MT tile tables).  D = 0: the lanes
// run along x from a-1, the rows along y (b..b+3) at z = c; lane l > 0 owns
// the face below its cell and takes the left state from lane l-1.  D = 1, 2:
// the lanes run along x from a, the rows along D over the faces b..b+3 (the
// third axis at c); row r > 0 takes the left state from row r-1, row 0
// forms the predictor of the cell below its face itself.  Every cell's
// predictor is thus formed once (plus one row per block across x).
template <int D, int PHYS, int PRED, int RK, int RS, typename R>
__global__ __launch_bounds__(NT) void k_mtflux(MtArgs<R> a)
{
    __shared__ R sVp[NV][NT];
    const KTile tl = a.tiles[blockIdx.x];
    const KBox bx = a.boxes[tl.box];
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, row = tid >> 6;
    const KOpts &o = a.o;
    const int dim = o.dim;
    int cc[3];
    if (D == 0) {
        cc[0] = tl.a - 1 + lane;
        cc[1] = tl.b + row;
        cc[2] = tl.c;
    } else if (D == 1) {
        cc[0] = tl.a + lane;
        cc[1] = tl.b + row;
        cc[2] = tl.c;
    } else {
        cc[0] = tl.a + lane;
        cc[1] = tl.c;
        cc[2] = tl.b + row;
    }
    bool valid = true;
#pragma unroll
    for (int e = 0; e < 3; e++) {
        if (e < dim) {
            const int lo = (e == D && D != 0) ? bx.g[e] : bx.g[e] - 1;
            valid = valid && cc[e] >= lo && cc[e] <= bx.g[e] + bx.n[e];
        } else {
            valid = valid && cc[e] == 0;
        }
    }
    const int sD = (D == 0) ? 1 : (D == 1 ? bx.N[0] : bx.N[0] * bx.N[1]);
    const R gam = R(o.gamma);
    const R dt = R(box_dt(bx, a.params)), ch = R(a.params[1]);
    const R dxD = R(bx.dx[D]);
    const R dtdx = dt / dxD;
    const Blk<R> bV(a.V + bx.woff, bx.cells);
    const int c = valid ? cidx(bx, cc[0], cc[1], cc[2]) : 0;
    R Vm[NV], Vp[NV], VL[NV];
    if (valid) {
        mt_predict<D, PHYS, PRED, RK>(bV, a.U, bx, c, sD, o, gam, dtdx, dxD, ch, Vm, Vp);
#pragma unroll
        for (int q = 0; q < NV; q++) sVp[q][tid] = Vp[q];
        if (D != 0 && row == 0) {
            R Vm2[NV];
            mt_predict<D, PHYS, PRED, RK>(bV, a.U, bx, c - sD, sD, o, gam, dtdx, dxD, ch, Vm2, VL);
        }
    }
    __syncthreads();
    const bool face = valid && (D == 0 ? (lane >= 1 && cc[0] >= bx.g[0]) : true);
    if (!face) return;
    if (D == 0 || row > 0) {
        const int src = (D == 0) ? tid - 1 : tid - 64;
#pragma unroll
        for (int q = 0; q < NV; q++) VL[q] = sVp[q][src];
    }
    R F[NV], smax;
    riemann<D, PHYS, RS>(VL, Vm, F, smax, gam, ch, o.glm, o.xspeeds);
    const Blk<R> bF(a.F[D] + bx.woff, bx.cells);
#pragma unroll
    for (int q = 0; q < NV; q++) bF.st(q, c, F[q]);
}

template <int DIM, typename R>
__global__ __launch_bounds__(NT) void k_mtT(MtArgs<R> a)
{
    const KTile tl = a.tiles[blockIdx.x];
    const KBox bx = a.boxes[tl.box];
    const int c = tl.a + (int)threadIdx.x;
    if (c >= bx.cells) return;
    const int cc[3] = { c % bx.N[0], (c / bx.N[0]) % bx.N[1], c / (bx.N[0] * bx.N[1]) };
    const int st[3] = { 1, bx.N[0], bx.N[0] * bx.N[1] };
    bool in[3], lay[3], need[3];
#pragma unroll
    for (int e = 0; e < DIM; e++) {
        in[e] = cc[e] >= bx.g[e] && cc[e] < bx.g[e] + bx.n[e];
        lay[e] = cc[e] >= bx.g[e] - 1 && cc[e] <= bx.g[e] + bx.n[e];
    }
    bool any = false;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        need[d] = lay[d];
#pragma unroll
        for (int e = 0; e < DIM; e++)
            if (e != d) need[d] = need[d] && in[e];
        any = any || need[d];
    }
    if (!any) return;
    // L_e = -(F_e(c + e) - F_e(c)) / dx_e, formed once for every T_d that uses it
    R L[DIM][NV];
#pragma unroll
    for (int e = 0; e < DIM; e++) {
        bool want = false;
#pragma unroll
        for (int d = 0; d < DIM; d++)
            if (d != e) want = want || need[d];
        const Blk<R> bF(a.F[e] + bx.woff, bx.cells);
        const R idx = R(1.0 / bx.dx[e]);
#pragma unroll
        for (int q = 0; q < NV; q++) L[e][q] = want ? -(bF.ld(q, c + st[e]) - bF.ld(q, c)) * idx : R(0);
    }
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        if (!need[d]) continue;
        const Blk<R> bT(a.T[d] + bx.woff, bx.cells);
#pragma unroll
        for (int q = 0; q < NV; q++) {
            R t;
            if constexpr (DIM == 3) t = (d == 0) ? L[1][q] + L[2][q] : ((d == 1) ? L[0][q] + L[2][q] : L[0][q] + L[1][q]);
            else t = (d == 0) ? L[1][q] : L[0][q];
            bT.st(q, c, t);
        }
    }
}

// ---------------------------------------------------------------------------
// k_sweep<D>: one direction of the corner-coupled update.
//
// A block owns a column of transverse positions and marches along D over
// the cells lo-1 .. lo+n (n+2 positions s = 0 .. n+1).  Items are processed
// in rounds of NT: each item computes its cell's normal predictor and
// corner-coupled states; the left state of the face below the item comes
// from the item DEL places earlier (in LDS, or carried over from the
// previous round); the update of a cell waits for the round holding the
// face above it.  DEL = 1 along x (pencils laid end to end), 64 across
// (64 transverse positions per row, x fastest for coalescing).
// ---------------------------------------------------------------------------

template <typename R> struct SweepArgs {
    const KBox *boxes;
    const KTile *tiles;
    const KReg *regs;
    const int *rface;  // per-face ranges of regs (see KBox::rface)
    const R *U;       // U^n (caller layout)
    R *Uout;          // U^{n+1} (caller layout)
    const R *V;       // V^n (workspace)
    const R *T[3];    // transverse increments of Eq. transv (workspace)
    const R *Vh;      // V^{n+1/2} (workspace) or null
    const R *PF;      // parabolic face slots of V^{n+1/2} (workspace) or null
    R *lam;           // per-cell rate accumulator (workspace, parabolic only)
    const R *L0;      // cooling coefficient (caller layout / 9) or null
    const unsigned char *leaf;  // cells entering max |dp/p| (caller layout / 9) or null = all
    const unsigned char *flag;  // App. B zone flags (workspace) or null
    double *reg;      // flux registers or null
    const double *params;
    double *rate;
    double *dpp;
    int *fails;
    KOpts o;
    int first, last;  // first / last sweep of the step
};

// Waves per SIMD the sweep is compiled for: the register budget is 512 /
// waves VGPRs.  FP32 fits two waves without spills; FP64 spills some of its
// doubled state at two waves, which measures faster on MI355X than one
// spill-free wave (13.5 vs 17.1 ms for a 256^3 step).  The FP32 par variant
// (non-ideal runs) needs ~180 registers: three waves with a few dozen bytes
// of spills measure 12 % faster than two waves on the x and y sweeps.
#ifndef CTU_SWEEP_WAVES_F32
#define CTU_SWEEP_WAVES_F32 2
#endif
#ifndef CTU_SWEEP_WAVES_F64
#define CTU_SWEEP_WAVES_F64 2
#endif
#ifndef CTU_SWEEP_WAVES_PAR_F32
#define CTU_SWEEP_WAVES_PAR_F32 3
#endif
template <int VAR, typename R> constexpr int sweep_waves()
{
    if constexpr (sizeof(R) == 8) return CTU_SWEEP_WAVES_F64;
    else return VAR == VAR_PAR ? CTU_SWEEP_WAVES_PAR_F32 : CTU_SWEEP_WAVES_F32;
}

template <int D, int PHYS, int PRED, int RK, int RS, int VAR, typename R>
__global__ __launch_bounds__(NT, (sweep_waves<VAR, R>())) void k_sweep(
    SweepArgs<R> a)
{
    constexpr int SHK = (VAR == VAR_SHOCK);
    constexpr int DEL = (D == 0) ? 1 : 64;
    __shared__ R sP[NV][NT];
    __shared__ R sF[NV][NT];
    __shared__ R sL[NT];
    __shared__ R cP[NV][DEL];
    __shared__ R cF[NV][DEL];
    __shared__ R cL[DEL];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const KTile tl = a.tiles[blockIdx.x];
    const KBox bx = a.boxes[tl.box];
    const KOpts o = variant_opts<VAR>(a.o);
    const int dim = o.dim;
    const int cs = (int)bx.cells;
    const int nD = bx.n[D];
    const int Lc = nD + 2;
    // transverse axes of D (t0 < t1 by direction index)
    constexpr int T0 = (D == 0) ? 1 : 0;
    constexpr int T1 = (D == 2) ? 1 : 2;
    const int nT0 = bx.n[T0], nT1 = (T1 < dim) ? bx.n[T1] : 1;
    const int npos_tot = nT0 * nT1;
    const int pos0 = tl.a;
    int items;
    int P = 0;
    // y / z: the tile owns rows [r0, r1) of its 64 pencils (faces and updates
    // below those rows); a segment that starts inside the line first re-runs
    // rows r0 - 2 and r0 - 1 for the states and the flux below row r0, with
    // the same arithmetic as the segment that owns them
    int r0 = 0, rs = 0;
    if (D == 0) {
        P = min(tl.b, npos_tot - pos0);
        items = P * Lc;
    } else {
        r0 = tl.b;
        rs = max(r0 - 2, 0);
        items = (tl.c - rs) * DEL;
    }
    const int sface = max(1, r0 - 1), supd = max(2, r0);
    const R gam = R(o.gamma);
    const R dt = R(box_dt(bx, a.params));
    const R ch = R(a.params[1]);
    const R dxD = R(bx.dx[D]);
    const R dtdx = dt / dxD;
    const R idxD = R(1) / dxD;
    const R hdt = R(0.5) * dt;
    int di, dj, dk;
    unit<D>(di, dj, dk);
    const Blk<R> bV(a.V + bx.woff, bx.cells), bU(a.U + bx.uoff, bx.cells), bUo(a.Uout + bx.uoff, bx.cells);
    const Blk<R> bT(a.T[D] + bx.woff, bx.cells);
    const unsigned char *fb = SHK ? a.flag + bx.woff / NV : nullptr;
    double rate_loc = 0.0, dpp_loc = 0.0;
    // last sweep: the cooling exponent 1 - beta and the floor's T^(1-beta);
    // the diffusive rate factor sum_d 2 / dx_d^2 of Eq. Ca
    const R com = R(1) - R(o.cool_beta);
    const R cxf = (a.last && o.cooling) ? powp(R(o.T_floor), com) : R(0);
    double rdx2 = 0.0;
#pragma unroll
    for (int e = 0; e < 3; e++)
        if (e < dim) rdx2 += 2.0 / (bx.dx[e] * bx.dx[e]);

    for (int base = 0; base < items; base += NT) {
        const int kit = base + tid;
        bool valid = kit < items;
        int s = 0, pos = 0;
        if (D == 0) {
            s = kit % Lc;
            pos = pos0 + kit / Lc;
        } else {
            s = rs + kit / DEL;
            pos = pos0 + kit % DEL;
            valid = valid && pos < npos_tot;
        }
        // ghosted coordinates of the item's cell
        int tc0 = pos % nT0, tc1 = pos / nT0;
        int cD = bx.g[D] - 1 + s;
        int ci = 0, cj = 0, ck = 0;
        if (D == 0) { ci = cD; cj = bx.g[1] + tc0; ck = bx.g[2] + tc1; }
        if (D == 1) { ci = bx.g[0] + tc0; cj = cD; ck = bx.g[2] + tc1; }
        if (D == 2) { ci = bx.g[0] + tc0; cj = bx.g[1] + tc1; ck = cD; }
        const int c = valid ? cidx(bx, ci, cj, ck) : 0;
        const int sD = (D == 0) ? 1 : (D == 1 ? bx.N[0] : bx.N[0] * bx.N[1]);

        R Um[NV];
        int fl = 0;
        double Wc = 0.0;  // RMHD: W of the item's cell, the start of the face-state inversions
        if (valid) {
            // ---- normal predictor (Sec. 3.2 / 3.3) ----
            R Vs[5][NV];
            constexpr int l0 = (RK == RK_PPM) ? 0 : 1, l1 = (RK == RK_PPM) ? 5 : 4;
#pragma unroll
            for (int l = l0; l < l1; l++)
#pragma unroll
                for (int q = 0; q < NV; q++) Vs[l][q] = bV.ld(q, c + (l - 2) * sD);
            // T_d of the item's cell (Eq. transv): in the FP32 fixed-option PPM
            // and MUSCL-Hancock sweeps loaded with the stencil, so that the
            // predictor covers its latency (their waves per SIMD stay as they
            // are); elsewhere just before the corner coupling
            constexpr bool TPRE = sizeof(R) == 4 && VAR == VAR_FAST && (RK == RK_PPM || PRED == PRED_MH);
            R tr[NV];
            if constexpr (TPRE) {
#pragma unroll
                for (int q = 0; q < NV; q++) tr[q] = bT.ld(q, c);
            }
            R Vm[NV], Vp[NV];
            Wc = w_guess<PHYS>(Vs[2], gam);
            // App. B: MinMod linear reconstruction near a flagged zone
            const bool mm = SHK && (fb[c] & FLAG_MINMOD);
            if (o.hyp_off) {
#pragma unroll
                for (int q = 0; q < NV; q++) Vm[q] = Vp[q] = Vs[2][q];
            } else if constexpr (PRED == PRED_CHAR) {
                if (SHK && mm) predict_char<D, RK_LIN>(Vs, o, gam, dtdx, dxD, ch, Vm, Vp, LIM_MINMOD);
                else predict_char<D, RK>(Vs, o, gam, dtdx, dxD, ch, Vm, Vp, o.limiter);
            } else {
                R U0[NV];
#pragma unroll
                for (int q = 0; q < NV; q++) U0[q] = bU.ld(q, c);
                fl |= predict_mh<D, PHYS>(Vs, U0, o, gam, dtdx, ch, Vm, Vp, mm ? LIM_MINMOD : o.limiter);
            }
            // ---- corner coupling (Eq. transv) ----
            // the T_d loads issue together, ahead of the conversions
            R Up[NV];
            if constexpr (!TPRE) {
#pragma unroll
                for (int q = 0; q < NV; q++) tr[q] = bT.ld(q, c);
            }
            p2c<PHYS>(Vm, Um, gam);
            p2c<PHYS>(Vp, Up, gam);
#pragma unroll
            for (int q = 0; q < NV; q++) {
                tr[q] *= hdt;
                Um[q] += tr[q];
                Up[q] += tr[q];
            }
#pragma unroll
            for (int q = 0; q < NV; q++) sP[q][tid] = Up[q];
        }
        __syncthreads();

        // ---- time-centred Riemann solve on the face below the item ----
        if (valid && s >= sface) {
            R UL[NV], VL[NV], VR[NV], F[NV];
#pragma unroll
            for (int q = 0; q < NV; q++) UL[q] = (tid >= DEL) ? sP[q][tid - DEL] : cP[q][tid];
            int fL = c2p<PHYS>(UL, VL, gam, Wc);
            int fR = c2p<PHYS>(Um, VR, gam, Wc);
            fl |= fL | fR;
            // rare fallback to the cell-centred states: reloaded, not kept live
            if (fL) {
#pragma unroll
                for (int q = 0; q < NV; q++) VL[q] = bV.ld(q, c - sD);
            }
            if (fR) {
#pragma unroll
                for (int q = 0; q < NV; q++) VR[q] = bV.ld(q, c);
            }
            R pL = VL[PRS], pR = VR[PRS], rL = VL[RHO], rR = VR[RHO];
            R smax = R(0);
            if (!o.hyp_off) {
                // App. B: HLL on the faces of a flagged zone
                if (SHK && ((fb[c - sD] | fb[c]) & FLAG_HLL))
                    riemann<D, PHYS, RS_HLL>(VL, VR, F, smax, gam, ch, o.glm, o.xspeeds);
                else riemann<D, PHYS, RS>(VL, VR, F, smax, gam, ch, o.glm, o.xspeeds);
            } else {
#pragma unroll
                for (int q = 0; q < NV; q++) F[q] = R(0);
            }
            if (o.parab) {
                R Pi[NV];
                parab_face<D>(a.PF + (bx.woff / NV) * (NPF * dim), cs, c, o, pL, pR, rL, rR, Pi);
#pragma unroll
                for (int q = 0; q < NV; q++) F[q] -= Pi[q];
            }
            // ---- flux registers: dt * A * (F - Pi) on listed faces ----
            if (a.reg && bx.reg1 > bx.reg0 && s >= r0) {
                int gt0 = bx.lo[T0] + tc0, gt1 = (T1 < dim) ? bx.lo[T1] + tc1 : 0;
                // only the rectangles on this face plane
                const int *rf = a.rface + bx.rface[D] + (s - 1);
                const int r0 = rf[0], r1 = rf[1];
                for (int r = r0; r < r1; r++) {
                    KReg rg = a.regs[r];
                    int u0 = gt0 - rg.tlo0, u1 = gt1 - rg.tlo1;
                    if (u0 < 0 || u0 >= rg.tn0 || u1 < 0 || u1 >= rg.tn1) continue;
                    double area = 1.0;
#pragma unroll
                    for (int e = 0; e < 3; e++)
                        if (e != D && e < dim) area *= bx.dx[e];
                    double *rp = a.reg + 9 * (rg.slot + (long long)u1 * rg.tn0 + u0);
                    double fac = (double)dt * area;
#pragma unroll
                    for (int q = 0; q < NV; q++) rp[q] += fac * (double)F[q];
                }
            }
#pragma unroll
            for (int q = 0; q < NV; q++) sF[q][tid] = F[q];
            sL[tid] = smax;
        }
        __syncthreads();

        // ---- conservative update (Eq. update) of the cell below the item ----
        if (valid && s >= supd) {
            const int cu = c - sD;
            R lamc = fmax(sL[tid], (tid >= DEL) ? sL[tid - DEL] : cL[tid]) * idxD;
            R u[NV];
            const Blk<R> bUb = a.first ? bU : bUo;
#pragma unroll
            for (int q = 0; q < NV; q++) {
                R Flo = (tid >= DEL) ? sF[q][tid - DEL] : cF[q][tid];
                u[q] = bUb.ld(q, cu) - dtdx * (sF[q][tid] - Flo);
            }
            R lamt = lamc;
            if (o.parab) {
                R *lp = a.lam + bx.woff / NV + cu;
                if (!a.first) lamt = fmax(lamt, *lp);
                if (!a.last) *lp = lamt;
            }
            if (a.last) {
                // ---- split point-local sources (Sec. 3.1) ----
                if (o.glm) {
                    R dxm = R(bx.dx[0]);
#pragma unroll
                    for (int e = 1; e < 3; e++)
                        if (e < dim) dxm = fmin(dxm, R(bx.dx[e]));
                    u[PSI] *= exp(-R(o.glm_alpha) * ch * dt / dxm);
                }
                if (o.cooling && a.L0) {
                    R v[NV];
                    c2p<PHYS_MHD>(u, v, gam);
                    R T = v[PRS] / v[RHO];
                    if (T > R(o.T_floor)) {
                        R x = powp(T, com) - com * (gam - R(1)) * v[RHO] * a.L0[bx.uoff / NV + cu] * dt;
                        x = fmax(x, cxf);
                        R pn = v[RHO] * powp(x, R(1) / com);
                        u[ENG] += (pn - v[PRS]) / (gam - R(1));
                        if (!a.leaf || a.leaf[bx.uoff / NV + cu])
                            dpp_loc = fmax(dpp_loc, (double)(fabs(pn - v[PRS]) / v[PRS]));
                    }
                }
                double r = (double)lamt;
                if (o.parab) {
                    R rho_h = a.Vh[bx.woff + RHO * cs + cu];
                    r += (double)diff_coeff(o, rho_h, gam) * rdx2;
                }
                rate_loc = fmax(rate_loc, r);
            } else if (!o.parab) {
                rate_loc = fmax(rate_loc, (double)lamt);
            }
#pragma unroll
            for (int q = 0; q < NV; q++) bUo.st(q, cu, u[q]);
        }
        count_fails(s >= r0 ? fl : 0, a.fails);
        __syncthreads();
        // ---- carry the last DEL items into the next round ----
        if (tid >= NT - DEL) {
            int ct = tid - (NT - DEL);
#pragma unroll
            for (int q = 0; q < NV; q++) {
                cP[q][ct] = sP[q][tid];
                cF[q][ct] = sF[q][tid];
            }
            cL[ct] = sL[tid];
        }
        __syncthreads();
    }
    double rb = ldexp(block_max(rate_loc, red), -bx.lshift);
    if (tid == 0 && a.rate) atomic_max_pos(a.rate, rb);
    if (a.last && a.dpp && o.cooling) {
        double db = block_max(dpp_loc, red);
        if (tid == 0) atomic_max_pos(a.dpp, db);
    }
}

// ---------------------------------------------------------------------------
// k_cfl: rate of Eq. Ca from cell-centred states (interior cells)
// ---------------------------------------------------------------------------

template <int PHYS, typename R>
__global__ __launch_bounds__(NT) void k_cfl(const KBox *boxes, const KTile *tiles, const R *U, double *rate, KOpts o)
{
    __shared__ double red[NT / 64];
    KTile tl = tiles[blockIdx.x];
    const KBox &bx = boxes[tl.box];
    const int it = tl.a + (int)threadIdx.x;
    const int tot = bx.n[0] * bx.n[1] * bx.n[2];
    double r = 0.0;
    if (it < tot) {
        int i = bx.g[0] + it % bx.n[0];
        int j = bx.g[1] + (it / bx.n[0]) % bx.n[1];
        int k = bx.g[2] + it / (bx.n[0] * bx.n[1]);
        int c = cidx(bx, i, j, k);
        R u[NV], v[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) u[q] = U[bx.uoff + q * bx.cells + c];
        R gam = R(o.gamma);
        c2p<PHYS>(u, v, gam);
        R lm, lp;
        wave_speeds<0, PHYS>(v, gam, lm, lp, o.xspeeds);
        r = fmax(r, (double)fmax(fabs(lm), fabs(lp)) / bx.dx[0]);
        wave_speeds<1, PHYS>(v, gam, lm, lp, o.xspeeds);
        r = fmax(r, (double)fmax(fabs(lm), fabs(lp)) / bx.dx[1]);
        if (o.dim == 3) {
            wave_speeds<2, PHYS>(v, gam, lm, lp, o.xspeeds);
            r = fmax(r, (double)fmax(fabs(lm), fabs(lp)) / bx.dx[2]);
        }
        if (o.parab) {
            R Dc = diff_coeff(o, v[RHO], gam);
#pragma unroll
            for (int e = 0; e < 3; e++)
                if (e < o.dim) r += 2.0 * (double)Dc / (bx.dx[e] * bx.dx[e]);
        }
    }
    double rb = ldexp(block_max(r, red), -bx.lshift);
    if (threadIdx.x == 0) atomic_max_pos(rate, rb);
}

// ---------------------------------------------------------------------------
// k_reflux: Eq. fluxcorr / Eq. addreflux, one thread per corrected coarse
// cell, entries of the cell applied in table order, FP64 arithmetic.
// ---------------------------------------------------------------------------

struct KRefl {
    int box, i, j, k, dir, side, nfine, pad;
    long long cslot;
    long long fslot[4];
    double scale;  // -side / (face area) / dx_dir of the coarse box (set on the host)
};

// With consume != 0 the register slots read are cleared afterwards: each
// slot belongs to one face and so to one corrected cell (one thread).
template <typename R>
__global__ __launch_bounds__(NT) void k_reflux(const KBox *boxes, const KRefl *ent, const int *cell_start, int ncell,
                                               R *U, double *reg, int consume)
{
    const int cid = xcd_block(blockIdx.x, gridDim.x) * NT + threadIdx.x;
    if (cid >= ncell) return;
    const int e0 = cell_start[cid], e1 = cell_start[cid + 1];
    const KRefl first = ent[e0];
    const KBox &bx = boxes[first.box];
    const int c = cidx(bx, first.i, first.j, first.k);
    double du[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) du[q] = 0.0;
    for (int e = e0; e < e1; e++) {
        const KRefl en = ent[e];
        // sum of the fine registers (slots in table order), fully unrolled so
        // that no slot index is taken from a run-time position in the entry
        double fine[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) fine[q] = 0.0;
#pragma unroll
        for (int f = 0; f < 4; f++) {
            if (f < en.nfine) {
                const double *r = reg + 9 * en.fslot[f];
#pragma unroll
                for (int q = 0; q < NV; q++) fine[q] += r[q];
            }
        }
        // reg holds dt*A*F; A/V = 1/dx on a Cartesian level
        const double *rc = reg + 9 * en.cslot;
#pragma unroll
        for (int q = 0; q < NV; q++) du[q] += en.scale * (fine[q] - rc[q]);
    }
#pragma unroll
    for (int q = 0; q < NV; q++) {
        R *p = &U[bx.uoff + q * bx.cells + c];
        *p = R((double)(*p) + du[q]);
    }
    if (consume) {
        for (int e = e0; e < e1; e++) {
            const KRefl en = ent[e];
#pragma unroll
            for (int q = 0; q < NV; q++) reg[9 * en.cslot + q] = 0.0;
#pragma unroll
            for (int f = 0; f < 4; f++) {
                if (f < en.nfine) {
#pragma unroll
                    for (int q = 0; q < NV; q++) reg[9 * en.fslot[f] + q] = 0.0;
                }
            }
        }
    }
}

}  // namespace ctu
