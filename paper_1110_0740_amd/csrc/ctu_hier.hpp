// ctu_hier.hpp -- device kernels of the AMR level cycle (Sec. 4): ghost
// filling by same-level periodic copy or coarse-to-fine prolongation of
// time-interpolated coarse data (Eq. prolong, Eq. intalpha), and restriction
// (Eq. avgdown), for refinement ratio 2 in 3D.
//
// A level's state array holds one ghosted block per box, q[v][k][j][i] with
// i fastest, at the box's element offset.  The ghost fill runs from copy and
// parent tables built on the host (below); restriction looks up the coarse
// box of each coarse cell in a candidate list built per fine box (the coarse
// interiors meeting its footprint), so no search spans the whole level.
#pragma once
#include <hip/hip_runtime.h>

#include "ctu_device.hpp"
#include "ctu_kernels.hpp"

namespace ctu {

struct HBox {
    int lo[3], n[3], N[3];  // interior origin (level-global) and extents; ghosted extents
    int pad;
    long long off;    // element offset of the box block in the level array
    long long cells;  // ghosted cells
};

struct HTile {
    int box, start;
};

__device__ __forceinline__ int wrapi(int a, int N)
{
    int r = a % N;
    return r < 0 ? r + N : r;
}

__device__ __forceinline__ bool holds(const HBox &b, int gi, int gj, int gk)
{
    return gi >= b.lo[0] && gi < b.lo[0] + b.n[0] && gj >= b.lo[1] && gj < b.lo[1] + b.n[1] && gk >= b.lo[2] &&
           gk < b.lo[2] + b.n[2];
}

// element index of interior cell (gi, gj, gk) of box b, variable 0
__device__ __forceinline__ long long hidx(const HBox &b, int gi, int gj, int gk, int ng)
{
    return b.off + ((long long)(gk - b.lo[2] + ng) * b.N[1] + (gj - b.lo[1] + ng)) * b.N[0] + (gi - b.lo[0] + ng);
}

// monotonised central slope of the one-sided differences (same value as
// minmod((dp + dm)/2, 2 minmod(dm, dp)))
template <typename R> __device__ __forceinline__ R mc_slope(R dp, R dm)
{
    R c = R(0.5) * (dp + dm);
    R m = fmin(fmin(fabs(c), R(2) * fabs(dp)), R(2) * fabs(dm));
    return (dp * dm > R(0)) ? copysign(m, c) : R(0);
}

// Ghost filling runs from tables built on the host when the hierarchy is
// created, so no thread searches for the box that holds its source:
//  * HCopy: a rectangle of a box's ghost cells that one same-level box
//    interior holds (under one periodic shift), with its place in both
//    boxes; every ghost cell of a level-0 box lies in exactly one;
//  * HPar: on levels >= 1, a coarse parent cell of a box's ghosted extent
//    with at least one child that is a ghost cell no same-level box holds
//    (`mask`, bit x + 2y + 4z), the parent's wrapped coarse coordinates, the
//    place of its first child in the box, and the coarse box whose interior
//    holds the parent and its six face neighbours (-1 - m: they lie in
//    several coarse boxes, listed as entry m of a table of seven box
//    indices, parent first, then -x, +x, -y, +y, -z, +z; INT_MIN: one of them
//    lies in no coarse interior, the children become NaN and are counted).
struct HCopy {
    int dst, src;  // box indices on the level
    int dlo[3];    // first cell in the destination's ghosted coordinates
    int slo[3];    // first cell in the source's ghosted coordinates
    int ext[3];
    int pad;
};

struct HPar {
    int box;
    int pc[3];     // parent, wrapped coarse-level coordinates
    int f0[3];     // child (0, 0, 0) in the box's ghosted coordinates
    int cbox;      // coarse box holding the 7-cell stencil, -1 - m, or HPAR_MISSING
    unsigned mask; // children to write
    int pad;
};

constexpr int HPAR_MISSING = -2147483647 - 1;

// same-level ghost copies, one thread per cell of a copy rectangle
template <typename R>
__global__ __launch_bounds__(NT) void k_hcopy(const HBox *box, const HCopy *cp, const HTile *tiles, R *U)
{
    const HTile t = tiles[xcd_block(blockIdx.x, gridDim.x)];
    const HCopy c = cp[t.box];
    const int li = t.start + threadIdx.x;
    if (li >= c.ext[0] * c.ext[1] * c.ext[2]) return;
    const int x = li % c.ext[0], y = (li / c.ext[0]) % c.ext[1], z = li / (c.ext[0] * c.ext[1]);
    const HBox D = box[c.dst], S = box[c.src];
    const long long dp = D.off + ((long long)(c.dlo[2] + z) * D.N[1] + (c.dlo[1] + y)) * D.N[0] + (c.dlo[0] + x);
    const long long sp = S.off + ((long long)(c.slo[2] + z) * S.N[1] + (c.slo[1] + y)) * S.N[0] + (c.slo[0] + x);
#pragma unroll
    for (int q = 0; q < NV; q++) U[dp + q * D.cells] = U[sp + q * S.cells];
}

// Eq. prolong for the ghost cells no same-level box holds, one thread per
// listed coarse parent: the parent's time-interpolated value (Eq. intalpha)
// and the MC slopes of its six face neighbours give each masked child
// u0 + sum_d (-+1/4) slope_d.  The nine variables are taken one after the
// other (the loop is kept rolled), so that a wave has the 7-cell stencil of
// one variable plane in flight rather than of all nine, which the L2 cannot
// hold for the parents of a box's x-ghost slabs (two to a row).  (One thread
// per parent and variable ran slower: each thread re-reads the parent's and
// the box's records.)
template <typename R>
__global__ __launch_bounds__(NT) void k_hprolong(const HBox *box, const HPar *par, int npar, const int *multi,
                                                 const HBox *cbox, int N, int ng, R *U, const R *Uo, const R *Un,
                                                 double alpha_d, int *missing)
{
    const int idx = xcd_block(blockIdx.x, gridDim.x) * NT + threadIdx.x;
    if (idx >= npar) return;
    const HPar P = par[idx];
    const HBox b = box[P.box];
    const int Nc = N / 2, pi = P.pc[0], pj = P.pc[1], pk = P.pc[2];
    const R alpha = R(alpha_d);
    const bool ok = P.cbox != HPAR_MISSING;
    // element offsets (variable 0) and variable strides of the parent and of
    // its -x, +x, -y, +y, -z, +z neighbours in their coarse boxes (one box,
    // or a row of the multi table), found once for the nine variables
    long long base[7];
    long long cl[7];
    if (ok) {
        const int *m = (P.cbox >= 0) ? nullptr : multi + 7 * (-1 - P.cbox);
#pragma unroll
        for (int t = 0; t < 7; t++) {
            int c[3] = { pi, pj, pk };
            if (t > 0) c[(t - 1) / 2] = wrapi(c[(t - 1) / 2] + ((t & 1) ? -1 : 1), Nc);
            const HBox C = cbox[m ? m[t] : P.cbox];
            base[t] = hidx(C, c[0], c[1], c[2], ng);
            cl[t] = C.cells;
        }
    }
    if (!ok && missing) atomicAdd(missing, __popc(P.mask));
    auto val = [&](int t, int q) -> R {
        const long long p = base[t] + (long long)q * cl[t];
        return (alpha == R(0)) ? Uo[p] : (R(1) - alpha) * Uo[p] + alpha * Un[p];
    };
#pragma unroll 1
    for (int q = 0; q < NV; q++) {
        R u0 = R(0), sl[3] = { R(0), R(0), R(0) };
        if (ok) {
            u0 = val(0, q);
#pragma unroll
            for (int d = 0; d < 3; d++) sl[d] = mc_slope(val(2 + 2 * d, q) - u0, u0 - val(1 + 2 * d, q));
        }
        for (int c8 = 0; c8 < 8; c8++) {
            if (!(P.mask & (1u << c8))) continue;
            const long long li = ((long long)(P.f0[2] + ((c8 >> 2) & 1)) * b.N[1] + (P.f0[1] + ((c8 >> 1) & 1))) *
                                     b.N[0] +
                                 P.f0[0] + (c8 & 1);
            R out;
            if (ok) {
                out = u0;
#pragma unroll
                for (int d = 0; d < 3; d++) out += (((c8 >> d) & 1) ? R(0.25) : R(-0.25)) * sl[d];
            } else {
                out = R(NAN);
            }
            U[b.off + li + (long long)q * b.cells] = out;
        }
    }
}

// Eq. avgdown (ratio 2, equal Cartesian volumes): each coarse cell under a
// fine box interior becomes the mean of its 8 children, summed in (k, j, i)
// child order.
template <typename R>
__global__ __launch_bounds__(NT) void k_havg(const HBox *fbox, const HTile *tiles, const int *pb_start,
                                             const int *pb_list, const HBox *cbox, int ng, const R *Uf, R *Uc,
                                             int *missing)
{
    const HTile t = tiles[blockIdx.x];
    const HBox f = fbox[t.box];
    const int m0 = f.n[0] / 2, m1 = f.n[1] / 2, m2 = f.n[2] / 2;
    const long long li = (long long)t.start + threadIdx.x;
    if (li >= (long long)m0 * m1 * m2) return;
    const int a = (int)(li % m0), b = (int)((li / m0) % m1), c = (int)(li / ((long long)m0 * m1));
    R s[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) s[q] = R(0);
    for (int dk = 0; dk < 2; dk++)
        for (int dj = 0; dj < 2; dj++)
            for (int di = 0; di < 2; di++) {
                const long long p = f.off + ((long long)(2 * c + dk + ng) * f.N[1] + (2 * b + dj + ng)) * f.N[0] +
                                    (2 * a + di + ng);
#pragma unroll
                for (int q = 0; q < NV; q++) s[q] += Uf[p + q * f.cells];
            }
    const int gi = f.lo[0] / 2 + a, gj = f.lo[1] / 2 + b, gk = f.lo[2] / 2 + c;
    for (int e = pb_start[t.box]; e < pb_start[t.box + 1]; e++) {
        const HBox cb = cbox[pb_list[e]];
        if (!holds(cb, gi, gj, gk)) continue;
        const long long p = hidx(cb, gi, gj, gk, ng);
#pragma unroll
        for (int q = 0; q < NV; q++) Uc[p + q * cb.cells] = s[q] / R(8);
        return;
    }
    if (missing) atomicAdd(missing, 1);
}

// fails_acc[q] += fails[q]
__global__ void k_add_fails(int *acc, const int *f)
{
    const int t = threadIdx.x;
    if (t < 5) acc[t] += f[t];
}

// Leaf mask of one level (one byte per ghosted cell, the state layout / 9):
// 1 on interior cells that no box of the next finer level covers (the
// cells of Sec. 4.2 whose source time step counts), 0 elsewhere.  fbox is
// null on the finest level.
__global__ __launch_bounds__(NT) void k_hleaf(const HBox *box, const HTile *tiles, const int *ch_start,
                                              const int *ch_list, const HBox *fbox, int ng, unsigned char *leaf)
{
    const HTile t = tiles[blockIdx.x];
    const HBox b = box[t.box];
    const long long li = (long long)t.start + threadIdx.x;
    if (li >= b.cells) return;
    const int i = (int)(li % b.N[0]), j = (int)((li / b.N[0]) % b.N[1]), k = (int)(li / ((long long)b.N[0] * b.N[1]));
    unsigned char v = 0;
    if (i >= ng && i < ng + b.n[0] && j >= ng && j < ng + b.n[1] && k >= ng && k < ng + b.n[2]) {
        v = 1;
        if (fbox) {
            const int gi = b.lo[0] + i - ng, gj = b.lo[1] + j - ng, gk = b.lo[2] + k - ng;
            for (int e = ch_start[t.box]; e < ch_start[t.box + 1]; e++) {
                const HBox f = fbox[ch_list[e]];
                if (2 * gi >= f.lo[0] && 2 * gi < f.lo[0] + f.n[0] && 2 * gj >= f.lo[1] && 2 * gj < f.lo[1] + f.n[1] &&
                    2 * gk >= f.lo[2] && 2 * gk < f.lo[2] + f.n[2]) {
                    v = 0;
                    break;
                }
            }
        }
    }
    leaf[b.off / NV + li] = v;
}

// Eq. RefCrit on sigma = U[var] for the interior cells of one level (ghosts
// filled): chi^2 = sum_d (D+ - D-)^2 / sum_d (|D+| + |D-| + eps sigma_ref,d)^2
// with undivided differences and sigma_ref,d = |s+| + 2|s0| + |s-|,
// evaluated in FP64; chi = 0 where the denominator vanishes.  tags (state
// layout / 9) get 1 where chi > chi_r, 0 on the other interior cells; the
// tagged cells are counted in *ntag (nullable).
template <typename R>
__global__ __launch_bounds__(NT) void k_htag(const HBox *box, const HTile *tiles, int ng, const R *U, int var,
                                             double eps, double chi_r, unsigned char *tags, int *ntag)
{
    const HTile t = tiles[blockIdx.x];
    const HBox b = box[t.box];
    const long long li = (long long)t.start + threadIdx.x;
    if (li >= b.cells) return;
    const int i = (int)(li % b.N[0]), j = (int)((li / b.N[0]) % b.N[1]), k = (int)(li / ((long long)b.N[0] * b.N[1]));
    if (!(i >= ng && i < ng + b.n[0] && j >= ng && j < ng + b.n[1] && k >= ng && k < ng + b.n[2])) return;
    const R *sg = U + b.off + (long long)var * b.cells;
    const double s0 = (double)sg[li];
    const long long st[3] = { 1, b.N[0], (long long)b.N[0] * b.N[1] };
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double sp = (double)sg[li + st[d]], sm = (double)sg[li - st[d]];
        const double dp = sp - s0, dm = s0 - sm;
        num += (dp - dm) * (dp - dm);
        const double ref = fabs(sp) + 2.0 * fabs(s0) + fabs(sm);
        const double e = fabs(dp) + fabs(dm) + eps * ref;
        den += e * e;
    }
    const double chi = (den > 0.0) ? sqrt(num / den) : 0.0;
    const unsigned char tag = chi > chi_r;
    tags[b.off / NV + li] = tag;
    if (tag && ntag) atomicAdd(ntag, 1);
}

// Next steps of every level (one thread): dt_l = min(C_a / rate_l,
// eps_c dt_l^n / dpp_l) (Eq. Ca, Eq. dt_cool, the latter where dpp_l > 0),
// dt0 = min_l 2^l dt_l (Eq. level_dt); params[l][0] <- dt0 / 2^l.
struct HDtArgs {
    double *params[16];
    const double *rate;
    const double *dpp;
    int nlev;
    double cfl, eps_c;
};

__global__ void k_next_dt(HDtArgs a)
{
    if (threadIdx.x != 0) return;
    double dt0 = INFINITY;
    for (int l = 0; l < a.nlev; l++) {
        double d = a.cfl / a.rate[l];
        if (a.dpp && a.dpp[l] > 0.0) d = fmin(d, a.eps_c * a.params[l][0] / a.dpp[l]);
        dt0 = fmin(dt0, d * (double)(1 << l));
    }
    for (int l = 0; l < a.nlev; l++) a.params[l][0] = dt0 / (double)(1 << l);
}

}  // namespace ctu
