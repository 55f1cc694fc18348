// ctu_device.hpp -- device building blocks of the CTU-GLM step for gfx950.
//
// Everything here is a __device__ inline function templated on the working
// precision R (float or double) and, where the cost matters, on the sweep
// direction D so that every vector component is addressed with a compile-time
// index (no scratch-memory indexing).  References are to Mignone et al.
// (ApJS 2012) and to the published methods it relies on.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctu {

enum { RHO = 0, MX1 = 1, MX2 = 2, MX3 = 3, ENG = 4, BX1 = 5, BX2 = 6, BX3 = 7, PSI = 8, NV = 9 };
enum { PRS = 4 };
// physics module: ideal MHD, relativistic MHD with the ideal EOS (Eq.
// gammaEos) or with the Taub-Matthews EOS (Eq. TMEos)
enum { PHYS_MHD = 0, PHYS_RMHD = 1, PHYS_RMHD_TM = 2 };
enum { RK_LIN = 0, RK_PPM = 1, RK_WENO = 2 };            // reconstruction kinds
enum { LIM_MC = 0, LIM_MINMOD = 1, LIM_VANLEER = 2, LIM_VANALBADA = 3 };
enum { PRED_CHAR = 0, PRED_MH = 1 };
enum { WREF_FACE = 0, WREF_CELL = 1, WREF_CW84 = 2 };
enum { RS_HLLD = 0, RS_HLL = 1, RS_RUSANOV = 2, RS_HLLC = 3, RS_ROE = 4 };
enum { F_RHO = 1, F_PRS = 2, F_INV = 4, F_VEL = 8, F_NAN = 16 };  // failure bits
enum { PB_VISC = 1, PB_RES = 2, PB_TC = 4 };

// Options as seen by the kernels (by value in every launch).
struct KOpts {
    int dim, limiter, wref, glm, parab, cooling, hyp_off, shock_r;  // shock_r: MinMod radius of App. B
    int xspeeds, pad;  // RMHD: 1 = exact fast magnetosonic speeds, 0 = isotropic bound
    double gamma, glm_alpha, nu, eta, kpar, kperp, phi, cool_beta, T_floor, shock_eps;
};

// App. B zone flags (one byte per cell): HLL on the zone's faces, MinMod
// linear reconstruction of the zone
constexpr unsigned char FLAG_HLL = 1, FLAG_MINMOD = 2;

// (normal, transverse, binormal) component indices of direction D.
template <int D> struct Ax {
    static constexpr int n = D, t = (D + 1) % 3, b = (D + 2) % 3;
};

template <typename R> __device__ __forceinline__ R sq(R x) { return x * x; }
// 1/sqrt(x): the hardware reciprocal root in FP32 (the FP32 unit runs with
// approximate divide / sqrt and flushed subnormals), the correctly rounded
// quotient in FP64
template <typename R> __device__ __forceinline__ R rsq(R x)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rsqf(x);
    else return R(1) / sqrt(x);
}
template <typename R> __device__ __forceinline__ R sgn1(R a) { return a < R(0) ? R(-1) : R(1); }

// ---------------------------------------------------------------------------
// Ideal MHD (Sec. 2.1, Eq. mhd, ideal-gas closure)
// ---------------------------------------------------------------------------

// igm1 = 1 / (Gamma - 1), formed once by the caller's hoisted division
template <typename R> __device__ __forceinline__ void p2c_mhd(const R *V, R *U, R igm1)
{
    R kin = V[RHO] * (sq(V[MX1]) + sq(V[MX2]) + sq(V[MX3]));
    R mag = sq(V[BX1]) + sq(V[BX2]) + sq(V[BX3]);
    U[RHO] = V[RHO];
    U[MX1] = V[RHO] * V[MX1];
    U[MX2] = V[RHO] * V[MX2];
    U[MX3] = V[RHO] * V[MX3];
    U[ENG] = V[PRS] * igm1 + R(0.5) * (kin + mag);
    U[BX1] = V[BX1];
    U[BX2] = V[BX2];
    U[BX3] = V[BX3];
    U[PSI] = V[PSI];
}

template <typename R> __device__ __forceinline__ int c2p_mhd(const R *U, R *V, R gm1)
{
    R rho = U[RHO];
    R ir = R(1) / rho;
    V[RHO] = rho;
    V[MX1] = U[MX1] * ir;
    V[MX2] = U[MX2] * ir;
    V[MX3] = U[MX3] * ir;
    V[BX1] = U[BX1];
    V[BX2] = U[BX2];
    V[BX3] = U[BX3];
    V[PSI] = U[PSI];
    R kin = U[MX1] * V[MX1] + U[MX2] * V[MX2] + U[MX3] * V[MX3];
    R mag = sq(U[BX1]) + sq(U[BX2]) + sq(U[BX3]);
    V[PRS] = gm1 * (U[ENG] - R(0.5) * (kin + mag));
    int f = 0;
    if (!(rho > R(0))) f |= F_RHO;
    if (!(V[PRS] > R(0))) f |= F_PRS;
    if (isnan(V[PRS]) || isnan(V[MX1] + V[MX2] + V[MX3])) f |= F_NAN;
    return f;
}

// fast magnetosonic speed along D
template <int D, typename R> __device__ __forceinline__ R cfast_mhd(const R *V, R gam)
{
    R ir = R(1) / V[RHO];
    R a2 = gam * V[PRS] * ir;
    R b2 = (sq(V[BX1]) + sq(V[BX2]) + sq(V[BX3])) * ir;
    R bn2 = sq(V[BX1 + D]) * ir;
    R s = a2 + b2;
    R disc = s * s - R(4) * a2 * bn2;
    disc = disc > R(0) ? disc : R(0);
    return sqrt(R(0.5) * (s + sqrt(disc)));
}

// conserved state and hyperbolic flux along D (GLM rows left to the caller)
template <int D, typename R> __device__ __forceinline__ void flux_mhd(const R *V, const R *U, R *F)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R vn = V[MX1 + n], Bn = V[BX1 + n];
    R pt = V[PRS] + R(0.5) * (sq(V[BX1]) + sq(V[BX2]) + sq(V[BX3]));
    R vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    F[RHO] = U[MX1 + n];
    F[MX1 + n] = U[MX1 + n] * vn - Bn * Bn + pt;
    F[MX1 + t] = U[MX1 + t] * vn - Bn * V[BX1 + t];
    F[MX1 + b] = U[MX1 + b] * vn - Bn * V[BX1 + b];
    F[ENG] = (U[ENG] + pt) * vn - vB * Bn;
    F[BX1 + n] = R(0);
    F[BX1 + t] = vn * V[BX1 + t] - Bn * V[MX1 + t];
    F[BX1 + b] = vn * V[BX1 + b] - Bn * V[MX1 + b];
    F[PSI] = R(0);
}

// ---------------------------------------------------------------------------
// Relativistic MHD (Sec. 2.2, Eq. rmhd; Eq. gammaEos or, TM = true, Eq.
// TMEos) -- always FP64 for the inversion; fluxes in the working precision.
// ---------------------------------------------------------------------------

// gas enthalpy w(rho, p)
template <bool TM, typename R> __device__ __forceinline__ R rmhd_w(R rho, R p, R gam)
{
    if constexpr (TM) return R(2.5) * p + sqrt(R(2.25) * p * p + rho * rho);
    else return rho + gam * p / (gam - R(1));
}

// sound speed squared, (dp/drho)_s rho / w along the adiabat de = (w/rho)
// drho of e = w - p: Gamma p / w, or p (5w - 8p) / (3 w (w - p)) for TM
template <bool TM, typename R> __device__ __forceinline__ R rmhd_cs2(R p, R w, R gam)
{
    if constexpr (TM) return p * (R(5) * w - R(8) * p) / (R(3) * w * (w - p));
    else return gam * p / w;
}

template <bool TM, typename R> __device__ __forceinline__ void p2c_rmhd(const R *V, R *U, R gam)
{
    R v2 = sq(V[MX1]) + sq(V[MX2]) + sq(V[MX3]);
    R B2 = sq(V[BX1]) + sq(V[BX2]) + sq(V[BX3]);
    R vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    R lor2 = R(1) / (R(1) - v2);
    R lor = sqrt(lor2);
    R w = rmhd_w<TM>(V[RHO], V[PRS], gam);
    R wl2 = w * lor2;
    U[RHO] = V[RHO] * lor;
    U[MX1] = (wl2 + B2) * V[MX1] - vB * V[BX1];
    U[MX2] = (wl2 + B2) * V[MX2] - vB * V[BX2];
    U[MX3] = (wl2 + B2) * V[MX3] - vB * V[BX3];
    U[ENG] = wl2 - V[PRS] + R(0.5) * (B2 + B2 * v2 - vB * vB) - U[RHO];
    U[BX1] = V[BX1];
    U[BX2] = V[BX2];
    U[BX3] = V[BX3];
    U[PSI] = V[PSI];
}

// Conserved -> primitive for RMHD: Newton-Raphson on W = w gamma^2 for the
// energy residual f(W) = W - p(W) + B^2/2 + (v^2(W) B^2 - S^2/W^2)/2 - D - E,
// with S = m.B and v^2(W) = (m^2 + S^2 (2W + B^2)/W^2)/(W + B^2)^2 and
// p(W) the EOS pressure of rho = D / gamma, w = W / gamma^2, kept inside a
// bracket [lo, hi] (bisection when a step leaves it).  As v^2 B^2 >= (v.B)^2
// and p <= k W (k = (Gamma - 1)/Gamma, or 1/4 for TM, whose p is at most
// w/4), f >= (1 - k) W - D - E: the upper end (E + D)/(1 - k) has f >= 0.
// Converged when |dW| <= tol max(W, E + D + B^2): the residual f carries
// rounding of order eps (E + D + B^2), so a strongly magnetised cell cannot
// resolve W better than that; tol = 1e-14 for FP64 storage, 1e-10 for FP32
// storage (Newton's quadratic convergence leaves an error far below the
// FP32 rounding of the result once a step is that small).
template <bool TM>
__device__ __forceinline__ int c2p_rmhd(const double *U, double *V, double gam, double Wguess, double tol = 1e-14)
{
    const double D = U[RHO], E = U[ENG];
    const double m2 = U[MX1] * U[MX1] + U[MX2] * U[MX2] + U[MX3] * U[MX3];
    const double S = U[MX1] * U[BX1] + U[MX2] * U[BX2] + U[MX3] * U[BX3];
    const double B2 = U[BX1] * U[BX1] + U[BX2] * U[BX2] + U[BX3] * U[BX3];
    const double gfac = (gam - 1.0) / gam;
    // p(rho, w) and its partial derivatives; TM: the root of
    // 4p^2 - 5wp + w^2 - rho^2 = 0 with w - 5p/2 >= 0
    auto pres = [&](double rho, double w, double &dpdw, double &dpdr) {
        if constexpr (TM) {
            const double s = sqrt(9.0 * w * w + 16.0 * rho * rho);
            dpdw = 0.125 * (5.0 - 9.0 * w / s);
            dpdr = -2.0 * rho / s;
            return 0.125 * (5.0 * w - s);
        } else {
            dpdw = gfac;
            dpdr = -gfac;
            return gfac * (w - rho);
        }
    };
    V[BX1] = U[BX1];
    V[BX2] = U[BX2];
    V[BX3] = U[BX3];
    V[PSI] = U[PSI];
    int fl = 0;
    if (!(D > 0.0)) fl |= F_RHO;
    double hi = TM ? (4.0 / 3.0) * (E + D) : gam * (E + D);
    double lo = 0.0;
    double W = (Wguess > 0.0 && Wguess < hi) ? Wguess : hi;
    const double wscale = fmax(E + D + B2, 0.0);
    bool conv = false;
    double v2 = 0.0;
    for (int it = 0; it < 60; ++it) {
        double sw = S / W;
        double WB = W + B2;
        double iWB = 1.0 / WB;
        v2 = (m2 + sw * sw * (2.0 * W + B2)) * iWB * iWB;
        double f, df;
        if (!(v2 < 1.0)) {
            // unphysical (superluminal) trial: the root lies above
            lo = W;
            f = -1.0;
            df = 0.0;
        } else {
            double sq1 = sqrt(1.0 - v2);
            double dpdw, dpdr;
            double p = pres(D * sq1, W * (1.0 - v2), dpdw, dpdr);
            f = W - p + 0.5 * B2 + 0.5 * (v2 * B2 - sw * sw) - D - E;
            double dv2 = -2.0 * sw * sw / (W * WB) - 2.0 * v2 * iWB;
            // w = W (1 - v^2), rho = D sqrt(1 - v^2)
            double dp = dpdw * ((1.0 - v2) - W * dv2) + dpdr * (-0.5 * D * dv2 / sq1);
            df = 1.0 - dp + 0.5 * B2 * dv2 + sw * sw / W;
            if (f > 0.0) hi = W; else lo = W;
        }
        double Wn = (df > 0.0) ? W - f / df : 0.5 * (lo + hi);
        // a Newton step within the tolerance has converged wherever it lands:
        // at the root the step rounds onto the bracket end just moved to W,
        // and falling back to bisection there would walk away from the root
        // (then back by halving the bracket, ~30 extra iterations)
        if (df > 0.0 && fabs(Wn - W) <= tol * fmax(W, wscale)) { W = Wn; conv = true; break; }
        if (!(Wn > lo && Wn < hi)) Wn = 0.5 * (lo + hi);
        if (fabs(Wn - W) <= tol * fmax(W, wscale)) { W = Wn; conv = true; break; }
        W = Wn;
    }
    double sw = S / W;
    v2 = (m2 + sw * sw * (2.0 * W + B2)) / ((W + B2) * (W + B2));
    double sq1 = sqrt(1.0 - v2);
    V[RHO] = D * sq1;
    {
        double dpdw, dpdr;
        V[PRS] = pres(V[RHO], W * (1.0 - v2), dpdw, dpdr);
    }
    double iWB = 1.0 / (W + B2);
    V[MX1] = (U[MX1] + sw * U[BX1]) * iWB;
    V[MX2] = (U[MX2] + sw * U[BX2]) * iWB;
    V[MX3] = (U[MX3] + sw * U[BX3]) * iWB;
    if (!conv) fl |= F_INV;
    if (!(V[RHO] > 0.0)) fl |= F_RHO;
    if (!(V[PRS] > 0.0)) fl |= F_PRS;
    if (!(v2 < 1.0)) fl |= F_VEL;
    if (isnan(V[PRS]) || isnan(V[RHO]) || isnan(V[MX1] + V[MX2] + V[MX3])) fl |= F_NAN;
    return fl;
}

template <int D, bool TM, typename R> __device__ __forceinline__ void flux_rmhd(const R *V, const R *U, R *F, R gam)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R v2 = sq(V[MX1]) + sq(V[MX2]) + sq(V[MX3]);
    R B2 = sq(V[BX1]) + sq(V[BX2]) + sq(V[BX3]);
    R vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    R wl2 = rmhd_w<TM>(V[RHO], V[PRS], gam) / (R(1) - v2);
    // E = -v x B; E_n E_c terms and |E|^2 = v^2 B^2 - (v.B)^2
    R E0 = V[MX3] * V[BX2] - V[MX2] * V[BX3];
    R E1 = V[MX1] * V[BX3] - V[MX3] * V[BX1];
    R E2 = V[MX2] * V[BX1] - V[MX1] * V[BX2];
    R Ev[3] = { E0, E1, E2 };
    R pt = V[PRS] + R(0.5) * (B2 + B2 * v2 - vB * vB);
    R vn = V[MX1 + n];
    F[RHO] = U[RHO] * vn;
    F[MX1 + n] = wl2 * vn * vn - V[BX1 + n] * V[BX1 + n] - Ev[n] * Ev[n] + pt;
    F[MX1 + t] = wl2 * vn * V[MX1 + t] - V[BX1 + n] * V[BX1 + t] - Ev[n] * Ev[t];
    F[MX1 + b] = wl2 * vn * V[MX1 + b] - V[BX1 + n] * V[BX1 + b] - Ev[n] * Ev[b];
    F[ENG] = U[MX1 + n] - U[RHO] * vn;
    F[BX1 + n] = R(0);
    F[BX1 + t] = vn * V[BX1 + t] - V[BX1 + n] * V[MX1 + t];
    F[BX1 + b] = vn * V[BX1 + b] - V[BX1 + n] * V[MX1 + b];
    F[PSI] = R(0);
}

// outer characteristic speeds along D from the isotropic bound
// a^2 = cs^2 + ca^2 - cs^2 ca^2 combined with v_n by relativistic addition
template <int D, bool TM, typename R>
__device__ __forceinline__ void speeds_rmhd(const R *V, R gam, R &lmin, R &lmax, int xs)
{
    R v2 = sq(V[MX1]) + sq(V[MX2]) + sq(V[MX3]);
    R B2 = sq(V[BX1]) + sq(V[BX2]) + sq(V[BX3]);
    R vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    R w = rmhd_w<TM>(V[RHO], V[PRS], gam);
    R cs2 = rmhd_cs2<TM>(V[PRS], w, gam);
    R bb2 = B2 * (R(1) - v2) + vB * vB;
    R ca2 = bb2 / (w + bb2);
    R a2 = cs2 + ca2 - cs2 * ca2;
    R vn = V[MX1 + D];
    R den = R(1) / (R(1) - v2 * a2);
    R disc = (R(1) - v2) * (R(1) - v2 * a2 - vn * vn * (R(1) - a2));
    disc = disc > R(0) ? disc : R(0);
    R root = sqrt(a2 * disc);
    lmin = (vn * (R(1) - a2) - root) * den;
    lmax = (vn * (R(1) - a2) + root) * den;
    if (!xs) return;
    // exact fast speeds: the outermost roots of the lab-frame dispersion
    // quartic g = w (1 - cs^2) A^4 - (w cs^2 + b^2) A^2 (1 - l^2)
    // + cs^2 Bl^2 (1 - l^2), A = gamma (v_n - l), Bl = b^n - l b^0; its four
    // roots are real and enclosed by the bounds above, so Newton from each
    // bound moves monotonically inwards to the fast root
    const R lor = R(1) / sqrt(R(1) - v2);
    const R b0 = lor * vB, bn = V[BX1 + D] / lor + b0 * vn;
    const R c4 = w * (R(1) - cs2), c2 = w * cs2 + bb2;
    const R tol = (sizeof(R) == 4) ? R(2e-7) : R(1e-15);
    R ls[2] = { lmin, lmax };
#pragma unroll
    for (int side = 0; side < 2; side++) {
        R l = ls[side];
        for (int it = 0; it < 100; it++) {
            const R A = lor * (vn - l), Bl = bn - l * b0, G = R(1) - l * l;
            const R g = c4 * A * A * A * A - c2 * A * A * G + cs2 * Bl * Bl * G;
            const R dg = -R(4) * lor * c4 * A * A * A - c2 * (-R(2) * lor * A * G - R(2) * l * A * A) +
                         cs2 * (-R(2) * b0 * Bl * G - R(2) * l * Bl * Bl);
            if (dg == R(0)) break;
            const R ln = l - g / dg;
            // speeds are bounded by 1: a step below tol is at the precision
            // of any root, also near l = 0, where a relative test would sit
            // under the rounding of g and run to the iteration cap
            const bool done = fabs(ln - l) <= tol * fmax(fabs(l), R(1));
            l = ln;
            if (done) break;
        }
        ls[side] = l;
    }
    lmin = ls[0];
    lmax = ls[1];
}

// ---------------------------------------------------------------------------
// Physics dispatch
// ---------------------------------------------------------------------------

template <int PHYS, typename R> __device__ __forceinline__ void p2c(const R *V, R *U, R gam)
{
    if constexpr (PHYS == PHYS_MHD) p2c_mhd(V, U, R(1) / (gam - R(1)));
    else p2c_rmhd<PHYS == PHYS_RMHD_TM>(V, U, gam);
}

// W = w gamma^2 of a primitive RMHD state (FP64): the starting point of the
// inversion of a nearby conserved state (0 for MHD, which needs none)
template <int PHYS, typename R> __device__ __forceinline__ double w_guess(const R *V, R gam)
{
    if constexpr (PHYS == PHYS_MHD) {
        return 0.0;
    } else {
        const double v2 = sq((double)V[MX1]) + sq((double)V[MX2]) + sq((double)V[MX3]);
        const double w = rmhd_w<PHYS == PHYS_RMHD_TM>((double)V[RHO], (double)V[PRS], (double)gam);
        return (v2 < 1.0) ? w / (1.0 - v2) : 0.0;
    }
}

// conserved -> primitive; RMHD always inverts in FP64
template <int PHYS, typename R> __device__ __forceinline__ int c2p(const R *U, R *V, R gam, double Wguess = 0.0)
{
    if constexpr (PHYS == PHYS_MHD) {
        return c2p_mhd(U, V, gam - R(1));
    } else {
        double u[NV], v[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) u[q] = (double)U[q];
        int f = c2p_rmhd<PHYS == PHYS_RMHD_TM>(u, v, (double)gam, Wguess, sizeof(R) == 4 ? 1e-10 : 1e-14);
#pragma unroll
        for (int q = 0; q < NV; q++) V[q] = (R)v[q];
        return f;
    }
}

// physical flux with the GLM rows: F_{B_n} = psi, F_psi = c_h^2 B_n
template <int D, int PHYS, typename R>
__device__ __forceinline__ void phys_flux(const R *V, R *U, R *F, R gam, R ch, int glm)
{
    p2c<PHYS>(V, U, gam);
    if constexpr (PHYS == PHYS_MHD) flux_mhd<D>(V, U, F);
    else flux_rmhd<D, PHYS == PHYS_RMHD_TM>(V, U, F, gam);
    if (glm) {
        F[BX1 + D] = V[PSI];
        F[PSI] = ch * ch * V[BX1 + D];
    }
}

template <int D, int PHYS, typename R>
__device__ __forceinline__ void wave_speeds(const R *V, R gam, R &lm, R &lp, int xs = 0)
{
    if constexpr (PHYS == PHYS_MHD) {
        R cf = cfast_mhd<D>(V, gam);
        lm = V[MX1 + D] - cf;
        lp = V[MX1 + D] + cf;
    } else {
        speeds_rmhd<D, PHYS == PHYS_RMHD_TM>(V, gam, lm, lp, xs);
    }
}

// ---------------------------------------------------------------------------
// Riemann solvers (Sec. 3.1: HLL, Rusanov, HLLC, HLLD; Roe further below) with the GLM interface subsystem
// ---------------------------------------------------------------------------

template <int D, int PHYS, typename R>
__device__ __forceinline__ void hll(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm, int xs)
{
    R lmL, lpL, lmR, lpR;
    wave_speeds<D, PHYS>(VL, gam, lmL, lpL, xs);
    wave_speeds<D, PHYS>(VR, gam, lmR, lpR, xs);
    R SL = fmin(lmL, lmR), SR = fmax(lpL, lpR);
    smax = fmax(fabs(SL), fabs(SR));
    R UL[NV], UR[NV], FL[NV], FR[NV];
    phys_flux<D, PHYS>(VL, UL, FL, gam, ch, glm);
    phys_flux<D, PHYS>(VR, UR, FR, gam, ch, glm);
    // upwind or fan flux, selected per lane
    R id = R(1) / (SR - SL);
#pragma unroll
    for (int q = 0; q < NV; q++) {
        R Fh = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) * id;
        F[q] = (SL >= R(0)) ? FL[q] : ((SR <= R(0)) ? FR[q] : Fh);
    }
}

// Rusanov (local Lax-Friedrichs; Sec. 3.1 lists it for both modules): the
// centred flux minus a (U_R - U_L)/2, a the largest signal speed magnitude
// of the two states (the HLL bounds' max(|S_L|, |S_R|))
template <int D, int PHYS, typename R>
__device__ __forceinline__ void rusanov(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm, int xs)
{
    R lmL, lpL, lmR, lpR;
    wave_speeds<D, PHYS>(VL, gam, lmL, lpL, xs);
    wave_speeds<D, PHYS>(VR, gam, lmR, lpR, xs);
    const R a = fmax(fmax(fabs(lmL), fabs(lpL)), fmax(fabs(lmR), fabs(lpR)));
    smax = a;
    R UL[NV], UR[NV], FL[NV], FR[NV];
    phys_flux<D, PHYS>(VL, UL, FL, gam, ch, glm);
    phys_flux<D, PHYS>(VR, UR, FR, gam, ch, glm);
#pragma unroll
    for (int q = 0; q < NV; q++) F[q] = R(0.5) * (FL[q] + FR[q]) - R(0.5) * a * (UR[q] - UL[q]);
}

// HLLD (Miyoshi & Kusano 2005) for states sharing the normal field.
//
// Evaluated without branches: all star states are formed and the flux of
// the region holding the interface is selected, so that the lanes of a wave
// never split over the five regions.  Quantities of regions not selected
// may be non-finite; they enter only through selects.
template <int D, typename R>
__device__ __forceinline__ void hlld(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R cfL = cfast_mhd<D>(VL, gam), cfR = cfast_mhd<D>(VR, gam);
    R uL = VL[MX1 + n], uR = VR[MX1 + n];
    R SL = fmin(uL - cfL, uR - cfR);
    R SR = fmax(uL + cfL, uR + cfR);
    smax = fmax(fabs(SL), fabs(SR));
    R UL[NV], UR[NV], FL[NV], FR[NV];
    phys_flux<D, PHYS_MHD>(VL, UL, FL, gam, ch, glm);
    phys_flux<D, PHYS_MHD>(VR, UR, FR, gam, ch, glm);
    const R Bn = VL[BX1 + n];
    const R Bn2 = Bn * Bn;
    R ptL = VL[PRS] + R(0.5) * (sq(VL[BX1]) + sq(VL[BX2]) + sq(VL[BX3]));
    R ptR = VR[PRS] + R(0.5) * (sq(VR[BX1]) + sq(VR[BX2]) + sq(VR[BX3]));
    R aL = (SL - uL) * VL[RHO], aR = (SR - uR) * VR[RHO];
    R iden = R(1) / (aR - aL);
    R SM = (aR * uR - aL * uL - ptR + ptL) * iden;
    R pts = (aR * ptL - aL * ptR + aL * aR * (uR - uL)) * iden;

    // single-star states; index 0 = left, 1 = right
    R rs[2], vt[2], vb[2], Bt[2], Bb[2], Es[2], sr[2], isr[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const R *V = s ? VR : VL;
        const R *U = s ? UR : UL;
        R S = s ? SR : SL;
        R pt = s ? ptR : ptL;
        R u = V[MX1 + n], rho = V[RHO];
        R Su = S - u, SSM = S - SM;
        R iSSM = R(1) / SSM;
        rs[s] = rho * Su * iSSM;
        R den = rho * Su * SSM - Bn2;
        R scale = rho * fabs(Su) * fabs(SSM) + Bn2;
        // degenerate case (S -> S_M with B_t -> 0): transverse values kept
        bool degen = fabs(den) <= R(sizeof(R) == 8 ? 1e-12 : 1e-6) * scale;
        R iden2 = R(1) / den;
        R fv = degen ? R(0) : Bn * (SM - u) * iden2;
        R fB = degen ? R(1) : (rho * Su * Su - Bn2) * iden2;
        vt[s] = V[MX1 + t] - V[BX1 + t] * fv;
        vb[s] = V[MX1 + b] - V[BX1 + b] * fv;
        Bt[s] = V[BX1 + t] * fB;
        Bb[s] = V[BX1 + b] * fB;
        R vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
        R vBs = SM * Bn + vt[s] * Bt[s] + vb[s] * Bb[s];
        Es[s] = (Su * U[ENG] - pt * u + pts * SM + Bn * (vB - vBs)) * iSSM;
        isr[s] = rsq(rs[s]);
        sr[s] = rs[s] * isr[s];
    }
    R SLs = SM - fabs(Bn) * isr[0];
    R SRs = SM + fabs(Bn) * isr[1];

    // region: outer (F_L or F_R), single star (L* or R*) or double star on
    // side k; k follows S_M inside the fan
    const bool outerL = SL >= R(0), outerR = SR <= R(0);
    const bool outer = outerL || outerR;
    const bool single = (SLs >= R(0)) || (SRs <= R(0));
    const bool k = outerL ? false : (outerR ? true : !(SM >= R(0)));

    // double-star states
    R sB = sgn1(Bn);
    R idn = R(1) / (sr[0] + sr[1]);
    R vtt = (sr[0] * vt[0] + sr[1] * vt[1] + (Bt[1] - Bt[0]) * sB) * idn;
    R vbb = (sr[0] * vb[0] + sr[1] * vb[1] + (Bb[1] - Bb[0]) * sB) * idn;
    R Btt = (sr[0] * Bt[1] + sr[1] * Bt[0] + sr[0] * sr[1] * (vt[1] - vt[0]) * sB) * idn;
    R Bbb = (sr[0] * Bb[1] + sr[1] * Bb[0] + sr[0] * sr[1] * (vb[1] - vb[0]) * sB) * idn;
    R vBss = SM * Bn + vtt * Btt + vbb * Bbb;

    // star and double-star states of side k
    const R rk = k ? rs[1] : rs[0], vtk = k ? vt[1] : vt[0], vbk = k ? vb[1] : vb[0];
    const R Btk = k ? Bt[1] : Bt[0], Bbk = k ? Bb[1] : Bb[0], Ek = k ? Es[1] : Es[0];
    const R srk = k ? sr[1] : sr[0];
    const R vBsk = SM * Bn + vtk * Btk + vbk * Bbk;
    R Us[NV], Uss[NV];
    Us[RHO] = rk;
    Us[MX1 + n] = rk * SM;
    Us[MX1 + t] = rk * vtk;
    Us[MX1 + b] = rk * vbk;
    Us[ENG] = Ek;
    Us[BX1 + n] = Bn;
    Us[BX1 + t] = Btk;
    Us[BX1 + b] = Bbk;
    Us[PSI] = k ? VR[PSI] : VL[PSI];
    Uss[RHO] = rk;
    Uss[MX1 + n] = rk * SM;
    Uss[MX1 + t] = rk * vtt;
    Uss[MX1 + b] = rk * vbb;
    Uss[ENG] = Ek + (k ? R(1) : R(-1)) * srk * (vBsk - vBss) * sB;
    Uss[BX1 + n] = Bn;
    Uss[BX1 + t] = Btt;
    Uss[BX1 + b] = Bbb;
    Uss[PSI] = Us[PSI];
    const R Sk = k ? SR : SL;
    const R Sks = k ? SRs : SLs;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        R Fk = k ? FR[q] : FL[q];
        R Uk = k ? UR[q] : UL[q];
        R f1 = Fk + Sk * (Us[q] - Uk);       // single-star flux
        R f2 = f1 + Sks * (Uss[q] - Us[q]);  // double-star flux
        F[q] = outer ? Fk : (single ? f1 : f2);
    }
}

// HLLC for MHD (Sec. 3.1 lists it for both modules), the single-contact
// solver of Li 2005 for states sharing the normal field.  HLL outer speeds;
// the contact moves with the HLL-averaged normal velocity S_M; both star
// states hold the HLL-averaged transverse field B*, and v*.B* is the HLL
// state's.  On the side k that holds the interface the jump conditions
// across its outer wave S give
//   rho* = rho (S - u)/(S - S_M),       p_t* = p_t + rho (S - u)(S_M - u),
//   (rho v_t)* = (rho v_t (S - u) - B_n (B_t* - B_t))/(S - S_M),
//   E* = ((S - u) E - p_t u + p_t* S_M + B_n (v.B - v*.B*))/(S - S_M),
// and the flux is F_k + S (U* - U_k).  As in HLLD only side k's star state
// is formed and every region is chosen by selects (no divergent branches);
// star quantities of a region not chosen may be non-finite.
template <int D, typename R>
__device__ __forceinline__ void hllc(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R cfL = cfast_mhd<D>(VL, gam), cfR = cfast_mhd<D>(VR, gam);
    R uL = VL[MX1 + n], uR = VR[MX1 + n];
    R SL = fmin(uL - cfL, uR - cfR);
    R SR = fmax(uL + cfL, uR + cfR);
    smax = fmax(fabs(SL), fabs(SR));
    R UL[NV], UR[NV], FL[NV], FR[NV];
    phys_flux<D, PHYS_MHD>(VL, UL, FL, gam, ch, glm);
    phys_flux<D, PHYS_MHD>(VR, UR, FR, gam, ch, glm);
    // HLL averages (S_R U_R - S_L U_L - (F_R - F_L)) / (S_R - S_L)
    const R id = R(1) / (SR - SL);
    auto hav = [&](int q) { return (SR * UR[q] - SL * UL[q] - (FR[q] - FL[q])) * id; };
    const R irh = R(1) / hav(RHO);
    const R SM = hav(MX1 + n) * irh;
    const R vth = hav(MX1 + t) * irh, vbh = hav(MX1 + b) * irh;
    const R Bth = hav(BX1 + t), Bbh = hav(BX1 + b);
    const R Bn = VL[BX1 + n];
    const R vBs = SM * Bn + vth * Bth + vbh * Bbh;

    const bool outerL = SL >= R(0), outerR = SR <= R(0);
    const bool outer = outerL || outerR;
    const bool k = outerL ? false : (outerR ? true : !(SM >= R(0)));
    R Vk[NV], Uk[NV], Fk[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Vk[q] = k ? VR[q] : VL[q];
        Uk[q] = k ? UR[q] : UL[q];
        Fk[q] = k ? FR[q] : FL[q];
    }
    const R S = k ? SR : SL;
    const R u = Vk[MX1 + n], rho = Vk[RHO];
    const R Su = S - u, iSSM = R(1) / (S - SM);
    const R pt = Vk[PRS] + R(0.5) * (sq(Vk[BX1]) + sq(Vk[BX2]) + sq(Vk[BX3]));
    const R pts = pt + rho * Su * (SM - u);
    const R vB = Vk[MX1] * Vk[BX1] + Vk[MX2] * Vk[BX2] + Vk[MX3] * Vk[BX3];
    R Us[NV];
    Us[RHO] = rho * Su * iSSM;
    Us[MX1 + n] = Us[RHO] * SM;
    Us[MX1 + t] = (Uk[MX1 + t] * Su - Bn * (Bth - Vk[BX1 + t])) * iSSM;
    Us[MX1 + b] = (Uk[MX1 + b] * Su - Bn * (Bbh - Vk[BX1 + b])) * iSSM;
    Us[ENG] = (Su * Uk[ENG] - pt * u + pts * SM + Bn * (vB - vBs)) * iSSM;
    Us[BX1 + n] = Bn;
    Us[BX1 + t] = Bth;
    Us[BX1 + b] = Bbh;
    Us[PSI] = Uk[PSI];
#pragma unroll
    for (int q = 0; q < NV; q++) F[q] = outer ? Fk[q] : Fk[q] + S * (Us[q] - Uk[q]);
}

// HLLC for relativistic MHD (Sec. 3.1 lists it for both modules; Mignone &
// Bodo 2006) for states sharing B_n.  With E the total energy U[ENG] + D
// (flux m_n) and the HLL averages U^hll, F^hll:
//  * B_n != 0: both star states hold the HLL transverse field B*; the
//    contact speed l* is the root with the minus sign of
//      (F_E - B*.F_B) l^2 - (E + F_mn - B*^2 - F_B^2) l + (m_n - B*.F_B) = 0
//    (F_B the HLL flux of the transverse field), the star transverse
//    velocity v*_t = (B*_t l* - F_Bt) / B_n, and
//    p_t* = F_mn - F_E l* + B_n (B_n / gamma*^2 + (v*.B*) l*);
//  * B_n = 0 (B_n^2 <= 1e-12 (B_n^2 + B*^2)): F_E l^2 - (E + F_mn) l + m_n = 0
//    and p_t* = F_mn - F_E l*; the transverse field jumps with the state.
// The star state of the side holding the interface comes from the jump
// conditions across its outer wave S, and the flux is F + S (U* - U).  The
// root is formed as 2c / (-b + sqrt(b^2 - 4ac)).  A star state that is not
// admissible (negative discriminant, l* outside (S_L, S_R), v*^2 >= 1,
// D* <= 0) gives the HLL flux.  Both field cases, both sides and the
// fallback are formed and chosen by selects.
template <int D, int PHYS, typename R>
__device__ __forceinline__ void hllc_rmhd(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm, int xs)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R lmL, lpL, lmR, lpR;
    wave_speeds<D, PHYS>(VL, gam, lmL, lpL, xs);
    wave_speeds<D, PHYS>(VR, gam, lmR, lpR, xs);
    const R SL = fmin(lmL, lmR), SR = fmax(lpL, lpR);
    smax = fmax(fabs(SL), fabs(SR));
    R UL[NV], UR[NV], FL[NV], FR[NV];
    phys_flux<D, PHYS>(VL, UL, FL, gam, ch, glm);
    phys_flux<D, PHYS>(VR, UR, FR, gam, ch, glm);
    const R id = R(1) / (SR - SL);
    R Uh[NV], Fh[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Uh[q] = (SR * UR[q] - SL * UL[q] - (FR[q] - FL[q])) * id;
        Fh[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) * id;
    }
    const R Eh = Uh[ENG] + Uh[RHO], FEh = Fh[ENG] + Fh[RHO];
    const R Bn = VL[BX1 + n];
    const R Bt = Uh[BX1 + t], Bb = Uh[BX1 + b], Ft = Fh[BX1 + t], Fb = Fh[BX1 + b];
    const bool mag = Bn * Bn > R(1e-12) * (Bn * Bn + Bt * Bt + Bb * Bb);
    const R BF = mag ? Bt * Ft + Bb * Fb : R(0);
    const R qa = FEh - BF;
    const R qb = -(Eh + Fh[MX1 + n]) + (mag ? Bt * Bt + Bb * Bb + Ft * Ft + Fb * Fb : R(0));
    const R qc = Uh[MX1 + n] - BF;
    const R disc = qb * qb - R(4) * qa * qc;
    bool ok = disc >= R(0);
    const R ls = R(2) * qc / (-qb + sqrt(fmax(disc, R(0))));
    ok = ok && ls > SL && ls < SR;
    const R iBn = mag ? R(1) / Bn : R(0);
    const R vt = (Bt * ls - Ft) * iBn, vb = (Bb * ls - Fb) * iBn;
    const R ig2 = R(1) - (ls * ls + vt * vt + vb * vb);
    ok = ok && (!mag || ig2 > R(0));
    const R vBs = mag ? ls * Bn + vt * Bt + vb * Bb : R(0);
    const R pts = Fh[MX1 + n] - FEh * ls + (mag ? Bn * (Bn * ig2 + vBs * ls) : R(0));

    const bool k = !(ls >= R(0));
    R Uk[NV], Fk[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Uk[q] = k ? UR[q] : UL[q];
        Fk[q] = k ? FR[q] : FL[q];
    }
    const R S = k ? SR : SL;
    const R iS = R(1) / (S - ls);
    R Us[NV];
    Us[RHO] = (S * Uk[RHO] - Fk[RHO]) * iS;
    const R Es = (S * (Uk[ENG] + Uk[RHO]) - Uk[MX1 + n] + pts * ls - vBs * Bn) * iS;
    Us[MX1 + n] = (Es + pts) * ls - vBs * Bn;
    const R mt = S * Uk[MX1 + t] - Fk[MX1 + t], mb = S * Uk[MX1 + b] - Fk[MX1 + b];
    Us[MX1 + t] = (mag ? mt - Bn * (Bt * ig2 + vBs * vt) : mt) * iS;
    Us[MX1 + b] = (mag ? mb - Bn * (Bb * ig2 + vBs * vb) : mb) * iS;
    Us[BX1 + t] = mag ? Bt : (S * Uk[BX1 + t] - Fk[BX1 + t]) * iS;
    Us[BX1 + b] = mag ? Bb : (S * Uk[BX1 + b] - Fk[BX1 + b]) * iS;
    Us[ENG] = Es - Us[RHO];
    Us[BX1 + n] = Bn;
    Us[PSI] = Uk[PSI];
    ok = ok && Us[RHO] > R(0);
    const bool outerL = SL >= R(0), outerR = SR <= R(0);
#pragma unroll
    for (int q = 0; q < NV; q++) {
        const R fs = ok ? Fk[q] + S * (Us[q] - Uk[q]) : Fh[q];
        F[q] = outerL ? FL[q] : (outerR ? FR[q] : fs);
    }
}

// HLLD for relativistic MHD (Mignone, Ugliano & Bodo 2009) for states
// sharing B_n.  Between the outer fast waves (HLL's speeds) the total
// pressure p is uniform; for a trial p the state a behind each fast wave S
// is closed-form in R = S U - F (E the total energy U[ENG] + D):
//   A = R_mn - S R_E + p (1 - S^2), G = R_Bt^2 + R_Bb^2, C = R_mt R_Bt + R_mb R_Bb,
//   Q = -A - G + B_n^2 (1 - S^2), X = B_n (A S B_n + C) - (A + G)(S p + R_E),
//   v_n = (B_n (A B_n + S C) - (A + G)(p + R_mn)) / X,
//   v_t = (Q R_mt + R_Bt (C + B_n (S R_mn - R_E))) / X,
//   B_t = (R_Bt - B_n v_t) / (S - v_n), w_t = p + (R_E - v.R_m) / (S - v_n);
// the rotational discontinuity beside it moves at K_n, K = (R_m + p e_n +
// eta R_B) / (S p + R_E + eta B_n), eta = -+ sgn(B_n) sqrt(w_t) (left /
// right); the contact region holds the field B_c conserved across both
// rotational discontinuities and, on each side, v_c = K - B_c (1 - K^2) /
// (eta - K.B_c).  p solves v_cn(R) = v_cn(L) by secant steps from the
// relativistic HLLC estimate (and 1.025 times it) until successive iterates
// agree to 1e-14 (FP64) / 1e-6 (FP32) relatively (FP32 also: the residual
// is below 4e-7, the rounding of the velocities), at most 40 steps.  The
// fan's states follow from the jump conditions and the flux from F* = F +
// S (U* - U) across each wave.  B_n = 0 (B_n^2 <= 1e-12 (B_n^2 + B^hll_t^2))
// or a fan that is not admissible (no convergence, |v| >= 1, D <= 0,
// w_t <= p, wave speeds out of order) takes the HLLC flux.
template <typename R> struct RHSide {
    R U[8];  // D, m_n, m_t, m_b, E, B_n, B_t, B_b
    R v[3], B[3], wt, eta, K[3];
    bool ok;
};

template <typename R>
__device__ __forceinline__ void rhlld_astate(const R *Rv, R S, R p, R Bn, R sg, RHSide<R> &a)
{
    const R A = Rv[1] - S * Rv[4] + p * (R(1) - S * S);
    const R Gq = Rv[6] * Rv[6] + Rv[7] * Rv[7];
    const R C = Rv[2] * Rv[6] + Rv[3] * Rv[7];
    const R Q = -A - Gq + Bn * Bn * (R(1) - S * S);
    const R X = Bn * (A * S * Bn + C) - (A + Gq) * (S * p + Rv[4]);
    const R iX = R(1) / X;
    a.v[0] = (Bn * (A * Bn + S * C) - (A + Gq) * (p + Rv[1])) * iX;
    a.v[1] = (Q * Rv[2] + Rv[6] * (C + Bn * (S * Rv[1] - Rv[4]))) * iX;
    a.v[2] = (Q * Rv[3] + Rv[7] * (C + Bn * (S * Rv[1] - Rv[4]))) * iX;
    const R iS = R(1) / (S - a.v[0]);
    a.B[0] = Bn;
    a.B[1] = (Rv[6] - Bn * a.v[1]) * iS;
    a.B[2] = (Rv[7] - Bn * a.v[2]) * iS;
    a.wt = p + (Rv[4] - (a.v[0] * Rv[1] + a.v[1] * Rv[2] + a.v[2] * Rv[3])) * iS;
    const R vB = a.v[0] * a.B[0] + a.v[1] * a.B[1] + a.v[2] * a.B[2];
    a.U[0] = Rv[0] * iS;
    a.U[4] = (Rv[4] + p * a.v[0] - vB * Bn) * iS;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        a.U[1 + k] = (a.U[4] + p) * a.v[k] - vB * a.B[k];
        a.U[5 + k] = a.B[k];
    }
    const R v2 = a.v[0] * a.v[0] + a.v[1] * a.v[1] + a.v[2] * a.v[2];
    a.ok = isfinite(X) && X != R(0) && v2 < R(1) && a.wt > p && a.U[0] > R(0);
    a.eta = sg * sgn1(Bn) * sqrt(fmax(a.wt, R(0)));
    const R iden = R(1) / (S * p + Rv[4] + a.eta * Bn);
    a.K[0] = (Rv[1] + p + a.eta * Rv[5]) * iden;
    a.K[1] = (Rv[2] + a.eta * Rv[6]) * iden;
    a.K[2] = (Rv[3] + a.eta * Rv[7]) * iden;
}

template <typename R>
__device__ __forceinline__ R rhlld_fan(const R *RL, const R *RR, R SL, R SR, R p, R Bn, RHSide<R> &aL, RHSide<R> &aR,
                                       R *Bc, R *vcL, R *vcR)
{
    rhlld_astate(RL, SL, p, Bn, R(-1), aL);
    rhlld_astate(RR, SR, p, Bn, R(1), aR);
    const R idK = R(1) / (aR.K[0] - aL.K[0]);
    Bc[0] = Bn;
#pragma unroll
    for (int k = 1; k < 3; k++)
        Bc[k] = ((aR.B[k] * (aR.K[0] - aR.v[0]) + Bn * aR.v[k]) - (aL.B[k] * (aL.K[0] - aL.v[0]) + Bn * aL.v[k])) * idK;
    {
        const R K2 = aL.K[0] * aL.K[0] + aL.K[1] * aL.K[1] + aL.K[2] * aL.K[2];
        const R KB = aL.K[0] * Bc[0] + aL.K[1] * Bc[1] + aL.K[2] * Bc[2];
        const R y = (R(1) - K2) / (aL.eta - KB);
#pragma unroll
        for (int k = 0; k < 3; k++) vcL[k] = aL.K[k] - Bc[k] * y;
    }
    {
        const R K2 = aR.K[0] * aR.K[0] + aR.K[1] * aR.K[1] + aR.K[2] * aR.K[2];
        const R KB = aR.K[0] * Bc[0] + aR.K[1] * Bc[1] + aR.K[2] * Bc[2];
        const R y = (R(1) - K2) / (aR.eta - KB);
#pragma unroll
        for (int k = 0; k < 3; k++) vcR[k] = aR.K[k] - Bc[k] * y;
    }
    return vcR[0] - vcL[0];
}

template <int D, int PHYS, typename R>
__device__ __forceinline__ void hlld_rmhd(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm, int xs)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R lmL, lpL, lmR, lpR;
    wave_speeds<D, PHYS>(VL, gam, lmL, lpL, xs);
    wave_speeds<D, PHYS>(VR, gam, lmR, lpR, xs);
    const R SL = fmin(lmL, lmR), SR = fmax(lpL, lpR);
    smax = fmax(fabs(SL), fabs(SR));
    R U9L[NV], U9R[NV], F9L[NV], F9R[NV];
    phys_flux<D, PHYS>(VL, U9L, F9L, gam, ch, glm);
    phys_flux<D, PHYS>(VR, U9R, F9R, gam, ch, glm);
    if (SL >= R(0) || SR <= R(0)) {
#pragma unroll
        for (int q = 0; q < NV; q++) F[q] = (SL >= R(0)) ? F9L[q] : F9R[q];
        return;
    }
    constexpr int map[8] = { RHO, MX1 + n, MX1 + t, MX1 + b, ENG, BX1 + n, BX1 + t, BX1 + b };
    R UL[8], UR[8], FL[8], FR[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        UL[k] = U9L[map[k]];
        UR[k] = U9R[map[k]];
        FL[k] = F9L[map[k]];
        FR[k] = F9R[map[k]];
    }
    UL[4] += UL[0];
    UR[4] += UR[0];
    FL[4] += FL[0];
    FR[4] += FR[0];
    FL[5] = R(0);
    FR[5] = R(0);
    const R Bn = VL[BX1 + n];
    const R id = R(1) / (SR - SL);
    R Uh[8], Fh[8], RL[8], RR[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        Uh[k] = (SR * UR[k] - SL * UL[k] - (FR[k] - FL[k])) * id;
        Fh[k] = (SR * FL[k] - SL * FR[k] + SL * SR * (UR[k] - UL[k])) * id;
        RL[k] = SL * UL[k] - FL[k];
        RR[k] = SR * UR[k] - FR[k];
    }
    bool ok = Bn * Bn > R(1e-12) * (Bn * Bn + Uh[6] * Uh[6] + Uh[7] * Uh[7]);
    R p0 = R(0);
    if (ok) {
        const R BF = Uh[6] * Fh[6] + Uh[7] * Fh[7];
        const R qa = Fh[4] - BF;
        const R qb = -(Uh[4] + Fh[1]) + Uh[6] * Uh[6] + Uh[7] * Uh[7] + Fh[6] * Fh[6] + Fh[7] * Fh[7];
        const R qc = Uh[1] - BF;
        const R disc = qb * qb - R(4) * qa * qc;
        const R ls = R(2) * qc / (-qb + sqrt(fmax(disc, R(0))));
        const R vt = (Uh[6] * ls - Fh[6]) / Bn, vb = (Uh[7] * ls - Fh[7]) / Bn;
        const R ig2 = R(1) - ls * ls - vt * vt - vb * vb;
        const R vBs = ls * Bn + vt * Uh[6] + vb * Uh[7];
        p0 = Fh[1] - Fh[4] * ls + Bn * (Bn * ig2 + vBs * ls);
        ok = disc >= R(0) && p0 > R(0) && isfinite(p0);
    }
    RHSide<R> aL, aR;
    R Bc[3], vcL[3], vcR[3], p = p0;
    if (ok) {
        constexpr R tol = (sizeof(R) == 8) ? R(1e-14) : R(1e-6);
        R pa = p0, pb = R(1.025) * p0;
        R fa = rhlld_fan(RL, RR, SL, SR, pa, Bn, aL, aR, Bc, vcL, vcR);
        R fb = rhlld_fan(RL, RR, SL, SR, pb, Bn, aL, aR, Bc, vcL, vcR);
        bool conv = false;
        for (int it = 0; it < 40; it++) {
            if (fb == fa || !isfinite(fa) || !isfinite(fb)) break;
            const R pc = pb - fb * (pb - pa) / (fb - fa);
            pa = pb;
            fa = fb;
            pb = pc;
            fb = rhlld_fan(RL, RR, SL, SR, pb, Bn, aL, aR, Bc, vcL, vcR);
            // FP32: a contact-velocity mismatch at the rounding of the
            // velocities (units of c) is converged even where the pressure
            // step cannot get below tol (small dv/dp)
            if (fabs(pb - pa) <= tol * fabs(pb) || (sizeof(R) == 4 && fabs(fb) <= R(4e-7))) {
                conv = true;
                break;
            }
        }
        if (fb == R(0)) conv = true;
        // FP32: iterates that stop moving within a few ulps count as converged
        if (sizeof(R) == 4 && fabs(pb - pa) <= tol * fabs(pb)) conv = true;
        p = pb;
        (void)rhlld_fan(RL, RR, SL, SR, p, Bn, aL, aR, Bc, vcL, vcR);
        const R vc2 = vcL[0] * vcL[0] + vcL[1] * vcL[1] + vcL[2] * vcL[2];
        const R vr2 = vcR[0] * vcR[0] + vcR[1] * vcR[1] + vcR[2] * vcR[2];
        ok = conv && p > R(0) && aL.ok && aR.ok && vc2 < R(1) && vr2 < R(1) && SL <= aL.K[0] &&
             aL.K[0] <= vcL[0] && vcR[0] <= aR.K[0] && aR.K[0] <= SR;
    }
    if (!ok) {
        R VLc[NV], VRc[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) {
            VLc[q] = VL[q];
            VRc[q] = VR[q];
        }
        hllc_rmhd<D, PHYS>(VLc, VRc, F, smax, gam, ch, glm, xs);
        return;
    }
    R vc[3];
#pragma unroll
    for (int k = 0; k < 3; k++) vc[k] = R(0.5) * (vcL[k] + vcR[k]);
    const R vBc = vc[0] * Bc[0] + vc[1] * Bc[1] + vc[2] * Bc[2];
    R UcL[8], UcR[8];
    {
        const R la = aL.K[0], iS = R(1) / (la - vc[0]);
        UcL[0] = aL.U[0] * (la - aL.v[0]) * iS;
        UcL[4] = (la * aL.U[4] - aL.U[1] + p * vc[0] - vBc * Bn) * iS;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            UcL[1 + k] = (UcL[4] + p) * vc[k] - vBc * Bc[k];
            UcL[5 + k] = Bc[k];
        }
    }
    {
        const R la = aR.K[0], iS = R(1) / (la - vc[0]);
        UcR[0] = aR.U[0] * (la - aR.v[0]) * iS;
        UcR[4] = (la * aR.U[4] - aR.U[1] + p * vc[0] - vBc * Bn) * iS;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            UcR[1 + k] = (UcR[4] + p) * vc[k] - vBc * Bc[k];
            UcR[5 + k] = Bc[k];
        }
    }
    R Fr[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const R FaL = FL[k] + SL * (aL.U[k] - UL[k]);
        const R FcL = FaL + aL.K[0] * (UcL[k] - aL.U[k]);
        const R FaR = FR[k] + SR * (aR.U[k] - UR[k]);
        const R FcR = FaR + aR.K[0] * (UcR[k] - aR.U[k]);
        Fr[k] = (aL.K[0] >= R(0)) ? FaL : ((vc[0] >= R(0)) ? FcL : ((aR.K[0] >= R(0)) ? FcR : FaR));
    }
    Fr[4] -= Fr[0];
#pragma unroll
    for (int k = 0; k < 8; k++) F[map[k]] = Fr[k];
    F[PSI] = R(0);
}

// Roe's solver (defined after the eigenvector helpers it uses)
template <int D, typename R>
__device__ __forceinline__ void roe(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm);

// Interface solve: exact solution of the linear (B_n, psi) subsystem of
// Eq. glm2x2 (psi + c_h B_n carried from the left, psi - c_h B_n from the
// right), then the chosen solver on the states with the common B_n.  VL, VR are
// modified in place (their B_n is replaced).
template <int D, int PHYS, int RS, typename R>
__device__ __forceinline__ void riemann(R *VL, R *VR, R *F, R &smax, R gam, R ch, int glm, int xs = 0)
{
    R Bm, psim;
    if (glm) {
        const R ih = R(0.5) / ch;  // loop-invariant, hoisted
        Bm = R(0.5) * (VL[BX1 + D] + VR[BX1 + D]) - (VR[PSI] - VL[PSI]) * ih;
        psim = R(0.5) * (VL[PSI] + VR[PSI]) - R(0.5) * ch * (VR[BX1 + D] - VL[BX1 + D]);
    } else {
        Bm = R(0.5) * (VL[BX1 + D] + VR[BX1 + D]);
        psim = R(0);
    }
    VL[BX1 + D] = Bm;
    VR[BX1 + D] = Bm;
    if constexpr (RS == RS_HLLD && PHYS == PHYS_MHD) hlld<D>(VL, VR, F, smax, gam, ch, glm);
    else if constexpr (RS == RS_HLLD) hlld_rmhd<D, PHYS>(VL, VR, F, smax, gam, ch, glm, xs);
    else if constexpr (RS == RS_HLLC && PHYS == PHYS_MHD) hllc<D>(VL, VR, F, smax, gam, ch, glm);
    else if constexpr (RS == RS_ROE && PHYS == PHYS_MHD) roe<D>(VL, VR, F, smax, gam, ch, glm);
    else if constexpr (RS == RS_HLLC) hllc_rmhd<D, PHYS>(VL, VR, F, smax, gam, ch, glm, xs);
    else if constexpr (RS == RS_RUSANOV) rusanov<D, PHYS>(VL, VR, F, smax, gam, ch, glm, xs);
    else hll<D, PHYS>(VL, VR, F, smax, gam, ch, glm, xs);
    F[BX1 + D] = glm ? psim : R(0);
    F[PSI] = glm ? ch * ch * Bm : R(0);
}

// ---------------------------------------------------------------------------
// Limiters and reconstruction (Sec. 3.2), on undivided differences.
// ---------------------------------------------------------------------------

// minmod: the argument of smaller magnitude when both share a sign, else 0.
// In FP32 it is the median of (a, b, 0), one v_med3_f32; in FP64 selects.
// The two agree up to the sign of a zero result, except where the sign
// product a * b of the select form would underflow (|a b| below the FP32
// normal range): there the select form gives 0 and the median the exact
// smaller argument.
template <typename R> __device__ __forceinline__ R minmod(R a, R b)
{
    if constexpr (sizeof(R) == 4) {
        return __builtin_amdgcn_fmed3f(a, b, 0.0f);
    } else {
        R m = (fabs(a) < fabs(b)) ? a : b;
        return (a * b > R(0)) ? m : R(0);
    }
}

// monotonised central limiter minmod((dp + dm)/2, 2 minmod(dp, dm)): for
// differences of one sign, that sign times min(|dp + dm|/2, 2|dp|, 2|dm|).
// FP32 nests the medians (minmod of three = minmod(x, minmod(y, z)), and
// doubling is exact): two v_med3_f32 in place of the sign test and selects.
template <typename R> __device__ __forceinline__ R lim_mc(R dp, R dm)
{
    R c = R(0.5) * (dp + dm);
    if constexpr (sizeof(R) == 4) {
        return __builtin_amdgcn_fmed3f(c, 2.0f * __builtin_amdgcn_fmed3f(dp, dm, 0.0f), 0.0f);
    } else {
        R m = fmin(fmin(fabs(c), R(2) * fabs(dp)), R(2) * fabs(dm));
        return (dp * dm > R(0)) ? copysign(m, c) : R(0);
    }
}

// lim_mc(dp, dm) / 2 in FP32: the same medians on halved arguments
__device__ __forceinline__ float lim_mc_half(float dp, float dm)
{
    return __builtin_amdgcn_fmed3f(0.25f * (dp + dm), __builtin_amdgcn_fmed3f(dp, dm, 0.0f), 0.0f);
}

template <typename R> __device__ __forceinline__ R limiter(int lim, R dp, R dm)
{
    R pr = dp * dm;
    switch (lim) {
    case LIM_MINMOD: return minmod(dp, dm);
    case LIM_VANLEER: return pr > R(0) ? R(2) * pr / (dp + dm) : R(0);
    case LIM_VANALBADA: return pr > R(0) ? pr * (dp + dm) / (dp * dp + dm * dm) : R(0);
    default: return lim_mc(dp, dm);
    }
}

// Interface offsets dm = w_- - w_0, dp = w_+ - w_0 from the differences
// d[l] = w_{l+1} - w_l, l = -2..1 stored at d[0..3] (linear / WENO3 use d[1],
// d[2] only).
template <int RK, typename R>
__device__ __forceinline__ void recon_offsets(const R *d, int lim, R dxr, R &dm, R &dp)
{
    if constexpr (RK == RK_LIN) {
        R s = limiter(lim, d[2], d[1]);
        dp = R(0.5) * s;
        dm = -dp;
    } else if constexpr (RK == RK_PPM) {
        R P, M;
        if constexpr (sizeof(R) == 4) {
            // half slopes lim_mc / 2 = med3((dp + dm)/4, minmod(dp, dm), 0) and
            // 1/3 in place of 1/6: power-of-two scalings, so the same bits
            R s0 = lim_mc_half(d[2], d[1]);
            R sp = lim_mc_half(d[3], d[2]);
            R sm = lim_mc_half(d[1], d[0]);
            P = 0.5f * d[2] - (sp - s0) * (1.0f / 3.0f);   // Eq. ppm1, w_+ - w_0
            M = -0.5f * d[1] + (sm - s0) * (1.0f / 3.0f);  // w_- - w_0
        } else {
            R s0 = lim_mc(d[2], d[1]);
            R sp = lim_mc(d[3], d[2]);
            R sm = lim_mc(d[1], d[0]);
            P = R(0.5) * d[2] - (sp - s0) * R(1.0 / 6.0);   // Eq. ppm1, w_+ - w_0
            M = -R(0.5) * d[1] + (sm - s0) * R(1.0 / 6.0);  // w_- - w_0
        }
        if constexpr (sizeof(R) == 4) {
            // Eq. ppm_parabolic_lim as medians: where P and M share a sign, -2M
            // and -2P have the other one and the median is 0; otherwise it is
            // the smaller in magnitude of P and -2M (of M and -2P)
            dp = __builtin_amdgcn_fmed3f(P, -2.0f * M, 0.0f);
            dm = __builtin_amdgcn_fmed3f(M, -2.0f * P, 0.0f);
        } else if (P * M > R(0)) {                        // Eq. ppm_parabolic_lim
            dp = R(0);
            dm = R(0);
        } else {
            dp = (fabs(P) >= R(2) * fabs(M)) ? R(-2) * M : P;
            dm = (fabs(M) >= R(2) * fabs(P)) ? R(-2) * P : M;
        }
    } else {
        R a = d[2], c = d[1];                              // Delta w_{+1/2}, Delta w_{-1/2}
        R num = sq(a - c);
        R ap = R(1) + num / (dxr * dxr + a * a);            // Eq. WENO3a
        R am = R(1) + num / (dxr * dxr + c * c);
        dp = (ap * a + R(0.5) * am * c) / (R(2) * ap + am); // Eq. WENO3
        dm = -(am * c + R(0.5) * ap * a) / (R(2) * am + ap);
    }
}

// Upwind tracing of one wave (Eq. wnorm_predp/m) in offset form: returns
// w*_{+-} - w_0.
template <typename R>
__device__ __forceinline__ void trace(int wref, R dm, R dp, R nu, R numax, R numin, R &sm, R &sp)
{
    R dw = dp - dm, d2 = dp + dm;
    // upwind weights (1 + sgn nu)/2 and (1 - sgn nu)/2
    R bp = (nu > R(0)) ? R(1) : ((nu < R(0)) ? R(0) : R(0.5));
    R bm = R(1) - bp;
    R tp = dp - R(0.5) * nu * (dw + d2 * (R(3) - R(2) * nu));
    R tm = dm - R(0.5) * nu * (dw - d2 * (R(3) + R(2) * nu));
    R rp, rm;
    if (wref == WREF_CELL) {
        rp = R(0);
        rm = R(0);
    } else if (wref == WREF_CW84) {
        rp = dp - R(0.5) * numax * (dw + d2 * (R(3) - R(2) * numax));
        rm = dm - R(0.5) * numin * (dw - d2 * (R(3) + R(2) * numin));
    } else {
        rp = dp;
        rm = dm;
    }
    sp = rp + bp * (tp - rp);
    sm = rm + bm * (tm - rm);
}

// ---------------------------------------------------------------------------
// Characteristic normal predictor (Sec. 3.2) with closed-form eigenvectors
// of the 7-wave primitive MHD system normalised after Roe & Balsara (1996).
// ---------------------------------------------------------------------------

template <typename R> struct Eigen {
    R rho, srho, a, a2, cf, cs, ca, af, as, by, bz, s;
    R X, Y, Z;  // 1/(2N), 1/(2 a sqrt(rho)), 1/(2 rho a^2), N = af^2 cf^2 + as^2 cs^2
    R isrho, ia2;  // 1/sqrt(rho), 1/a^2
};

template <int D, typename R> __device__ __forceinline__ void eigen_setup(const R *V, R gam, Eigen<R> &e)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    // reciprocal roots carry the divisions: 1/sqrt(rho), 1/a, 1/c_f
    R rho = V[RHO];
    R isr = rsq(rho);
    R ir = isr * isr;
    R Bn = V[BX1 + n], Bt = V[BX1 + t], Bb = V[BX1 + b];
    R a2 = gam * V[PRS] * ir;
    R bn2 = Bn * Bn * ir;
    R Bt2 = Bt * Bt + Bb * Bb;
    R bt2 = Bt2 * ir;
    R b2 = bn2 + bt2;
    R dab = a2 - b2;
    R root = sqrt(dab * dab + R(4) * a2 * bt2);  // c_f^2 - c_s^2, exact for b_t = 0
    R cf2 = R(0.5) * (a2 + b2 + root);
    R ia = rsq(a2), icf = rsq(cf2);
    e.rho = rho;
    e.srho = rho * isr;
    e.isrho = isr;
    e.a2 = a2;
    e.ia2 = ia * ia;
    e.a = a2 * ia;
    e.cf = cf2 * icf;
    e.ca = fabs(Bn) * isr;
    e.cs = e.a * e.ca * icf;                     // c_f c_s = a c_a
    R cs2 = e.cs * e.cs;
    if (root > R(0)) {
        R ir2 = R(0.5) / root;
        R af2 = (root + dab) * ir2, as2 = (root - dab) * ir2;
        e.af = sqrt(af2 > R(0) ? af2 : R(0));
        e.as = sqrt(as2 > R(0) ? as2 : R(0));
    } else {
        e.af = R(1);
        e.as = R(0);
    }
    if (Bt2 <= R(1e-12) * (Bt2 + Bn * Bn)) {
        e.by = R(0.70710678118654752440);
        e.bz = R(0.70710678118654752440);
    } else {
        R ib = rsq(Bt2);
        e.by = Bt * ib;
        e.bz = Bb * ib;
    }
    e.s = sgn1(Bn);
    R N = e.af * e.af * cf2 + e.as * e.as * cs2;
    e.X = R(0.5) / N;
    e.Y = R(0.5) * ia * isr;
    e.Z = R(0.5) * ir * e.ia2;
}

// project a primitive difference dq onto the 7 left eigenvectors
template <int D, typename R> __device__ __forceinline__ void project(const Eigen<R> &e, const R *dq, R *w)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R u = dq[MX1 + n];
    R vpa = e.by * dq[MX1 + t] + e.bz * dq[MX1 + b];
    R vpe = -e.bz * dq[MX1 + t] + e.by * dq[MX1 + b];
    R Bpa = e.by * dq[BX1 + t] + e.bz * dq[BX1 + b];
    R Bpe = -e.bz * dq[BX1 + t] + e.by * dq[BX1 + b];
    R dp = dq[PRS];
    R fu = e.X * e.af * e.cf * u, su = e.X * e.as * e.cs * u;
    R fv = e.X * e.s * e.as * e.cs * vpa, sv = e.X * e.s * e.af * e.cf * vpa;
    R fB = e.Y * e.as * Bpa, sB = e.Y * e.af * Bpa;
    R fp = e.Z * e.af * dp, sp = e.Z * e.as * dp;
    w[0] = -fu + fv + fB + fp;  // v - c_f
    w[6] = fu - fv + fB + fp;   // v + c_f
    w[2] = -su - sv - sB + sp;  // v - c_s
    w[4] = su + sv - sB + sp;   // v + c_s
    R hv = R(0.5) * vpe, hB = R(0.5) * e.s * Bpe * e.isrho;
    w[1] = hv + hB;             // v - c_a
    w[5] = hv - hB;             // v + c_a
    w[3] = dq[RHO] - dp * e.ia2; // entropy
}

// dV = sum_k c_k r_k (right eigenvectors), added to V
template <int D, typename R> __device__ __forceinline__ void recombine(const Eigen<R> &e, const R *c, R *V)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R f = c[0] + c[6], sl = c[2] + c[4];
    V[RHO] += e.rho * (e.af * f + e.as * sl) + c[3];
    V[MX1 + n] += e.af * e.cf * (c[6] - c[0]) + e.as * e.cs * (c[4] - c[2]);
    R vpa = e.s * (e.as * e.cs * (c[0] - c[6]) + e.af * e.cf * (c[4] - c[2]));
    R vpe = c[1] + c[5];
    R asr = e.a * e.srho;
    R Bpa = asr * (e.as * f - e.af * sl);
    R Bpe = e.s * e.srho * (c[1] - c[5]);
    V[MX1 + t] += e.by * vpa - e.bz * vpe;
    V[MX1 + b] += e.bz * vpa + e.by * vpe;
    V[BX1 + t] += e.by * Bpa - e.bz * Bpe;
    V[BX1 + b] += e.bz * Bpa + e.by * Bpe;
    V[PRS] += e.rho * e.a2 * (e.af * f + e.as * sl);
}

// Roe's linearised solver for MHD (Sec. 3.1 lists it) for states sharing
// B_n: F = (F_L + F_R)/2 - |A| (U_R - U_L)/2 with F_R - F_L = A (U_R - U_L)
// exactly.  Averages with weights sqrt(rho): v~ and H~ = (E + p_t)/rho; the
// transverse field with the weights swapped, rho^ = sqrt(rho_L rho_R) and
// X = |dB_t|^2 / (2 (sqrt(rho_L) + sqrt(rho_R))^2) (Cargo & Gallice 1997).
// In the differences dW = (drho, (dm - v~ drho)/rho^, dB_t, dp) with
//   dp = (gamma - 1)(dE - v~.dm + v~^2 drho/2 - B~_t.dB_t) - (gamma - 2) X drho
// A acts as the primitive-variable Jacobian of the state (rho^, v~, B_n,
// B~_t, p^), gamma p^ = rho^ a~^2, a~^2 = (gamma - 1)(H~ - v~^2/2 - B~^2/rho^)
// - (gamma - 2) X, so |A| dU is the closed-form eigen-decomposition of that
// state (project / recombine) weighted by |lambda| and mapped back to
// conserved differences.  No entropy fix.  Signal speed: the largest fast
// |lambda| of the average and of both states.
template <int D, typename R>
__device__ __forceinline__ void roe(const R *VL, const R *VR, R *F, R &smax, R gam, R ch, int glm)
{
    constexpr int n = Ax<D>::n, t = Ax<D>::t, b = Ax<D>::b;
    R UL[NV], UR[NV], FL[NV], FR[NV];
    phys_flux<D, PHYS_MHD>(VL, UL, FL, gam, ch, glm);
    phys_flux<D, PHYS_MHD>(VR, UR, FR, gam, ch, glm);
    const R gm1 = gam - R(1), gm2 = gam - R(2);
    const R sL = sqrt(VL[RHO]), sR = sqrt(VR[RHO]);
    const R is = R(1) / (sL + sR);
    const R wL = sL * is, wR = sR * is;
    const R rh = sL * sR, irh = R(1) / rh;
    R Vh[NV];
    Vh[RHO] = rh;
    R q2 = R(0);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        Vh[MX1 + k] = wL * VL[MX1 + k] + wR * VR[MX1 + k];
        q2 += Vh[MX1 + k] * Vh[MX1 + k];
    }
    const R ptL = VL[PRS] + R(0.5) * (sq(VL[BX1]) + sq(VL[BX2]) + sq(VL[BX3]));
    const R ptR = VR[PRS] + R(0.5) * (sq(VR[BX1]) + sq(VR[BX2]) + sq(VR[BX3]));
    const R H = wL * (UL[ENG] + ptL) / VL[RHO] + wR * (UR[ENG] + ptR) / VR[RHO];
    const R Bn = VL[BX1 + n];
    const R Bt = wR * VL[BX1 + t] + wL * VR[BX1 + t];
    const R Bb = wR * VL[BX1 + b] + wL * VR[BX1 + b];
    const R dBt = VR[BX1 + t] - VL[BX1 + t], dBb = VR[BX1 + b] - VL[BX1 + b];
    const R X = R(0.5) * (dBt * dBt + dBb * dBb) * is * is;
    const R a2 = gm1 * (H - R(0.5) * q2 - (Bn * Bn + Bt * Bt + Bb * Bb) * irh) - gm2 * X;
    Vh[BX1 + n] = Bn;
    Vh[BX1 + t] = Bt;
    Vh[BX1 + b] = Bb;
    Vh[PRS] = rh * a2 / gam;
    Vh[PSI] = R(0);
    Eigen<R> e;
    eigen_setup<D>(Vh, gam, e);

    // conserved differences -> dW
    R dq[NV];
    dq[RHO] = UR[RHO] - UL[RHO];
    R vdm = R(0);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const R dm = UR[MX1 + k] - UL[MX1 + k];
        dq[MX1 + k] = (dm - Vh[MX1 + k] * dq[RHO]) * irh;
        vdm += Vh[MX1 + k] * dm;
    }
    dq[BX1 + n] = R(0);
    dq[BX1 + t] = dBt;
    dq[BX1 + b] = dBb;
    dq[PSI] = R(0);
    dq[PRS] = gm1 * (UR[ENG] - UL[ENG] - vdm + R(0.5) * q2 * dq[RHO] - Bt * dBt - Bb * dBb) - gm2 * X * dq[RHO];

    // sum_k |lambda_k| (l_k . dW) r_k
    R w[7];
    project<D>(e, dq, w);
    const R u = Vh[MX1 + n];
    R c[7];
    c[0] = fabs(u - e.cf) * w[0];
    c[1] = fabs(u - e.ca) * w[1];
    c[2] = fabs(u - e.cs) * w[2];
    c[3] = fabs(u) * w[3];
    c[4] = fabs(u + e.cs) * w[4];
    c[5] = fabs(u + e.ca) * w[5];
    c[6] = fabs(u + e.cf) * w[6];
    R Dw[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) Dw[q] = R(0);
    recombine<D>(e, c, Dw);

    // dW -> conserved differences, then the flux
    R Du[NV];
    Du[RHO] = Dw[RHO];
    R vdv = R(0);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        Du[MX1 + k] = Vh[MX1 + k] * Dw[RHO] + rh * Dw[MX1 + k];
        vdv += Vh[MX1 + k] * Dw[MX1 + k];
    }
    Du[BX1 + n] = R(0);
    Du[BX1 + t] = Dw[BX1 + t];
    Du[BX1 + b] = Dw[BX1 + b];
    Du[PSI] = R(0);
    Du[ENG] = (Dw[PRS] + gm2 * X * Dw[RHO]) / gm1 + Bt * Dw[BX1 + t] + Bb * Dw[BX1 + b] + R(0.5) * q2 * Dw[RHO] +
              rh * vdv;
#pragma unroll
    for (int q = 0; q < NV; q++) F[q] = R(0.5) * (FL[q] + FR[q]) - R(0.5) * Du[q];
    const R cfL = cfast_mhd<D>(VL, gam), cfR = cfast_mhd<D>(VR, gam);
    const R uL = VL[MX1 + n], uR = VR[MX1 + n];
    smax = fmax(fmax(fabs(u - e.cf), fabs(u + e.cf)),
                fmax(fmax(fabs(uL - cfL), fabs(uL + cfL)), fmax(fabs(uR - cfR), fabs(uR + cfR))));
}

// Characteristic predictor for cell 0 of the primitive stencil Vs[l+2]
// (l = -2..2; linear and WENO3 read l = -1..1).  Outputs V*_- and V*_+.
template <int D, int RK, typename R>
__device__ __forceinline__ void predict_char(const R (*Vs)[NV], const KOpts &o, R gam, R dtdx, R dxr, R ch, R *Vm,
                                             R *Vp, int lim)
{
    const R *V0 = Vs[2];
    Eigen<R> e;
    eigen_setup<D>(V0, gam, e);
    constexpr int L0 = (RK == RK_PPM) ? 0 : 1;
    constexpr int L1 = (RK == RK_PPM) ? 4 : 3;
    // characteristic differences d[k][l] = l_k . (V_{l+1} - V_l)
    R d[7][4];
    R dh[2][4];
#pragma unroll
    for (int l = L0; l < L1; l++) {
        R dq[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) dq[q] = Vs[l + 1][q] - Vs[l][q];
        R w[7];
        project<D>(e, dq, w);
#pragma unroll
        for (int k = 0; k < 7; k++) d[k][l] = w[k];
        if (o.glm) {
            R ih = R(0.5) / ch;
            dh[0][l] = (ch * dq[BX1 + D] - dq[PSI]) * ih;
            dh[1][l] = (ch * dq[BX1 + D] + dq[PSI]) * ih;
        } else {
            dh[0][l] = dq[BX1 + D];
            dh[1][l] = R(0);
        }
    }
    R vn = V0[MX1 + D];
    R nu[7] = { (vn - e.cf) * dtdx, (vn - e.ca) * dtdx, (vn - e.cs) * dtdx, vn * dtdx,
                (vn + e.cs) * dtdx, (vn + e.ca) * dtdx, (vn + e.cf) * dtdx };
    R nuh = ch * dtdx;
    R numax = R(0), numin = R(0);
    if (o.wref == WREF_CW84) {
#pragma unroll
        for (int k = 0; k < 7; k++) {
            numax = fmax(numax, nu[k]);
            numin = fmin(numin, nu[k]);
        }
        if (o.glm) {
            numax = fmax(numax, nuh);
            numin = fmin(numin, -nuh);
        }
    }
    R cm[7], cp[7];
#pragma unroll
    for (int k = 0; k < 7; k++) {
        R dm, dp;
        recon_offsets<RK>(d[k], lim, dxr, dm, dp);
        trace(o.wref, dm, dp, nu[k], numax, numin, cm[k], cp[k]);
    }
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Vm[q] = V0[q];
        Vp[q] = V0[q];
    }
    recombine<D>(e, cm, Vm);
    recombine<D>(e, cp, Vp);

    // (B_n, psi): GLM pair with speeds -+c_h, or plain reconstruction of B_n
    R dBn, dpsi;
    if (o.glm) {
        R hm[2], hp[2], tm[2], tp[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            recon_offsets<RK>(dh[k], lim, dxr, hm[k], hp[k]);
            trace(o.wref, hm[k], hp[k], k ? nuh : -nuh, numax, numin, tm[k], tp[k]);
        }
        dBn = (hp[0] + hp[1]) - (hm[0] + hm[1]);
        dpsi = ch * ((hp[1] - hp[0]) - (hm[1] - hm[0]));
        Vm[BX1 + D] += tm[0] + tm[1];
        Vp[BX1 + D] += tp[0] + tp[1];
        Vm[PSI] += ch * (tm[1] - tm[0]);
        Vp[PSI] += ch * (tp[1] - tp[0]);
    } else {
        R bm, bp;
        recon_offsets<RK>(dh[0], lim, dxr, bm, bp);
        dBn = bp - bm;
        dpsi = R(0);
        Vm[BX1 + D] += bm;
        Vp[BX1 + D] += bp;
    }
    // terms that the 7-wave primitive system omits: d(B_n)/dn and d(psi)/dn
    constexpr int t = Ax<D>::t, b = Ax<D>::b;
    R h = R(0.5) * dtdx;
    R gB = h * dBn, gP = h * dpsi;
    R ir = e.isrho * e.isrho;
    R vB = V0[MX1] * V0[BX1] + V0[MX2] * V0[BX2] + V0[MX3] * V0[BX3];
    R src[NV] = { R(0) };
    src[MX1 + D] = gB * V0[BX1 + D] * ir;
    src[MX1 + t] = gB * V0[BX1 + t] * ir;
    src[MX1 + b] = gB * V0[BX1 + b] * ir;
    src[BX1 + t] = gB * V0[MX1 + t];
    src[BX1 + b] = gB * V0[MX1 + b];
    src[PRS] = gB * (R(1) - gam) * vB + gP * (gam - R(1)) * V0[BX1 + D];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Vm[q] += src[q];
        Vp[q] += src[q];
    }
}

// MUSCL-Hancock primitive predictor (Sec. 3.3, Eq. MUSCL-Hancock, beta = 1):
// limited slopes of the primitive variables, a conservative half step of
// the cell with the physical fluxes of its two interface values, and
// V*_{+-} = V(U*) +- dV/2.  A superluminal reconstruction (RMHD) drops the
// slopes of the cell; a failed V(U*) falls back to V_i.  Returns failure bits.
template <int D, int PHYS, typename R>
__device__ __forceinline__ int predict_mh(const R (*Vs)[NV], const R *U0, const KOpts &o, R gam, R dtdx, R ch, R *Vm,
                                          R *Vp, int lim)
{
    int fl = 0;
    R dV[NV], Vlo[NV], Vhi[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) {
        dV[q] = limiter(lim, Vs[3][q] - Vs[2][q], Vs[2][q] - Vs[1][q]);
        Vlo[q] = Vs[2][q] - R(0.5) * dV[q];
        Vhi[q] = Vs[2][q] + R(0.5) * dV[q];
    }
    if constexpr (PHYS != PHYS_MHD) {
        R v2l = sq(Vlo[MX1]) + sq(Vlo[MX2]) + sq(Vlo[MX3]);
        R v2h = sq(Vhi[MX1]) + sq(Vhi[MX2]) + sq(Vhi[MX3]);
        if (!(v2l < R(1)) || !(v2h < R(1))) {
            fl |= F_VEL;
#pragma unroll
            for (int q = 0; q < NV; q++) {
                dV[q] = R(0);
                Vlo[q] = Vs[2][q];
                Vhi[q] = Vs[2][q];
            }
        }
    }
    R Ut[NV], Flo[NV], Fhi[NV], Us[NV], Vh[NV];
    phys_flux<D, PHYS>(Vlo, Ut, Flo, gam, ch, o.glm);
    phys_flux<D, PHYS>(Vhi, Ut, Fhi, gam, ch, o.glm);
#pragma unroll
    for (int q = 0; q < NV; q++) Us[q] = U0[q] - R(0.5) * dtdx * (Fhi[q] - Flo[q]);
    // the half step starts the inversion from the cell's own W
    int f2 = c2p<PHYS>(Us, Vh, gam, w_guess<PHYS>(Vs[2], gam));
    if (f2) {
        fl |= f2;
#pragma unroll
        for (int q = 0; q < NV; q++) Vh[q] = Vs[2][q];
    }
#pragma unroll
    for (int q = 0; q < NV; q++) {
        Vm[q] = Vh[q] - R(0.5) * dV[q];
        Vp[q] = Vh[q] + R(0.5) * dV[q];
    }
    return fl;
}

}  // namespace ctu
