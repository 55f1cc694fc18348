/*
 * ctu_oracle.c -- plain FP64 CPU oracle for the single-patch CTU-GLM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or helper with the HIP library under paper_1110_0740_amd/.
 *
 * It follows Mignone et al., "The PLUTO code for adaptive mesh computations
 * in astrophysical fluid dynamics" (ApJS 2012):
 *   Sec. 2.1  ideal / non-ideal MHD equations (Eq. mhd, visc_tens, tc_flux)
 *   Sec. 2.2  relativistic MHD (Eq. rmhd, gammaEos, TMEos)
 *   Sec. 3    GLM cleaning (Eq. glm2x2)
 *   Sec. 3.1  unsplit CTU update (Eq. update, incrementop_hyp/par, ctu_flux,
 *             transv, Ca, dt_cool); the listed solvers Rusanov, HLL, HLLC,
 *             HLLD and Roe; the predictor-flux corner coupling for Pi = 0
 *   App. B    shock-adaptive hybrid (HLL and MinMod near flagged zones)
 *   Sec. 3.2  characteristic normal predictors (Eq. char_var, wnorm_predp/m,
 *             ppm1, MClim, minmod, ppm_parabolic_lim, WENO3, WENO3a, Linear,
 *             harmonic_lim, vanalbada_lim)
 *   Sec. 3.3  MUSCL-Hancock primitive predictor (Eq. MUSCL-Hancock)
 *   App. A    saturated conduction flux (Eq. sat_eq, sat_flux)
 * and, where the paper defers to published methods, their textbook form:
 *   HLLD (Miyoshi & Kusano 2005), HLL (Harten, Lax & van Leer 1983),
 *   normalized MHD eigenvectors (Roe & Balsara 1996), GLM Riemann subsystem
 *   (Dedner et al. 2002), MHD HLLC (Li 2005), MHD Roe averages (Cargo &
 *   Gallice 1997), relativistic HLLC (Mignone & Bodo 2006) and HLLD
 *   (Mignone, Ugliano & Bodo 2009), each re-derived from its jump conditions
 *   as its comment states.
 *
 * Plain scalar loops, one box at a time, full-size temporaries, no tiling and
 * no fusion.  The cell and face loops of a stage are independent, so they
 * are shared among OpenMP threads (orc_set_threads) with the failure counts
 * summed and the CFL rate and |dp/p| maxima reduced; every value is computed
 * by the same expression in the same order whatever the thread count, so
 * the results are bitwise those of one thread.  Left eigenvectors are obtained by numerically inverting the
 * right-eigenvector matrix; the relativistic conserved-to-primitive map is
 * solved by bracketing bisection.  Both are slow and obviously correct.
 *
 * Array layout: every cell field is SoA  q[v][k][j][i]  over the ghosted box
 * (i fastest), extents NX=nx+2g, NY=ny+2g, NZ=nz+2g (NZ=1 when dim==2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NVAR 9
enum { RHO = 0, MX1 = 1, MX2 = 2, MX3 = 3, ENG = 4, BX1 = 5, BX2 = 6, BX3 = 7, PSI = 8 };
#define PRS ENG /* primitive pressure sits where the conserved energy sits */

enum { PHYS_MHD = 0, PHYS_RMHD = 1 };
enum { REC_LIN_MC = 0, REC_LIN_MINMOD = 1, REC_LIN_VANLEER = 2, REC_LIN_VANALBADA = 3,
       REC_PPM = 4, REC_WENO3 = 5 };
enum { PRED_CHAR = 0, PRED_MH = 1 };
enum { WREF_FACE = 0, WREF_CELL = 1, WREF_CW84 = 2 };
enum { RS_HLLD = 0, RS_HLL = 1, RS_RUSANOV = 2, RS_HLLC = 3, RS_ROE = 4 };
enum { CORNER_TN = 0, CORNER_MT = 1 };
enum { FAIL_RHO = 0, FAIL_PRS = 1, FAIL_NEWTON = 2, FAIL_VEL = 3, FAIL_NAN = 4, NFAIL = 5 };

#define PARAB_VISC 1u
#define PARAB_RES 2u
#define PARAB_TC 4u

typedef struct {
    int dim, physics, recon, predictor, wref, riemann;
    double gamma;
    double dx[3];
    int glm;
    double glm_alpha;
    unsigned parabolic_mask;
    double nu, eta, kappa_par, kappa_perp, tc_phi;
    int cooling;
    double cool_beta, T_floor;
    int hyperbolic_off;
    double shock_eps; /* App. B shock detection threshold eps_q; 0 = off */
    int eos;          /* RMHD equation of state: EOS_IDEAL (Eq. gammaEos) or EOS_TM (Eq. TMEos) */
    int exact_speeds; /* RMHD signal speeds: 0 = isotropic bound, 1 = fast roots of the quartic */
    int corner;       /* CORNER_TN (Eq. transv with t^n fluxes) or CORNER_MT (predictor fluxes) */
} orc_opts;

enum { EOS_IDEAL = 0, EOS_TM = 1 };

/* Stage boundaries of orc_step, where the op-counting build of the oracle
 * (oracle/opcount.cpp) reads its operation counters; nothing otherwise. */
#ifndef ORC_STAGE
#define ORC_STAGE(k) ((void)0)
#endif
/* Around the numerical inversion of the right-eigenvector matrix, which
 * stands in for the closed-form left eigenvectors, and around the
 * relativistic conserved-to-primitive root finding, done here by bisection
 * to machine precision: the op-counting build books their operations apart
 * from the rest (ORC_SIDE_* for the former, ORC_ROOT_* for the latter). */
#ifndef ORC_SIDE_BEGIN
#define ORC_SIDE_BEGIN ((void)0)
#define ORC_SIDE_END ((void)0)
#endif
#ifndef ORC_ROOT_BEGIN
#define ORC_ROOT_BEGIN ((void)0)
#define ORC_ROOT_END ((void)0)
#endif

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */

static double sgn0(double a) { return (a > 0.0) - (a < 0.0); } /* sign(0) = 0 */
static double sgn1(double a) { return a < 0.0 ? -1.0 : 1.0; }  /* sign(0) = +1 */

/* Component indices of (normal, transverse, binormal) for direction d; the
 * cyclic order keeps the triad right-handed. */
static void dir_axes(int d, int *n, int *t, int *b)
{
    *n = d;
    *t = (d + 1) % 3;
    *b = (d + 2) % 3;
}

/* ------------------------------------------------------------------------ */
/* Ideal MHD: Eq. mhd with the ideal-gas closure (Sec. 2.1)                  */
/* ------------------------------------------------------------------------ */

static void mhd_prim2cons(const orc_opts *o, const double *V, double *U)
{
    double v2 = V[MX1] * V[MX1] + V[MX2] * V[MX2] + V[MX3] * V[MX3];
    double b2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    U[RHO] = V[RHO];
    U[MX1] = V[RHO] * V[MX1];
    U[MX2] = V[RHO] * V[MX2];
    U[MX3] = V[RHO] * V[MX3];
    U[ENG] = V[PRS] / (o->gamma - 1.0) + 0.5 * V[RHO] * v2 + 0.5 * b2;
    U[BX1] = V[BX1];
    U[BX2] = V[BX2];
    U[BX3] = V[BX3];
    U[PSI] = V[PSI];
}

static void mhd_cons2prim(const orc_opts *o, const double *U, double *V, int *fails)
{
    double rho = U[RHO];
    V[RHO] = rho;
    V[MX1] = U[MX1] / rho;
    V[MX2] = U[MX2] / rho;
    V[MX3] = U[MX3] / rho;
    V[BX1] = U[BX1];
    V[BX2] = U[BX2];
    V[BX3] = U[BX3];
    V[PSI] = U[PSI];
    double v2 = V[MX1] * V[MX1] + V[MX2] * V[MX2] + V[MX3] * V[MX3];
    double b2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    V[PRS] = (o->gamma - 1.0) * (U[ENG] - 0.5 * rho * v2 - 0.5 * b2);
    if (fails) {
        if (!(rho > 0.0)) fails[FAIL_RHO]++;
        if (!(V[PRS] > 0.0)) fails[FAIL_PRS]++;
        for (int v = 0; v < NVAR; v++)
            if (isnan(V[v])) { fails[FAIL_NAN]++; break; }
    }
}

/* Fast magnetosonic speed along direction d. */
static double mhd_fast_speed(const orc_opts *o, const double *V, int d)
{
    double a2 = o->gamma * V[PRS] / V[RHO];
    double b2 = (V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3]) / V[RHO];
    double bn2 = V[BX1 + d] * V[BX1 + d] / V[RHO];
    double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * bn2;
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (s + sqrt(disc)));
}

/* Hyperbolic flux along d (rows of Eq. mhd) without the GLM rows; the GLM
 * rows (B_n, psi) are filled by the caller. */
static void mhd_flux(const orc_opts *o, const double *V, const double *U, int d, double *F)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double vn = V[MX1 + n];
    double Bn = V[BX1 + n];
    double b2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    double vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    double pt = V[PRS] + 0.5 * b2;
    F[RHO] = U[RHO] * vn;
    F[MX1 + n] = U[MX1 + n] * vn - Bn * Bn + pt;
    F[MX1 + t] = U[MX1 + t] * vn - Bn * V[BX1 + t];
    F[MX1 + b] = U[MX1 + b] * vn - Bn * V[BX1 + b];
    F[ENG] = (U[ENG] + pt) * vn - vB * Bn;
    F[BX1 + n] = 0.0;
    F[BX1 + t] = vn * V[BX1 + t] - Bn * V[MX1 + t];
    F[BX1 + b] = vn * V[BX1 + b] - Bn * V[MX1 + b];
    F[PSI] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Relativistic MHD: Eq. rmhd with the ideal EOS Eq. gammaEos or the TM EOS  */
/* Eq. TMEos (Sec. 2.2)                                                      */
/* ------------------------------------------------------------------------ */

/* Gas enthalpy w(rho, p). */
static double rmhd_enthalpy(const orc_opts *o, double rho, double p)
{
    if (o->eos == EOS_TM) return 2.5 * p + sqrt(2.25 * p * p + rho * rho);
    return rho + o->gamma * p / (o->gamma - 1.0);
}

/* Pressure from (rho, w), the inverse of rmhd_enthalpy.  TM: squaring
 * w - 5p/2 = sqrt(9p^2/4 + rho^2) gives 4p^2 - 5wp + w^2 - rho^2 = 0, whose
 * root with w - 5p/2 >= 0 is the smaller one. */
static double rmhd_pressure(const orc_opts *o, double rho, double w)
{
    if (o->eos == EOS_TM) return (5.0 * w - sqrt(9.0 * w * w + 16.0 * rho * rho)) / 8.0;
    return (o->gamma - 1.0) / o->gamma * (w - rho);
}

/* Sound speed squared c_s^2 = (dp/drho)_s rho / w (the adiabat has
 * de = (w/rho) drho for the energy density e = w - p).  Ideal: Gamma p / w.
 * TM: differentiating e = 3p/2 + sqrt(9p^2/4 + rho^2) along the adiabat and
 * eliminating rho^2 = w^2 - 5wp + 4p^2 gives p (5w - 8p) / (3 w (w - p)). */
static double rmhd_cs2(const orc_opts *o, double p, double w)
{
    if (o->eos == EOS_TM) return p * (5.0 * w - 8.0 * p) / (3.0 * w * (w - p));
    return o->gamma * p / w;
}

static void rmhd_prim2cons(const orc_opts *o, const double *V, double *U)
{
    double v2 = V[MX1] * V[MX1] + V[MX2] * V[MX2] + V[MX3] * V[MX3];
    double B2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    double vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    double lor2 = 1.0 / (1.0 - v2);
    double lor = sqrt(lor2);
    double w = rmhd_enthalpy(o, V[RHO], V[PRS]);
    double E2 = B2 * v2 - vB * vB; /* |v x B|^2 */
    U[RHO] = V[RHO] * lor;
    /* m = w gamma^2 v + E x B, with E = -v x B  =>  E x B = B^2 v - (v.B) B */
    for (int c = 0; c < 3; c++) U[MX1 + c] = (w * lor2 + B2) * V[MX1 + c] - vB * V[BX1 + c];
    U[ENG] = w * lor2 - V[PRS] + 0.5 * (B2 + E2) - U[RHO];
    U[BX1] = V[BX1];
    U[BX2] = V[BX2];
    U[BX3] = V[BX3];
    U[PSI] = V[PSI];
}

/* Velocity squared and pressure as functions of W = w gamma^2 for fixed
 * conserved variables (the map that the inversion must undo). */
typedef struct {
    double D, E, m2, S, B2;
    const orc_opts *o;
} rmhd_inv;

static double rmhd_v2_of_W(const rmhd_inv *q, double W)
{
    double sw = q->S / W;
    double num = q->m2 + sw * sw * (2.0 * W + q->B2);
    double den = (W + q->B2) * (W + q->B2);
    return num / den;
}

/* Residual of the energy definition: f(W) = W - p + B^2/2 + (v^2 B^2 - S^2/W^2)/2 - D - E. */
static double rmhd_resid(const rmhd_inv *q, double W, double *p_out, double *v2_out)
{
    double v2 = rmhd_v2_of_W(q, W);
    double sq = sqrt(1.0 - v2);
    /* w = W / gamma^2, rho = D / gamma */
    double p = rmhd_pressure(q->o, q->D * sq, W * (1.0 - v2));
    if (p_out) *p_out = p;
    if (v2_out) *v2_out = v2;
    double sw = q->S / W;
    return W - p + 0.5 * q->B2 + 0.5 * (v2 * q->B2 - sw * sw) - q->D - q->E;
}

/* Conserved -> primitive for RMHD by bisection on W.  v^2(W) decreases
 * monotonically, so the physical branch is W > W*, with v^2(W*) = 1; the
 * root of f is bracketed on (W*, W_hi] and bisected to machine precision. */
static int rmhd_cons2prim(const orc_opts *o, const double *U, double *V, int *fails)
{
    rmhd_inv q;
    q.o = o;
    q.D = U[RHO];
    q.E = U[ENG];
    q.m2 = U[MX1] * U[MX1] + U[MX2] * U[MX2] + U[MX3] * U[MX3];
    q.S = U[MX1] * U[BX1] + U[MX2] * U[BX2] + U[MX3] * U[BX3];
    q.B2 = U[BX1] * U[BX1] + U[BX2] * U[BX2] + U[BX3] * U[BX3];
    V[BX1] = U[BX1];
    V[BX2] = U[BX2];
    V[BX3] = U[BX3];
    V[PSI] = U[PSI];
    int ok = 1;
    if (!(q.D > 0.0)) ok = 0;
    /* lower end: largest W with v^2 >= 1 */
    double lo = 0.0, hi = 1.0;
    double scale = q.D + q.E + sqrt(q.m2) + q.B2 + 1e-300;
    hi = scale;
    while (rmhd_v2_of_W(&q, hi) >= 1.0 && hi < 1e300) hi *= 2.0;
    if (rmhd_v2_of_W(&q, 1e-300) < 1.0) {
        lo = 0.0; /* v^2 < 1 everywhere */
    } else {
        double a = 0.0, c = hi;
        for (int it = 0; it < 2000 && c - a > 0.0; it++) {
            double mid = 0.5 * (a + c);
            if (mid <= a || mid >= c) break;
            if (rmhd_v2_of_W(&q, mid) >= 1.0) a = mid; else c = mid;
        }
        lo = c; /* first W with v^2 < 1 */
    }
    /* upper end: grow until f > 0 */
    double whi = (lo > 0.0 ? 2.0 * lo : scale);
    if (whi < scale) whi = scale;
    int grow = 0;
    while (rmhd_resid(&q, whi, NULL, NULL) <= 0.0 && grow < 4000) { whi *= 2.0; grow++; }
    double flo = rmhd_resid(&q, lo > 0.0 ? lo : 1e-300, NULL, NULL);
    if (!(flo < 0.0)) ok = 0;
    double a = (lo > 0.0 ? lo : 1e-300), c = whi;
    for (int it = 0; it < 5000; it++) {
        double mid = 0.5 * (a + c);
        if (mid <= a || mid >= c) break;
        if (rmhd_resid(&q, mid, NULL, NULL) > 0.0) c = mid; else a = mid;
    }
    double W = 0.5 * (a + c);
    double p, v2;
    rmhd_resid(&q, W, &p, &v2);
    double lor = 1.0 / sqrt(1.0 - v2);
    V[RHO] = q.D / lor;
    V[PRS] = p;
    for (int c3 = 0; c3 < 3; c3++)
        V[MX1 + c3] = (U[MX1 + c3] + q.S / W * U[BX1 + c3]) / (W + q.B2);
    if (fails) {
        if (!ok) fails[FAIL_NEWTON]++;
        if (!(V[RHO] > 0.0)) fails[FAIL_RHO]++;
        if (!(p > 0.0)) fails[FAIL_PRS]++;
        if (!(v2 < 1.0)) fails[FAIL_VEL]++;
        for (int v = 0; v < NVAR; v++)
            if (isnan(V[v])) { fails[FAIL_NAN]++; break; }
    }
    return ok;
}

static void rmhd_flux(const orc_opts *o, const double *V, const double *U, int d, double *F)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double v2 = V[MX1] * V[MX1] + V[MX2] * V[MX2] + V[MX3] * V[MX3];
    double B2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    double vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    double lor2 = 1.0 / (1.0 - v2);
    double w = rmhd_enthalpy(o, V[RHO], V[PRS]);
    double E[3];
    /* E = -v x B */
    E[0] = -(V[MX2] * V[BX3] - V[MX3] * V[BX2]);
    E[1] = -(V[MX3] * V[BX1] - V[MX1] * V[BX3]);
    E[2] = -(V[MX1] * V[BX2] - V[MX2] * V[BX1]);
    double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    double pt = V[PRS] + 0.5 * (B2 + E2);
    double vn = V[MX1 + n];
    (void)vB;
    F[RHO] = U[RHO] * vn;
    for (int c = 0; c < 3; c++)
        F[MX1 + c] = w * lor2 * vn * V[MX1 + c] - V[BX1 + n] * V[BX1 + c] - E[n] * E[c] + (c == n ? pt : 0.0);
    F[ENG] = U[MX1 + n] - U[RHO] * vn;
    F[BX1 + n] = 0.0;
    F[BX1 + t] = vn * V[BX1 + t] - V[BX1 + n] * V[MX1 + t];
    F[BX1 + b] = vn * V[BX1 + b] - V[BX1 + n] * V[MX1 + b];
    F[PSI] = 0.0;
}

/* Outer signal speeds along d: the isotropic upper bound on the fast
 * magnetosonic speeds built from a^2 = cs^2 + ca^2 - cs^2 ca^2 and the
 * relativistic velocity addition along d. */
static void rmhd_speeds(const orc_opts *o, const double *V, int d, double *lmin, double *lmax)
{
    double v2 = V[MX1] * V[MX1] + V[MX2] * V[MX2] + V[MX3] * V[MX3];
    double B2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    double vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    double w = rmhd_enthalpy(o, V[RHO], V[PRS]);
    double cs2 = rmhd_cs2(o, V[PRS], w);
    double bb2 = B2 * (1.0 - v2) + vB * vB; /* b^2 = B^2/gamma^2 + (v.B)^2 */
    double ca2 = bb2 / (w + bb2);
    double a2 = cs2 + ca2 - cs2 * ca2;
    double vn = V[MX1 + d];
    double den = 1.0 - v2 * a2;
    double disc = (1.0 - v2) * (1.0 - v2 * a2 - vn * vn * (1.0 - a2));
    if (disc < 0.0) disc = 0.0;
    double root = sqrt(a2) * sqrt(disc);
    *lmin = (vn * (1.0 - a2) - root) / den;
    *lmax = (vn * (1.0 - a2) + root) / den;
    if (!o->exact_speeds) return;
    /* The exact fast magnetosonic speeds are the outermost roots of the
     * lab-frame dispersion relation (a quartic in lambda)
     *   g = w (1 - cs^2) A^4 - (w cs^2 + b^2) A^2 (1 - l^2) + cs^2 Bl^2 (1 - l^2)
     * with A = gamma (v_d - l), Bl = b^d - l b^0, b^0 = gamma v.B,
     * b^d = B_d / gamma + b^0 v_d.  Its four roots are real and the bounds
     * above enclose them, so Newton from each bound moves monotonically
     * inwards to the fast root. */
    double lor = 1.0 / sqrt(1.0 - v2);
    double b0 = lor * vB;
    double bd = V[BX1 + d] / lor + b0 * vn;
    double c4 = w * (1.0 - cs2), c2 = w * cs2 + bb2;
    for (int side = 0; side < 2; side++) {
        double l = side ? *lmax : *lmin;
        for (int it = 0; it < 100; it++) {
            double A = lor * (vn - l), Bl = bd - l * b0, G = 1.0 - l * l;
            double g = c4 * A * A * A * A - c2 * A * A * G + cs2 * Bl * Bl * G;
            double dg = -4.0 * lor * c4 * A * A * A - c2 * (-2.0 * lor * A * G - 2.0 * l * A * A) +
                        cs2 * (-2.0 * b0 * Bl * G - 2.0 * l * Bl * Bl);
            if (dg == 0.0) break;
            double ln = l - g / dg;
            if (fabs(ln - l) <= 1e-15 * fmax(fabs(l), 1e-300)) { l = ln; break; }
            l = ln;
        }
        if (side) *lmax = l; else *lmin = l;
    }
}

/* ------------------------------------------------------------------------ */
/* Physics dispatch                                                          */
/* ------------------------------------------------------------------------ */

static void prim2cons(const orc_opts *o, const double *V, double *U)
{
    if (o->physics == PHYS_MHD) mhd_prim2cons(o, V, U); else rmhd_prim2cons(o, V, U);
}

static void cons2prim(const orc_opts *o, const double *U, double *V, int *fails)
{
    if (o->physics == PHYS_MHD) {
        mhd_cons2prim(o, U, V, fails);
    } else {
        ORC_ROOT_BEGIN;
        rmhd_cons2prim(o, U, V, fails);
        ORC_ROOT_END;
    }
}

/* Physical flux along d including the GLM rows (Eq. glm2x2): F_{B_n} = psi,
 * F_psi = c_h^2 B_n. */
static void phys_flux(const orc_opts *o, const double *V, int d, double ch, double *F)
{
    double U[NVAR];
    prim2cons(o, V, U);
    if (o->physics == PHYS_MHD) mhd_flux(o, V, U, d, F); else rmhd_flux(o, V, U, d, F);
    if (o->glm) {
        F[BX1 + d] = V[PSI];
        F[PSI] = ch * ch * V[BX1 + d];
    }
}

static void signal_speeds(const orc_opts *o, const double *V, int d, double *lmin, double *lmax)
{
    if (o->physics == PHYS_MHD) {
        double cf = mhd_fast_speed(o, V, d);
        *lmin = V[MX1 + d] - cf;
        *lmax = V[MX1 + d] + cf;
    } else {
        rmhd_speeds(o, V, d, lmin, lmax);
    }
}

/* ------------------------------------------------------------------------ */
/* Riemann solvers                                                           */
/* ------------------------------------------------------------------------ */

/* HLL: single intermediate state between the outer signal speeds. */
static void riemann_hll(const orc_opts *o, const double *VL, const double *VR, int d, double ch,
                        double *F, double *smax)
{
    double lminL, lmaxL, lminR, lmaxR;
    signal_speeds(o, VL, d, &lminL, &lmaxL);
    signal_speeds(o, VR, d, &lminR, &lmaxR);
    double SL = fmin(lminL, lminR);
    double SR = fmax(lmaxL, lmaxR);
    *smax = fmax(fabs(SL), fabs(SR));
    double FL[NVAR], FR[NVAR], UL[NVAR], UR[NVAR];
    phys_flux(o, VL, d, ch, FL);
    phys_flux(o, VR, d, ch, FR);
    prim2cons(o, VL, UL);
    prim2cons(o, VR, UR);
    if (SL >= 0.0) {
        memcpy(F, FL, sizeof(FL));
    } else if (SR <= 0.0) {
        memcpy(F, FR, sizeof(FR));
    } else {
        for (int v = 0; v < NVAR; v++)
            F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) / (SR - SL);
    }
}

/* Rusanov (local Lax-Friedrichs), Sec. 3.1's list of solvers common to the
 * classical and relativistic modules: the centred flux minus a dissipation
 * set by the largest signal speed magnitude a of the two states,
 * F = (F_L + F_R)/2 - a (U_R - U_L)/2. */
static void riemann_rusanov(const orc_opts *o, const double *VL, const double *VR, int d, double ch,
                            double *F, double *smax)
{
    double lminL, lmaxL, lminR, lmaxR;
    signal_speeds(o, VL, d, &lminL, &lmaxL);
    signal_speeds(o, VR, d, &lminR, &lmaxR);
    double a = fmax(fmax(fabs(lminL), fabs(lmaxL)), fmax(fabs(lminR), fabs(lmaxR)));
    *smax = a;
    double FL[NVAR], FR[NVAR], UL[NVAR], UR[NVAR];
    phys_flux(o, VL, d, ch, FL);
    phys_flux(o, VR, d, ch, FR);
    prim2cons(o, VL, UL);
    prim2cons(o, VR, UR);
    for (int v = 0; v < NVAR; v++) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * a * (UR[v] - UL[v]);
}

/* HLLC for ideal MHD (Sec. 3.1's list; the single-contact construction of
 * Li 2005), for states sharing B_n.  The outer speeds are HLL's; the contact
 * moves with the HLL average of the normal velocity, S_M = m_n^hll /
 * rho^hll; both star states carry the HLL average B* of the transverse
 * field, and v*.B* is taken from the HLL state.  The rest follows from the
 * jump conditions across the outer wave S of each side:
 *   rho*      = rho (S - u) / (S - S_M),
 *   p_t*      = p_t + rho (S - u)(S_M - u),
 *   (rho v_t)* = (rho v_t (S - u) - B_n (B_t* - B_t)) / (S - S_M),
 *   E*        = ((S - u) E - p_t u + p_t* S_M + B_n (v.B - v*.B*)) / (S - S_M),
 * and F* = F + S (U* - U) on the side holding the interface.  With B = 0 it
 * is the hydrodynamic HLLC of Toro, Spruce & Speares. */
static void riemann_hllc(const orc_opts *o, const double *VL, const double *VR, int d, double ch,
                         double *F, double *smax)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double cfL = mhd_fast_speed(o, VL, d), cfR = mhd_fast_speed(o, VR, d);
    double uL = VL[MX1 + n], uR = VR[MX1 + n];
    double SL = fmin(uL - cfL, uR - cfR);
    double SR = fmax(uL + cfL, uR + cfR);
    *smax = fmax(fabs(SL), fabs(SR));
    double UL[NVAR], UR[NVAR], FL[NVAR], FR[NVAR];
    prim2cons(o, VL, UL);
    prim2cons(o, VR, UR);
    phys_flux(o, VL, d, ch, FL);
    phys_flux(o, VR, d, ch, FR);
    if (SL >= 0.0) { memcpy(F, FL, sizeof(FL)); return; }
    if (SR <= 0.0) { memcpy(F, FR, sizeof(FR)); return; }
    double Uh[NVAR];
    for (int v = 0; v < NVAR; v++) Uh[v] = (SR * UR[v] - SL * UL[v] - (FR[v] - FL[v])) / (SR - SL);
    double SM = Uh[MX1 + n] / Uh[RHO];
    double vt = Uh[MX1 + t] / Uh[RHO], vb = Uh[MX1 + b] / Uh[RHO];
    double Bn = VL[BX1 + n], Bt = Uh[BX1 + t], Bb = Uh[BX1 + b];
    double vBs = SM * Bn + vt * Bt + vb * Bb;
    const double *V = (SM >= 0.0) ? VL : VR;
    const double *U = (SM >= 0.0) ? UL : UR;
    const double *Fs = (SM >= 0.0) ? FL : FR;
    double S = (SM >= 0.0) ? SL : SR;
    double u = V[MX1 + n];
    double B2 = V[BX1] * V[BX1] + V[BX2] * V[BX2] + V[BX3] * V[BX3];
    double pt = V[PRS] + 0.5 * B2;
    double vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
    double rs = V[RHO] * (S - u) / (S - SM);
    double pts = pt + V[RHO] * (S - u) * (SM - u);
    double Us[NVAR];
    Us[RHO] = rs;
    Us[MX1 + n] = rs * SM;
    Us[MX1 + t] = (U[MX1 + t] * (S - u) - Bn * (Bt - V[BX1 + t])) / (S - SM);
    Us[MX1 + b] = (U[MX1 + b] * (S - u) - Bn * (Bb - V[BX1 + b])) / (S - SM);
    Us[ENG] = ((S - u) * U[ENG] - pt * u + pts * SM + Bn * (vB - vBs)) / (S - SM);
    Us[BX1 + n] = Bn;
    Us[BX1 + t] = Bt;
    Us[BX1 + b] = Bb;
    Us[PSI] = U[PSI];
    for (int v = 0; v < NVAR; v++) F[v] = Fs[v] + S * (Us[v] - U[v]);
}

/* HLLC for relativistic MHD (Sec. 3.1's list; Mignone & Bodo 2006), for
 * states sharing B_n.  E below is the total energy U[ENG] + D, whose flux is
 * m_n.  From the HLL averages U^hll, F^hll:
 *  B_n != 0: both star states hold B*_t = B_t^hll; the contact speed
 *    lambda* is the root with the minus sign of
 *      (F_E - B*.F_B) l^2 - (E + F_mn - B*^2 - F_B^2) l + (m_n - B*.F_B) = 0
 *    (B* and F_B the transverse HLL field and its HLL flux), which follows
 *    from m*_n = (E* + p_t*) lambda* - (v*.B*) B_n and
 *    F*_mn = F*_E lambda* - B_n (B_n / gamma*^2 + (v*.B*) lambda*) + p_t*
 *    taken on the HLL state and flux, with the transverse velocity from the
 *    induction flux v*_t = (B*_t lambda* - F_Bt) / B_n (the cubic terms
 *    cancel); p_t* then follows from the second relation;
 *  B_n = 0 (B_n^2 <= 1e-12 (B_n^2 + B*^2)): the hydrodynamic relations with
 *    p_t: F_E l^2 - (E + F_mn) l + m_n = 0, p_t* = F_mn - F_E lambda*.
 * The star state of the side holding the interface follows from the jump
 * conditions across its outer wave S:
 *   D* = (S D - F_D) / (S - l*),  E* = (S E - m_n + p_t* l* - (v*.B*) B_n) / (S - l*),
 *   m*_n = (E* + p_t*) l* - (v*.B*) B_n,
 *   m*_t = (S m_t - F_mt - B_n (B*_t / gamma*^2 + (v*.B*) v*_t)) / (S - l*)
 *   (B_n = 0: m*_t = (S m_t - F_mt)/(S - l*), B*_t = (S B_t - F_Bt)/(S - l*)),
 * and F* = F + S (U* - U).  The root is taken in the form 2c / (-b +
 * sqrt(b^2 - 4ac)), which has no cancellation as a -> 0.  Where the star
 * state is not admissible (negative discriminant, l* outside (S_L, S_R),
 * v*^2 >= 1 or D* <= 0) the face takes the HLL flux. */
static void riemann_hllc_rmhd(const orc_opts *o, const double *VL, const double *VR, int d, double ch, double *F,
                              double *smax)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double lminL, lmaxL, lminR, lmaxR;
    signal_speeds(o, VL, d, &lminL, &lmaxL);
    signal_speeds(o, VR, d, &lminR, &lmaxR);
    double SL = fmin(lminL, lminR), SR = fmax(lmaxL, lmaxR);
    *smax = fmax(fabs(SL), fabs(SR));
    double UL[NVAR], UR[NVAR], FL[NVAR], FR[NVAR];
    prim2cons(o, VL, UL);
    prim2cons(o, VR, UR);
    phys_flux(o, VL, d, ch, FL);
    phys_flux(o, VR, d, ch, FR);
    if (SL >= 0.0) { memcpy(F, FL, sizeof(FL)); return; }
    if (SR <= 0.0) { memcpy(F, FR, sizeof(FR)); return; }
    double Uh[NVAR], Fh[NVAR];
    for (int v = 0; v < NVAR; v++) {
        Uh[v] = (SR * UR[v] - SL * UL[v] - (FR[v] - FL[v])) / (SR - SL);
        Fh[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) / (SR - SL);
    }
    double Eh = Uh[ENG] + Uh[RHO], FEh = Fh[ENG] + Fh[RHO];
    double Bn = VL[BX1 + n];
    double Bt = Uh[BX1 + t], Bb = Uh[BX1 + b], Ft = Fh[BX1 + t], Fb = Fh[BX1 + b];
    int magnetic = Bn * Bn > 1e-12 * (Bn * Bn + Bt * Bt + Bb * Bb);
    double qa, qb, qc;
    if (magnetic) {
        double BF = Bt * Ft + Bb * Fb;
        qa = FEh - BF;
        qb = -(Eh + Fh[MX1 + n]) + Bt * Bt + Bb * Bb + Ft * Ft + Fb * Fb;
        qc = Uh[MX1 + n] - BF;
    } else {
        qa = FEh;
        qb = -(Eh + Fh[MX1 + n]);
        qc = Uh[MX1 + n];
    }
    double disc = qb * qb - 4.0 * qa * qc;
    int ok = disc >= 0.0;
    double ls = ok ? 2.0 * qc / (-qb + sqrt(disc)) : 0.0;
    ok = ok && ls > SL && ls < SR;
    double vt = 0.0, vb = 0.0, vBs = 0.0, ig2 = 1.0, pts;
    if (magnetic) {
        vt = (Bt * ls - Ft) / Bn;
        vb = (Bb * ls - Fb) / Bn;
        double vs2 = ls * ls + vt * vt + vb * vb;
        ok = ok && vs2 < 1.0;
        ig2 = 1.0 - vs2;
        vBs = ls * Bn + vt * Bt + vb * Bb;
        pts = Fh[MX1 + n] - FEh * ls + Bn * (Bn * ig2 + vBs * ls);
    } else {
        pts = Fh[MX1 + n] - FEh * ls;
    }
    int right = !(ls >= 0.0);
    const double *U = right ? UR : UL;
    const double *Fk = right ? FR : FL;
    double S = right ? SR : SL;
    double iS = 1.0 / (S - ls);
    double Us[NVAR];
    Us[RHO] = (S * U[RHO] - Fk[RHO]) * iS;
    double Ek = U[ENG] + U[RHO];
    double Es = (S * Ek - U[MX1 + n] + pts * ls - vBs * Bn) * iS;
    Us[MX1 + n] = (Es + pts) * ls - vBs * Bn;
    if (magnetic) {
        Us[MX1 + t] = (S * U[MX1 + t] - Fk[MX1 + t] - Bn * (Bt * ig2 + vBs * vt)) * iS;
        Us[MX1 + b] = (S * U[MX1 + b] - Fk[MX1 + b] - Bn * (Bb * ig2 + vBs * vb)) * iS;
        Us[BX1 + t] = Bt;
        Us[BX1 + b] = Bb;
    } else {
        Us[MX1 + t] = (S * U[MX1 + t] - Fk[MX1 + t]) * iS;
        Us[MX1 + b] = (S * U[MX1 + b] - Fk[MX1 + b]) * iS;
        Us[BX1 + t] = (S * U[BX1 + t] - Fk[BX1 + t]) * iS;
        Us[BX1 + b] = (S * U[BX1 + b] - Fk[BX1 + b]) * iS;
    }
    Us[ENG] = Es - Us[RHO];
    Us[BX1 + n] = Bn;
    Us[PSI] = U[PSI];
    ok = ok && Us[RHO] > 0.0;
    for (int v = 0; v < NVAR; v++) F[v] = ok ? Fk[v] + S * (Us[v] - U[v]) : Fh[v];
}

/* HLLD for relativistic MHD (Mignone, Ugliano & Bodo 2009), for states
 * sharing B_n.  Five waves: the outer fast waves S_L, S_R (HLL's speeds),
 * two rotational discontinuities and the contact, with the total pressure
 * p uniform between the fast waves.  E is the total energy U[ENG] + D.
 *  - Across a fast wave S with R = S U - F (known from the outer state), the
 *    state a for a trial p has, with A = R_mn - S R_E + p (1 - S^2),
 *    G = R_Bt^2 + R_Bb^2, C = R_mt R_Bt + R_mb R_Bb, Q = -A - G + B_n^2 (1 - S^2)
 *    and X = B_n (A S B_n + C) - (A + G)(S p + R_E):
 *      v_n = (B_n (A B_n + S C) - (A + G)(p + R_mn)) / X,
 *      v_t = (Q R_mt + R_Bt (C + B_n (S R_mn - R_E))) / X  (and b),
 *      B_t = (R_Bt - B_n v_t) / (S - v_n),  w_t = p + (R_E - v.R_m) / (S - v_n),
 *    D_a = R_D / (S - v_n), E_a = (R_E + p v_n - (v.B) B_n) / (S - v_n),
 *    m_a = (E_a + p) v - (v.B) B.
 *  - The rotational discontinuity next to it moves at K_n with
 *      K = (R_m + p e_n + eta R_B) / (S p + R_E + eta B_n),
 *    eta = -+ sgn(B_n) sqrt(w_t) on the left / right (R_Bn = S B_n).
 *  - The contact region holds B_c, the field that conserves B across the two
 *    rotational discontinuities,
 *      B_c = ((B (K_n - v_n) + B_n v)_R - (B (K_n - v_n) + B_n v)_L) / (K_nR - K_nL),
 *    and on each side v_c = K - B_c (1 - K^2) / (eta - K.B_c).
 *  - p solves v_cn(R) - v_cn(L) = 0 (secant iteration from the HLLC estimate
 *    of p_t* and 1.025 times it, until successive iterates agree to 1e-14).
 *  - The contact states follow from the jump conditions across the
 *    rotational discontinuities: D_c = D_a (K_n - v_an) / (K_n - v_cn),
 *    E_c = (K_n E_a - m_an + p v_cn - (v_c.B_c) B_n) / (K_n - v_cn),
 *    m_c = (E_c + p) v_c - (v_c.B_c) B_c.
 * The flux of the region holding the interface follows by F* = F + S (U* - U)
 * across each wave in turn.  B_n = 0 (B_n^2 <= 1e-12 (B_n^2 + B^hll_t^2)), or
 * a fan that is not admissible (no convergence, |v| >= 1, D <= 0, w_t <= p,
 * or wave speeds out of order), gives the HLLC flux. */
static void riemann_hllc_rmhd(const orc_opts *o, const double *VL, const double *VR, int d, double ch, double *F,
                              double *smax);

typedef struct {
    double U[8]; /* D, m_n, m_t, m_b, E, B_n, B_t, B_b */
    double v[3], B[3], wt, eta, K[3];
    int ok;
} rhlld_side;

/* state a behind a fast wave of speed S for the trial pressure p */
static void rhlld_astate(const double *R, double S, double p, double Bn, double sg, rhlld_side *a)
{
    double A = R[1] - S * R[4] + p * (1.0 - S * S);
    double G = R[6] * R[6] + R[7] * R[7];
    double C = R[2] * R[6] + R[3] * R[7];
    double Q = -A - G + Bn * Bn * (1.0 - S * S);
    double X = Bn * (A * S * Bn + C) - (A + G) * (S * p + R[4]);
    a->v[0] = (Bn * (A * Bn + S * C) - (A + G) * (p + R[1])) / X;
    a->v[1] = (Q * R[2] + R[6] * (C + Bn * (S * R[1] - R[4]))) / X;
    a->v[2] = (Q * R[3] + R[7] * (C + Bn * (S * R[1] - R[4]))) / X;
    double iS = 1.0 / (S - a->v[0]);
    a->B[0] = Bn;
    a->B[1] = (R[6] - Bn * a->v[1]) * iS;
    a->B[2] = (R[7] - Bn * a->v[2]) * iS;
    a->wt = p + (R[4] - (a->v[0] * R[1] + a->v[1] * R[2] + a->v[2] * R[3])) * iS;
    double vB = a->v[0] * a->B[0] + a->v[1] * a->B[1] + a->v[2] * a->B[2];
    a->U[0] = R[0] * iS;
    a->U[4] = (R[4] + p * a->v[0] - vB * Bn) * iS;
    for (int k = 0; k < 3; k++) a->U[1 + k] = (a->U[4] + p) * a->v[k] - vB * a->B[k];
    for (int k = 0; k < 3; k++) a->U[5 + k] = a->B[k];
    double v2 = a->v[0] * a->v[0] + a->v[1] * a->v[1] + a->v[2] * a->v[2];
    a->ok = isfinite(X) && X != 0.0 && v2 < 1.0 && a->wt > p && a->U[0] > 0.0;
    a->eta = sg * sgn1(Bn) * sqrt(fmax(a->wt, 0.0));
    double den = S * p + R[4] + a->eta * Bn;
    a->K[0] = (R[1] + p + a->eta * R[5]) / den;
    a->K[1] = (R[2] + a->eta * R[6]) / den;
    a->K[2] = (R[3] + a->eta * R[7]) / den;
}

/* both sides for the trial p; returns v_cn(R) - v_cn(L) and the contact data */
static double rhlld_fan(const double *RL, const double *RR, double SL, double SR, double p, double Bn,
                        rhlld_side *aL, rhlld_side *aR, double *Bc, double *vcL, double *vcR)
{
    rhlld_astate(RL, SL, p, Bn, -1.0, aL);
    rhlld_astate(RR, SR, p, Bn, +1.0, aR);
    double dK = aR->K[0] - aL->K[0];
    Bc[0] = Bn;
    for (int k = 1; k < 3; k++)
        Bc[k] = ((aR->B[k] * (aR->K[0] - aR->v[0]) + Bn * aR->v[k]) - (aL->B[k] * (aL->K[0] - aL->v[0]) + Bn * aL->v[k])) /
                dK;
    const rhlld_side *sd[2] = { aL, aR };
    double *vc[2] = { vcL, vcR };
    for (int s2 = 0; s2 < 2; s2++) {
        const double *K = sd[s2]->K;
        double K2 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
        double KB = K[0] * Bc[0] + K[1] * Bc[1] + K[2] * Bc[2];
        double y = (1.0 - K2) / (sd[s2]->eta - KB);
        for (int k = 0; k < 3; k++) vc[s2][k] = K[k] - Bc[k] * y;
    }
    return vcR[0] - vcL[0];
}

static void riemann_hlld_rmhd(const orc_opts *o, const double *VL, const double *VR, int d, double ch, double *F,
                              double *smax)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double lminL, lmaxL, lminR, lmaxR;
    signal_speeds(o, VL, d, &lminL, &lmaxL);
    signal_speeds(o, VR, d, &lminR, &lmaxR);
    double SL = fmin(lminL, lminR), SR = fmax(lmaxL, lmaxR);
    *smax = fmax(fabs(SL), fabs(SR));
    double UL9[NVAR], UR9[NVAR], FL9[NVAR], FR9[NVAR];
    prim2cons(o, VL, UL9);
    prim2cons(o, VR, UR9);
    phys_flux(o, VL, d, ch, FL9);
    phys_flux(o, VR, d, ch, FR9);
    if (SL >= 0.0) { memcpy(F, FL9, sizeof(FL9)); return; }
    if (SR <= 0.0) { memcpy(F, FR9, sizeof(FR9)); return; }
    /* rotated 8-vectors with the total energy; the hyperbolic B_n flux is 0 */
    double UL[8], UR[8], FL[8], FR[8];
    const int map[8] = { RHO, MX1 + n, MX1 + t, MX1 + b, ENG, BX1 + n, BX1 + t, BX1 + b };
    for (int k = 0; k < 8; k++) {
        UL[k] = UL9[map[k]];
        UR[k] = UR9[map[k]];
        FL[k] = FL9[map[k]];
        FR[k] = FR9[map[k]];
    }
    UL[4] += UL[0]; UR[4] += UR[0];
    FL[4] += FL[0]; FR[4] += FR[0];
    FL[5] = FR[5] = 0.0;
    double Bn = VL[BX1 + n];
    double Uh[8], Fh[8], RL[8], RR[8];
    for (int k = 0; k < 8; k++) {
        Uh[k] = (SR * UR[k] - SL * UL[k] - (FR[k] - FL[k])) / (SR - SL);
        Fh[k] = (SR * FL[k] - SL * FR[k] + SL * SR * (UR[k] - UL[k])) / (SR - SL);
        RL[k] = SL * UL[k] - FL[k];
        RR[k] = SR * UR[k] - FR[k];
    }
    int use_hllc = !(Bn * Bn > 1e-12 * (Bn * Bn + Uh[6] * Uh[6] + Uh[7] * Uh[7]));
    /* initial guess: the relativistic HLLC total pressure */
    double p0 = 0.0;
    if (!use_hllc) {
        double BF = Uh[6] * Fh[6] + Uh[7] * Fh[7];
        double qa = Fh[4] - BF;
        double qb = -(Uh[4] + Fh[1]) + Uh[6] * Uh[6] + Uh[7] * Uh[7] + Fh[6] * Fh[6] + Fh[7] * Fh[7];
        double qc = Uh[1] - BF;
        double disc = qb * qb - 4.0 * qa * qc;
        double ls = 2.0 * qc / (-qb + sqrt(fmax(disc, 0.0)));
        double vt = (Uh[6] * ls - Fh[6]) / Bn, vb = (Uh[7] * ls - Fh[7]) / Bn;
        double ig2 = 1.0 - ls * ls - vt * vt - vb * vb;
        double vBs = ls * Bn + vt * Uh[6] + vb * Uh[7];
        p0 = Fh[1] - Fh[4] * ls + Bn * (Bn * ig2 + vBs * ls);
        if (!(disc >= 0.0) || !(p0 > 0.0) || !isfinite(p0)) use_hllc = 1;
    }
    rhlld_side aL, aR;
    double Bc[3], vcL[3], vcR[3], p = p0;
    int ok = !use_hllc;
    if (ok) {
        double pa = p0, pb = 1.025 * p0;
        double fa = rhlld_fan(RL, RR, SL, SR, pa, Bn, &aL, &aR, Bc, vcL, vcR);
        double fb = rhlld_fan(RL, RR, SL, SR, pb, Bn, &aL, &aR, Bc, vcL, vcR);
        int conv = 0;
        for (int it = 0; it < 40; it++) {
            if (fb == fa || !isfinite(fa) || !isfinite(fb)) break;
            double pc = pb - fb * (pb - pa) / (fb - fa);
            pa = pb;
            fa = fb;
            pb = pc;
            fb = rhlld_fan(RL, RR, SL, SR, pb, Bn, &aL, &aR, Bc, vcL, vcR);
            if (fabs(pb - pa) <= 1e-14 * fabs(pb)) { conv = 1; break; }
        }
        if (fb == 0.0) conv = 1;
        p = pb;
        rhlld_fan(RL, RR, SL, SR, p, Bn, &aL, &aR, Bc, vcL, vcR);
        double vc2 = vcL[0] * vcL[0] + vcL[1] * vcL[1] + vcL[2] * vcL[2];
        double vr2 = vcR[0] * vcR[0] + vcR[1] * vcR[1] + vcR[2] * vcR[2];
        ok = conv && p > 0.0 && aL.ok && aR.ok && vc2 < 1.0 && vr2 < 1.0 && SL <= aL.K[0] && aL.K[0] <= vcL[0] &&
             vcR[0] <= aR.K[0] && aR.K[0] <= SR;
    }
    if (!ok) {
        riemann_hllc_rmhd(o, VL, VR, d, ch, F, smax);
        return;
    }
    /* contact states */
    double vc[3];
    for (int k = 0; k < 3; k++) vc[k] = 0.5 * (vcL[k] + vcR[k]);
    double vBc = vc[0] * Bc[0] + vc[1] * Bc[1] + vc[2] * Bc[2];
    double UcL[8], UcR[8];
    const rhlld_side *sd[2] = { &aL, &aR };
    double *Uc[2] = { UcL, UcR };
    for (int s2 = 0; s2 < 2; s2++) {
        const rhlld_side *a = sd[s2];
        double la = a->K[0];
        double iS = 1.0 / (la - vc[0]);
        Uc[s2][0] = a->U[0] * (la - a->v[0]) * iS;
        Uc[s2][4] = (la * a->U[4] - a->U[1] + p * vc[0] - vBc * Bn) * iS;
        for (int k = 0; k < 3; k++) Uc[s2][1 + k] = (Uc[s2][4] + p) * vc[k] - vBc * Bc[k];
        for (int k = 0; k < 3; k++) Uc[s2][5 + k] = Bc[k];
    }
    double Fr[8];
    for (int k = 0; k < 8; k++) {
        double FaL = FL[k] + SL * (aL.U[k] - UL[k]);
        double FcL = FaL + aL.K[0] * (UcL[k] - aL.U[k]);
        double FaR = FR[k] + SR * (aR.U[k] - UR[k]);
        double FcR = FaR + aR.K[0] * (UcR[k] - aR.U[k]);
        if (aL.K[0] >= 0.0) Fr[k] = FaL;
        else if (vc[0] >= 0.0) Fr[k] = FcL;
        else if (aR.K[0] >= 0.0) Fr[k] = FcR;
        else Fr[k] = FaR;
    }
    Fr[4] -= Fr[0];
    for (int k = 0; k < 8; k++) F[map[k]] = Fr[k];
    F[PSI] = 0.0;
}

/* HLLD for ideal MHD (Miyoshi & Kusano 2005), for states sharing B_n. */
static void riemann_hlld(const orc_opts *o, const double *VL, const double *VR, int d, double ch,
                         double *F, double *smax)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double cfL = mhd_fast_speed(o, VL, d), cfR = mhd_fast_speed(o, VR, d);
    double uL = VL[MX1 + n], uR = VR[MX1 + n];
    double SL = fmin(uL - cfL, uR - cfR);
    double SR = fmax(uL + cfL, uR + cfR);
    *smax = fmax(fabs(SL), fabs(SR));

    double UL[NVAR], UR[NVAR], FL[NVAR], FR[NVAR];
    prim2cons(o, VL, UL);
    prim2cons(o, VR, UR);
    phys_flux(o, VL, d, ch, FL);
    phys_flux(o, VR, d, ch, FR);
    if (SL >= 0.0) { memcpy(F, FL, sizeof(FL)); return; }
    if (SR <= 0.0) { memcpy(F, FR, sizeof(FR)); return; }

    double Bn = VL[BX1 + n]; /* equal to VR[BX1+n] by construction */
    double B2L = VL[BX1] * VL[BX1] + VL[BX2] * VL[BX2] + VL[BX3] * VL[BX3];
    double B2R = VR[BX1] * VR[BX1] + VR[BX2] * VR[BX2] + VR[BX3] * VR[BX3];
    double ptL = VL[PRS] + 0.5 * B2L, ptR = VR[PRS] + 0.5 * B2R;
    double rhoL = VL[RHO], rhoR = VR[RHO];
    double aL = (SL - uL) * rhoL, aR = (SR - uR) * rhoR;
    double SM = (aR * uR - aL * uL - ptR + ptL) / (aR - aL);
    double pts = (aR * ptL - aL * ptR + aL * aR * (uR - uL)) / (aR - aL);

    /* single-star states */
    double Us[2][NVAR], vs[2][3], Bs[2][3], sqr[2];
    const double *Vk[2] = { VL, VR };
    const double *Uk[2] = { UL, UR };
    double Sk[2] = { SL, SR };
    for (int s = 0; s < 2; s++) {
        const double *V = Vk[s];
        double S = Sk[s], u = V[MX1 + n], rho = V[RHO];
        double rhos = rho * (S - u) / (S - SM);
        double den = rho * (S - u) * (S - SM) - Bn * Bn;
        double scale = rho * fabs(S - u) * fabs(S - SM) + Bn * Bn;
        vs[s][n] = SM;
        Bs[s][n] = Bn;
        if (fabs(den) <= 1e-12 * scale) {
            /* degenerate: transverse velocity and field are continuous */
            vs[s][t] = V[MX1 + t];
            vs[s][b] = V[MX1 + b];
            Bs[s][t] = V[BX1 + t];
            Bs[s][b] = V[BX1 + b];
        } else {
            double fv = Bn * (SM - u) / den;
            double fB = (rho * (S - u) * (S - u) - Bn * Bn) / den;
            vs[s][t] = V[MX1 + t] - V[BX1 + t] * fv;
            vs[s][b] = V[MX1 + b] - V[BX1 + b] * fv;
            Bs[s][t] = V[BX1 + t] * fB;
            Bs[s][b] = V[BX1 + b] * fB;
        }
        double vB = V[MX1] * V[BX1] + V[MX2] * V[BX2] + V[MX3] * V[BX3];
        double vBs = vs[s][0] * Bs[s][0] + vs[s][1] * Bs[s][1] + vs[s][2] * Bs[s][2];
        double pt = (s == 0 ? ptL : ptR);
        double Es = ((S - u) * Uk[s][ENG] - pt * u + pts * SM + Bn * (vB - vBs)) / (S - SM);
        Us[s][RHO] = rhos;
        for (int c = 0; c < 3; c++) {
            Us[s][MX1 + c] = rhos * vs[s][c];
            Us[s][BX1 + c] = Bs[s][c];
        }
        Us[s][ENG] = Es;
        Us[s][PSI] = V[PSI];
        sqr[s] = sqrt(rhos);
    }
    double SLs = SM - fabs(Bn) / sqr[0];
    double SRs = SM + fabs(Bn) / sqr[1];

    if (SLs >= 0.0) {
        for (int v = 0; v < NVAR; v++) F[v] = FL[v] + SL * (Us[0][v] - UL[v]);
    } else if (SRs <= 0.0) {
        for (int v = 0; v < NVAR; v++) F[v] = FR[v] + SR * (Us[1][v] - UR[v]);
    } else {
        /* double-star states */
        double sB = sgn1(Bn);
        double den = sqr[0] + sqr[1];
        double vss[3], Bss[3];
        vss[n] = SM;
        Bss[n] = Bn;
        vss[t] = (sqr[0] * vs[0][t] + sqr[1] * vs[1][t] + (Bs[1][t] - Bs[0][t]) * sB) / den;
        vss[b] = (sqr[0] * vs[0][b] + sqr[1] * vs[1][b] + (Bs[1][b] - Bs[0][b]) * sB) / den;
        Bss[t] = (sqr[0] * Bs[1][t] + sqr[1] * Bs[0][t] + sqr[0] * sqr[1] * (vs[1][t] - vs[0][t]) * sB) / den;
        Bss[b] = (sqr[0] * Bs[1][b] + sqr[1] * Bs[0][b] + sqr[0] * sqr[1] * (vs[1][b] - vs[0][b]) * sB) / den;
        double vBss = vss[0] * Bss[0] + vss[1] * Bss[1] + vss[2] * Bss[2];
        double Uss[2][NVAR];
        for (int s = 0; s < 2; s++) {
            double vBs = vs[s][0] * Bs[s][0] + vs[s][1] * Bs[s][1] + vs[s][2] * Bs[s][2];
            double sgn = (s == 0 ? -1.0 : 1.0);
            Uss[s][RHO] = Us[s][RHO];
            for (int c = 0; c < 3; c++) {
                Uss[s][MX1 + c] = Us[s][RHO] * vss[c];
                Uss[s][BX1 + c] = Bss[c];
            }
            Uss[s][ENG] = Us[s][ENG] + sgn * sqr[s] * (vBs - vBss) * sB;
            Uss[s][PSI] = Us[s][PSI];
        }
        if (SM >= 0.0) {
            for (int v = 0; v < NVAR; v++)
                F[v] = FL[v] + SLs * Uss[0][v] - (SLs - SL) * Us[0][v] - SL * UL[v];
        } else {
            for (int v = 0; v < NVAR; v++)
                F[v] = FR[v] + SRs * Uss[1][v] - (SRs - SR) * Us[1][v] - SR * UR[v];
        }
    }
}

static void rot7(const double *V, int d, double *q);
static void unrot7(const double *q, int d, double *V);
static void mhd_right_eigen(const orc_opts *o, const double *V, int d, double R[7][7], double lam[7]);
static int invert7(double A[7][7], double Ainv[7][7]);

/* Roe's linearised solver for ideal MHD (Sec. 3.1's list), for states
 * sharing B_n:  F = (F_L + F_R)/2 - (1/2) |A| (U_R - U_L)  with a matrix A
 * for which F_R - F_L = A (U_R - U_L) holds exactly.
 *
 * Averages (weights sqrt(rho_L), sqrt(rho_R)): v~ and H~ = (E + p_t)/rho;
 * the transverse field takes the swapped weights,
 *   B~_t = (sqrt(rho_R) B_tL + sqrt(rho_L) B_tR) / (sqrt(rho_L) + sqrt(rho_R)),
 * rho^ = sqrt(rho_L rho_R) and X = |B_tR - B_tL|^2 / (2 (sqrt(rho_L) +
 * sqrt(rho_R))^2) (Cargo & Gallice 1997).  The exact jump identities
 *   d(rho v^2/2) = v~.dm - v~^2/2 drho,   d(B_t^2/2) = B~_t.dB_t + X drho,
 *   d(v_k B_t) = v~_k dB_t + B~_t dv_k,   dv = (dm - v~ drho)/rho^,
 *   d(rho H v_n) = H~ dm_n + v~_n d(rho H) - H~ v~_n drho
 * make the flux jump A dU with A the primitive-variable Jacobian at the
 * state (rho^, v~, B_n, B~_t, p^), gamma p^ / rho^ = a~^2 =
 * (gamma - 1)(H~ - v~^2/2 - (B_n^2 + B~_t^2)/rho^) - (gamma - 2) X, acting on
 *   dW = (drho, (dm - v~ drho)/rho^, dB_t, dp),
 *   dp = (gamma - 1)(dE - v~.dm + v~^2/2 drho - B~_t.dB_t) - (gamma - 2) X drho.
 * So |A| dU is sum_k |lambda_k| (l_k . dW) r_k mapped back to conserved
 * differences, with the primitive eigenvectors of that state.  No entropy
 * fix is applied: |lambda| depends on the averaged speed alone, so waves of
 * equal speed are damped alike whichever family their degenerate
 * eigenvectors are counted in.  The signal speed is the largest fast-wave
 * |lambda| of the average and both states. */
static void riemann_roe(const orc_opts *o, const double *VL, const double *VR, int d, double ch,
                        double *F, double *smax)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    const double g = o->gamma;
    double UL[NVAR], UR[NVAR], FL[NVAR], FR[NVAR];
    prim2cons(o, VL, UL);
    prim2cons(o, VR, UR);
    phys_flux(o, VL, d, ch, FL);
    phys_flux(o, VR, d, ch, FR);

    double sL = sqrt(VL[RHO]), sR = sqrt(VR[RHO]);
    double wL = sL / (sL + sR), wR = sR / (sL + sR);
    double rhoh = sL * sR;
    double v[3], q2 = 0.0;
    for (int k = 0; k < 3; k++) {
        v[k] = wL * VL[MX1 + k] + wR * VR[MX1 + k];
        q2 += v[k] * v[k];
    }
    double B2L = VL[BX1] * VL[BX1] + VL[BX2] * VL[BX2] + VL[BX3] * VL[BX3];
    double B2R = VR[BX1] * VR[BX1] + VR[BX2] * VR[BX2] + VR[BX3] * VR[BX3];
    double HL = (UL[ENG] + VL[PRS] + 0.5 * B2L) / VL[RHO];
    double HR = (UR[ENG] + VR[PRS] + 0.5 * B2R) / VR[RHO];
    double H = wL * HL + wR * HR;
    double Bn = VL[BX1 + n];
    double Bt[3] = { 0.0, 0.0, 0.0 };
    double dB2 = 0.0;
    Bt[t] = wR * VL[BX1 + t] + wL * VR[BX1 + t];
    Bt[b] = wR * VL[BX1 + b] + wL * VR[BX1 + b];
    dB2 = (VR[BX1 + t] - VL[BX1 + t]) * (VR[BX1 + t] - VL[BX1 + t]) +
          (VR[BX1 + b] - VL[BX1 + b]) * (VR[BX1 + b] - VL[BX1 + b]);
    double X = dB2 / (2.0 * (sL + sR) * (sL + sR));
    double a2 = (g - 1.0) * (H - 0.5 * q2 - (Bn * Bn + Bt[t] * Bt[t] + Bt[b] * Bt[b]) / rhoh) - (g - 2.0) * X;

    /* the averaged primitive state and its eigensystem */
    double Vh[NVAR];
    memset(Vh, 0, sizeof(Vh));
    Vh[RHO] = rhoh;
    for (int k = 0; k < 3; k++) Vh[MX1 + k] = v[k];
    Vh[BX1 + n] = Bn;
    Vh[BX1 + t] = Bt[t];
    Vh[BX1 + b] = Bt[b];
    Vh[PRS] = rhoh * a2 / g;
    double R[7][7], L[7][7], lam[7], RL[7][7], lamL[7], RR[7][7], lamR[7];
    mhd_right_eigen(o, Vh, d, R, lam);
    ORC_SIDE_BEGIN;
    invert7(R, L);
    ORC_SIDE_END;
    mhd_right_eigen(o, VL, d, RL, lamL);
    mhd_right_eigen(o, VR, d, RR, lamR);

    /* dU -> dW */
    double dU[NVAR], dW[NVAR], q[7];
    for (int k = 0; k < NVAR; k++) dU[k] = UR[k] - UL[k];
    memset(dW, 0, sizeof(dW));
    dW[RHO] = dU[RHO];
    double vdm = 0.0;
    for (int k = 0; k < 3; k++) {
        dW[MX1 + k] = (dU[MX1 + k] - v[k] * dU[RHO]) / rhoh;
        vdm += v[k] * dU[MX1 + k];
    }
    dW[BX1 + t] = dU[BX1 + t];
    dW[BX1 + b] = dU[BX1 + b];
    dW[PRS] = (g - 1.0) * (dU[ENG] - vdm + 0.5 * q2 * dU[RHO] - Bt[t] * dU[BX1 + t] - Bt[b] * dU[BX1 + b]) -
              (g - 2.0) * X * dU[RHO];
    rot7(dW, d, q);

    /* sum_k |lambda_k| (l_k . dW) r_k */
    double D7[7] = { 0.0 };
    for (int k = 0; k < 7; k++) {
        double al = 0.0;
        for (int m = 0; m < 7; m++) al += L[k][m] * q[m];
        for (int m = 0; m < 7; m++) D7[m] += fabs(lam[k]) * al * R[m][k];
    }
    double DW[NVAR];
    memset(DW, 0, sizeof(DW));
    unrot7(D7, d, DW);

    /* dW -> dU */
    double DU[NVAR];
    memset(DU, 0, sizeof(DU));
    DU[RHO] = DW[RHO];
    double vdv = 0.0;
    for (int k = 0; k < 3; k++) {
        DU[MX1 + k] = v[k] * DW[RHO] + rhoh * DW[MX1 + k];
        vdv += v[k] * DW[MX1 + k];
    }
    DU[BX1 + t] = DW[BX1 + t];
    DU[BX1 + b] = DW[BX1 + b];
    DU[ENG] = (DW[PRS] + (g - 2.0) * X * DW[RHO]) / (g - 1.0) + Bt[t] * DW[BX1 + t] + Bt[b] * DW[BX1 + b] +
              0.5 * q2 * DW[RHO] + rhoh * vdv;
    for (int k = 0; k < NVAR; k++) F[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * DU[k];
    *smax = fmax(fmax(fabs(lam[0]), fabs(lam[6])),
                 fmax(fmax(fabs(lamL[0]), fabs(lamL[6])), fmax(fabs(lamR[0]), fabs(lamR[6]))));
}

/* Full interface solve along d: the linear (B_n, psi) subsystem of Eq.
 * glm2x2 is solved exactly (characteristics psi +- c_h B_n), its interface
 * value of B_n is imposed on both states, then HLLD or HLL gives the other
 * seven fluxes.  Without GLM the two normal fields are averaged. */
/* Number of Riemann solves since the last orc_riemann_count(1): an
 * instrument for the statement of Sec. 3.1 that a 3D step takes six solves
 * per zone (two per face direction). */
static long orc_nsolve = 0;

static void riemann(const orc_opts *o, const double *VLin, const double *VRin, int d, double ch,
                    double *F, double *smax)
{
#pragma omp atomic
    orc_nsolve++;
    double VL[NVAR], VR[NVAR];
    memcpy(VL, VLin, sizeof(VL));
    memcpy(VR, VRin, sizeof(VR));
    double Bm, psim;
    if (o->glm) {
        Bm = 0.5 * (VL[BX1 + d] + VR[BX1 + d]) - (VR[PSI] - VL[PSI]) / (2.0 * ch);
        psim = 0.5 * (VL[PSI] + VR[PSI]) - 0.5 * ch * (VR[BX1 + d] - VL[BX1 + d]);
    } else {
        Bm = 0.5 * (VL[BX1 + d] + VR[BX1 + d]);
        psim = 0.0;
    }
    VL[BX1 + d] = VR[BX1 + d] = Bm;
    if (o->riemann == RS_HLLD && o->physics == PHYS_MHD)
        riemann_hlld(o, VL, VR, d, ch, F, smax);
    else if (o->riemann == RS_HLLD)
        riemann_hlld_rmhd(o, VL, VR, d, ch, F, smax);
    else if (o->riemann == RS_HLLC && o->physics == PHYS_MHD)
        riemann_hllc(o, VL, VR, d, ch, F, smax);
    else if (o->riemann == RS_HLLC)
        riemann_hllc_rmhd(o, VL, VR, d, ch, F, smax);
    else if (o->riemann == RS_ROE && o->physics == PHYS_MHD)
        riemann_roe(o, VL, VR, d, ch, F, smax);
    else if (o->riemann == RS_RUSANOV)
        riemann_rusanov(o, VL, VR, d, ch, F, smax);
    else
        riemann_hll(o, VL, VR, d, ch, F, smax);
    if (o->glm) {
        F[BX1 + d] = psim;
        F[PSI] = ch * ch * Bm;
    } else {
        F[BX1 + d] = 0.0;
        F[PSI] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Limiters and reconstruction (Sec. 3.2)                                    */
/* ------------------------------------------------------------------------ */

static double minmod(double a, double b) /* Eq. minmod */
{
    return 0.5 * (sgn0(a) + sgn0(b)) * fmin(fabs(a), fabs(b));
}

static double lim_mc(double dp, double dm) /* Eq. MClim */
{
    return minmod(0.5 * (dp + dm), 2.0 * minmod(dm, dp));
}

static double lim_vanleer(double dp, double dm) /* Eq. harmonic_lim */
{
    return (dp * dm > 0.0) ? 2.0 * dp * dm / (dp + dm) : 0.0;
}

static double lim_vanalbada(double dp, double dm) /* Eq. vanalbada_lim */
{
    return (dp * dm > 0.0) ? dp * dm * (dp + dm) / (dp * dp + dm * dm) : 0.0;
}

static double limited_slope(int recon, double dp, double dm)
{
    switch (recon) {
    case REC_LIN_MINMOD: return minmod(dp, dm);
    case REC_LIN_VANLEER: return lim_vanleer(dp, dm);
    case REC_LIN_VANALBADA: return lim_vanalbada(dp, dm);
    default: return lim_mc(dp, dm);
    }
}

/* Interface values w_{-}, w_{+} of cell 0 from the stencil w[l+2], l=-2..2
 * (linear and WENO3 use l=-1..1 only). */
static void reconstruct(int recon, const double *w, double dx, double *wm, double *wp)
{
    double w0 = w[2];
    double dp = w[3] - w[2]; /* Delta w_{+1/2} */
    double dm = w[2] - w[1]; /* Delta w_{-1/2} */
    if (recon == REC_PPM) {
        double s0 = lim_mc(dp, dm);
        double sp = lim_mc(w[4] - w[3], w[3] - w[2]);
        double sm = lim_mc(w[1] - w[0], w[2] - w[1]);
        double wP = 0.5 * (w0 + w[3]) - (sp - s0) / 6.0; /* Eq. ppm1 */
        double wM = 0.5 * (w0 + w[1]) + (sm - s0) / 6.0;
        double dP = wP - w0, dM = wM - w0;
        double nP, nM;
        if (dP * dM > 0.0) { /* Eq. ppm_parabolic_lim: local extremum */
            nP = 0.0;
            nM = 0.0;
        } else {
            nP = (fabs(dP) >= 2.0 * fabs(dM)) ? -2.0 * dM : dP;
            nM = (fabs(dM) >= 2.0 * fabs(dP)) ? -2.0 * dP : dM;
        }
        *wp = w0 + nP;
        *wm = w0 + nM;
    } else if (recon == REC_WENO3) {
        double d2 = (dp - dm) * (dp - dm);
        double ap = 1.0 + d2 / (dx * dx + dp * dp); /* Eq. WENO3a */
        double am = 1.0 + d2 / (dx * dx + dm * dm);
        *wp = w0 + (ap * dp + 0.5 * am * dm) / (2.0 * ap + am); /* Eq. WENO3 */
        *wm = w0 - (am * dm + 0.5 * ap * dp) / (2.0 * am + ap);
    } else {
        double s = limited_slope(recon, dp, dm); /* Eq. Linear */
        *wp = w0 + 0.5 * s;
        *wm = w0 - 0.5 * s;
    }
}

/* Upwind tracing of one characteristic field to the half step (Eq.
 * wnorm_predp / wnorm_predm).  nu = lambda dt / dx. */
static void trace_wave(int wref, double w0, double wm, double wp, double nu, double numax, double numin,
                       double *wsm, double *wsp)
{
    double dw = wp - wm;
    double d2w = wp - 2.0 * w0 + wm;
    double bp = 0.5 * (1.0 + sgn0(nu));
    double bm = 0.5 * (1.0 - sgn0(nu));
    double tp = wp - 0.5 * nu * (dw + d2w * (3.0 - 2.0 * nu));
    double tm = wm - 0.5 * nu * (dw - d2w * (3.0 + 2.0 * nu));
    double rp, rm;
    if (wref == WREF_CELL) {
        rp = w0;
        rm = w0;
    } else if (wref == WREF_CW84) {
        rp = wp - 0.5 * numax * (dw + d2w * (3.0 - 2.0 * numax));
        rm = wm - 0.5 * numin * (dw - d2w * (3.0 + 2.0 * numin));
    } else {
        rp = wp;
        rm = wm;
    }
    *wsp = rp + bp * (tp - rp);
    *wsm = rm + bm * (tm - rm);
}

/* ------------------------------------------------------------------------ */
/* Eigenvectors of the primitive MHD system (normalized after Roe & Balsara)  */
/* ------------------------------------------------------------------------ */

/* Rotated 7-component primitive vector (rho, v_n, v_t, v_b, B_t, B_b, p). */
static void rot7(const double *V, int d, double *q)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    q[0] = V[RHO];
    q[1] = V[MX1 + n];
    q[2] = V[MX1 + t];
    q[3] = V[MX1 + b];
    q[4] = V[BX1 + t];
    q[5] = V[BX1 + b];
    q[6] = V[PRS];
}

static void unrot7(const double *q, int d, double *V)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    V[RHO] = q[0];
    V[MX1 + n] = q[1];
    V[MX1 + t] = q[2];
    V[MX1 + b] = q[3];
    V[BX1 + t] = q[4];
    V[BX1 + b] = q[5];
    V[PRS] = q[6];
}

/* Right eigenvectors R[m][k] (component m of wave k) and eigenvalues of the
 * 7-wave primitive system along d, with B_n held as a parameter.  Waves in
 * order: v-cf, v-ca, v-cs, v, v+cs, v+ca, v+cf. */
static void mhd_right_eigen(const orc_opts *o, const double *V, int d, double R[7][7], double lam[7])
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    double rho = V[RHO], p = V[PRS];
    double Bn = V[BX1 + n], Bt = V[BX1 + t], Bb = V[BX1 + b];
    double a2 = o->gamma * p / rho;
    double a = sqrt(a2);
    double srho = sqrt(rho);
    double bn2 = Bn * Bn / rho;
    double bt2 = (Bt * Bt + Bb * Bb) / rho;
    double b2 = bn2 + bt2;
    /* c_f^2 - c_s^2 = sqrt((a^2 + b^2)^2 - 4 a^2 b_n^2), written as
     * sqrt((a^2 - b^2)^2 + 4 a^2 b_t^2) so that it is exact when b_t = 0;
     * a^2 - c_s^2 and c_f^2 - a^2 then follow without cancellation. */
    double dab = a2 - b2;
    double sq = sqrt(dab * dab + 4.0 * a2 * bt2);
    double cf2 = 0.5 * (a2 + b2 + sq);
    double cs2 = a2 * bn2 / cf2; /* c_f^2 c_s^2 = a^2 c_a^2 */
    double cf = sqrt(cf2), cs = sqrt(cs2), ca = sqrt(bn2);
    double af, as;
    if (sq <= 0.0) {
        af = 1.0; /* triple degeneracy a = c_a, b_t = 0 */
        as = 0.0;
    } else {
        af = sqrt(fmax(0.5 * (sq + dab) / sq, 0.0)); /* (a^2 - c_s^2)/(c_f^2 - c_s^2) */
        as = sqrt(fmax(0.5 * (sq - dab) / sq, 0.0)); /* (c_f^2 - a^2)/(c_f^2 - c_s^2) */
    }
    double Btn2 = Bt * Bt + Bb * Bb;
    double B2 = Btn2 + Bn * Bn;
    double by, bz;
    if (Btn2 <= 1e-12 * B2) {
        by = 1.0 / sqrt(2.0);
        bz = 1.0 / sqrt(2.0);
    } else {
        double bt = sqrt(Btn2);
        by = Bt / bt;
        bz = Bb / bt;
    }
    double sB = sgn1(Bn);
    double vn = V[MX1 + n];
    lam[0] = vn - cf; lam[1] = vn - ca; lam[2] = vn - cs; lam[3] = vn;
    lam[4] = vn + cs; lam[5] = vn + ca; lam[6] = vn + cf;
    memset(R, 0, sizeof(double) * 49);
    /* fast waves */
    for (int k = 0; k < 7; k += 6) {
        double e = (k == 0 ? -1.0 : 1.0);
        R[0][k] = rho * af;
        R[1][k] = e * af * cf;
        R[2][k] = -e * sB * as * cs * by;
        R[3][k] = -e * sB * as * cs * bz;
        R[4][k] = as * a * srho * by;
        R[5][k] = as * a * srho * bz;
        R[6][k] = rho * a2 * af;
    }
    /* slow waves */
    for (int k = 2; k <= 4; k += 2) {
        double e = (k == 2 ? -1.0 : 1.0);
        R[0][k] = rho * as;
        R[1][k] = e * as * cs;
        R[2][k] = e * sB * af * cf * by;
        R[3][k] = e * sB * af * cf * bz;
        R[4][k] = -af * a * srho * by;
        R[5][k] = -af * a * srho * bz;
        R[6][k] = rho * a2 * as;
    }
    /* Alfven waves */
    for (int k = 1; k <= 5; k += 4) {
        double e = (k == 1 ? 1.0 : -1.0);
        R[2][k] = -bz;
        R[3][k] = by;
        R[4][k] = -e * sB * srho * bz;
        R[5][k] = e * sB * srho * by;
    }
    /* entropy wave */
    R[0][3] = 1.0;
}

/* Matrix inverse by Gauss-Jordan elimination with partial pivoting. */
static int invert7(double A[7][7], double Ainv[7][7])
{
    double M[7][14];
    for (int i = 0; i < 7; i++) {
        for (int j = 0; j < 7; j++) {
            M[i][j] = A[i][j];
            M[i][7 + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < 7; c++) {
        int piv = c;
        for (int r = c + 1; r < 7; r++)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (M[piv][c] == 0.0) return 0;
        if (piv != c)
            for (int j = 0; j < 14; j++) { double tmp = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = tmp; }
        double inv = 1.0 / M[c][c];
        for (int j = 0; j < 14; j++) M[c][j] *= inv;
        for (int r = 0; r < 7; r++) {
            if (r == c) continue;
            double f = M[r][c];
            if (f != 0.0)
                for (int j = 0; j < 14; j++) M[r][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < 7; i++)
        for (int j = 0; j < 7; j++) Ainv[i][j] = M[i][7 + j];
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Normal predictors                                                         */
/* ------------------------------------------------------------------------ */

/* Characteristic normal predictor (Sec. 3.2) for cell 0 of the stencil
 * Vs[l+2], l=-2..2 (primitive), along d.  Output: V*_{-}, V*_{+}. */
static void predict_char(const orc_opts *o, const double Vs[5][NVAR], int d, double dt, double ch,
                         double *Vm, double *Vp)
{
    double dx = o->dx[d];
    const double *V0 = Vs[2];
    double R[7][7], L[7][7], lam[7];
    mhd_right_eigen(o, V0, d, R, lam);
    ORC_SIDE_BEGIN;
    invert7(R, L);
    ORC_SIDE_END;

    /* Eq. char_var: project the stencil on the left eigenvectors of cell 0 */
    double q[5][7], w[7][5];
    for (int l = 0; l < 5; l++) rot7(Vs[l], d, q[l]);
    for (int k = 0; k < 7; k++)
        for (int l = 0; l < 5; l++) {
            double acc = 0.0;
            for (int m = 0; m < 7; m++) acc += L[k][m] * q[l][m];
            w[k][l] = acc;
        }
    /* GLM pair (B_n, psi) of Eq. glm2x2: speeds -c_h, +c_h with right
     * eigenvectors (1, -+c_h) and left eigenvectors (c_h, -+1)/(2 c_h) */
    double wh[2][5], lamh[2] = { -ch, ch };
    int use_glm = o->glm && ch > 0.0;
    if (use_glm) {
        for (int l = 0; l < 5; l++) {
            wh[0][l] = (ch * Vs[l][BX1 + d] - Vs[l][PSI]) / (2.0 * ch);
            wh[1][l] = (ch * Vs[l][BX1 + d] + Vs[l][PSI]) / (2.0 * ch);
        }
    }

    double nu[9], numax = 0.0, numin = 0.0;
    for (int k = 0; k < 7; k++) nu[k] = lam[k] * dt / dx;
    int nw = 7;
    if (use_glm) { nu[7] = lamh[0] * dt / dx; nu[8] = lamh[1] * dt / dx; nw = 9; }
    for (int k = 0; k < nw; k++) { numax = fmax(numax, nu[k]); numin = fmin(numin, nu[k]); }

    double wsm[7], wsp[7];
    for (int k = 0; k < 7; k++) {
        double wm, wp;
        reconstruct(o->recon, w[k], dx, &wm, &wp);
        trace_wave(o->wref, w[k][2], wm, wp, nu[k], numax, numin, &wsm[k], &wsp[k]);
    }
    double Bnm, Bnp, psim, psip, dBn, dpsi;
    if (use_glm) {
        double hm[2], hp[2], hsm[2], hsp[2];
        for (int k = 0; k < 2; k++) {
            reconstruct(o->recon, wh[k], dx, &hm[k], &hp[k]);
            trace_wave(o->wref, wh[k][2], hm[k], hp[k], nu[7 + k], numax, numin, &hsm[k], &hsp[k]);
        }
        /* r_{-} = (1, -c_h), r_{+} = (1, +c_h) in (B_n, psi) */
        dBn = (hp[0] + hp[1]) - (hm[0] + hm[1]);
        dpsi = ch * ((hp[1] - hp[0]) - (hm[1] - hm[0]));
        Bnm = hsm[0] + hsm[1];
        Bnp = hsp[0] + hsp[1];
        psim = ch * (hsm[1] - hsm[0]);
        psip = ch * (hsp[1] - hsp[0]);
    } else {
        double bn[5], bm, bp;
        for (int l = 0; l < 5; l++) bn[l] = Vs[l][BX1 + d];
        reconstruct(o->recon, bn, dx, &bm, &bp);
        dBn = bp - bm;
        dpsi = 0.0;
        Bnm = bm;
        Bnp = bp;
        psim = psip = V0[PSI];
    }

    /* right-eigenvector recombination */
    double qm[7], qp[7];
    for (int m = 0; m < 7; m++) {
        double am = 0.0, ap = 0.0;
        for (int k = 0; k < 7; k++) { am += R[m][k] * wsm[k]; ap += R[m][k] * wsp[k]; }
        qm[m] = am;
        qp[m] = ap;
    }
    unrot7(qm, d, Vm);
    unrot7(qp, d, Vp);
    Vm[BX1 + d] = Bnm;
    Vp[BX1 + d] = Bnp;
    Vm[PSI] = psim;
    Vp[PSI] = psip;

    /* Multidimensional terms: the 1D conservative system differs from the
     * 7-wave primitive one by d(B_n)/dn (0, B/rho, v_t, v_b, (1-G) v.B) and
     * d(psi)/dn in the pressure row ((G-1) B_n). */
    double rho = V0[RHO];
    double vB = V0[MX1] * V0[BX1] + V0[MX2] * V0[BX2] + V0[MX3] * V0[BX3];
    double SB[NVAR] = { 0 }, Spsi[NVAR] = { 0 };
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    SB[MX1 + n] = V0[BX1 + n] / rho;
    SB[MX1 + t] = V0[BX1 + t] / rho;
    SB[MX1 + b] = V0[BX1 + b] / rho;
    SB[BX1 + t] = V0[MX1 + t];
    SB[BX1 + b] = V0[MX1 + b];
    SB[PRS] = (1.0 - o->gamma) * vB;
    Spsi[PRS] = (o->gamma - 1.0) * V0[BX1 + n];
    for (int v = 0; v < NVAR; v++) {
        double src = 0.5 * dt * (SB[v] * dBn / dx + Spsi[v] * dpsi / dx);
        Vm[v] += src;
        Vp[v] += src;
    }
}

/* MUSCL-Hancock primitive predictor (Sec. 3.3) with beta = 1. */
static void predict_mh(const orc_opts *o, const double Vs[5][NVAR], const double *U0, int d, double dt,
                       double ch, double *Vm, double *Vp, int *fails)
{
    double dx = o->dx[d];
    double dV[NVAR], Vlo[NVAR], Vhi[NVAR];
    for (int v = 0; v < NVAR; v++) {
        dV[v] = limited_slope(o->recon, Vs[3][v] - Vs[2][v], Vs[2][v] - Vs[1][v]);
        Vlo[v] = Vs[2][v] - 0.5 * dV[v];
        Vhi[v] = Vs[2][v] + 0.5 * dV[v];
    }
    if (o->physics == PHYS_RMHD) {
        double v2lo = Vlo[MX1] * Vlo[MX1] + Vlo[MX2] * Vlo[MX2] + Vlo[MX3] * Vlo[MX3];
        double v2hi = Vhi[MX1] * Vhi[MX1] + Vhi[MX2] * Vhi[MX2] + Vhi[MX3] * Vhi[MX3];
        if (!(v2lo < 1.0) || !(v2hi < 1.0)) {
            /* superluminal reconstruction: first order in this cell */
            if (fails) fails[FAIL_VEL]++;
            for (int v = 0; v < NVAR; v++) { dV[v] = 0.0; Vlo[v] = Vhi[v] = Vs[2][v]; }
        }
    }
    double Flo[NVAR], Fhi[NVAR], Us[NVAR], Vh[NVAR];
    phys_flux(o, Vlo, d, ch, Flo);
    phys_flux(o, Vhi, d, ch, Fhi);
    for (int v = 0; v < NVAR; v++) Us[v] = U0[v] - 0.5 * dt / dx * (Fhi[v] - Flo[v]);
    int fl[NFAIL] = { 0 };
    cons2prim(o, Us, Vh, fl);
    int bad = 0;
    for (int k = 0; k < NFAIL; k++) bad |= fl[k];
    if (bad) {
        if (fails) for (int k = 0; k < NFAIL; k++) fails[k] += fl[k];
        memcpy(Vh, Vs[2], sizeof(Vh));
    }
    for (int v = 0; v < NVAR; v++) {
        Vm[v] = Vh[v] - 0.5 * dV[v];
        Vp[v] = Vh[v] + 0.5 * dV[v];
    }
}

/* ------------------------------------------------------------------------ */
/* Parabolic fluxes (Sec. 2.1.1, Sec. 3.1, App. A)                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int NX, NY, NZ;
    long NC;
} grid_t;

static long cidx(const grid_t *g, int i, int j, int k) { return ((long)k * g->NY + j) * g->NX + i; }

/* Parabolic face flux Pi (9 components) on the d-face between cell A = c - e_d
 * and cell B = c.  Vc: primitive point values; Uc: conserved values (face
 * coefficients use g((U_A + U_B)/2)).  pL, pR, rL, rR: pressures and
 * densities of the Riemann input states used by the saturated flux. */
static void parab_flux(const orc_opts *o, const grid_t *g, const double *Vc, const double *Uc, int i, int j,
                       int k, int d, double pL, double pR, double rL, double rR, double *Pi)
{
    int n, t, b;
    dir_axes(d, &n, &t, &b);
    int off[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };
    long NC = g->NC;
    long cB = cidx(g, i, j, k);
    long cA = cidx(g, i - off[d][0], j - off[d][1], k - off[d][2]);
    /* face averages of conserved variables */
    double rhof = 0.5 * (Uc[RHO * NC + cA] + Uc[RHO * NC + cB]);
    double vf[3], Bf[3];
    for (int c = 0; c < 3; c++) {
        vf[c] = (Uc[(MX1 + c) * NC + cA] + Uc[(MX1 + c) * NC + cB]) / (Uc[RHO * NC + cA] + Uc[RHO * NC + cB]);
        Bf[c] = 0.5 * (Uc[(BX1 + c) * NC + cA] + Uc[(BX1 + c) * NC + cB]);
    }
    /* gradients of f = (v_x, v_y, v_z, B_x, B_y, B_z, T) at the face */
    double grad[7][3];
    for (int f = 0; f < 7; f++) {
        for (int e = 0; e < 3; e++) {
            if (e >= o->dim) { grad[f][e] = 0.0; continue; }
#define FVAL(ii, jj, kk)                                                                            \
    (f < 3 ? Vc[(MX1 + f) * NC + cidx(g, ii, jj, kk)]                                              \
           : (f < 6 ? Vc[(BX1 + f - 3) * NC + cidx(g, ii, jj, kk)]                                 \
                    : Vc[PRS * NC + cidx(g, ii, jj, kk)] / Vc[RHO * NC + cidx(g, ii, jj, kk)]))
            if (e == d) {
                grad[f][e] = (FVAL(i, j, k) - FVAL(i - off[d][0], j - off[d][1], k - off[d][2])) / o->dx[d];
            } else {
                int ai = i - off[d][0], aj = j - off[d][1], ak = k - off[d][2];
                int ei = off[e][0], ej = off[e][1], ek = off[e][2];
                double up = FVAL(i + ei, j + ej, k + ek) + FVAL(ai + ei, aj + ej, ak + ek);
                double dn = FVAL(i - ei, j - ej, k - ek) + FVAL(ai - ei, aj - ej, ak - ek);
                grad[f][e] = (up - dn) / (4.0 * o->dx[e]);
            }
#undef FVAL
        }
    }
    for (int v = 0; v < NVAR; v++) Pi[v] = 0.0;
    double G = o->gamma;
    if (o->parabolic_mask & PARAB_VISC) {
        /* Eq. visc_tens, row n */
        double divv = grad[0][0] + grad[1][1] + grad[2][2];
        double tau[3];
        for (int c = 0; c < 3; c++) {
            tau[c] = rhof * o->nu * (grad[c][n] + grad[n][c] - (c == n ? 2.0 / 3.0 * divv : 0.0));
            Pi[MX1 + c] += tau[c];
        }
        Pi[ENG] += vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2];
    }
    if (o->parabolic_mask & PARAB_RES) {
        /* J = curl B;  d B/dt = -curl(eta J)  =>  flux of B_t is eta J_b, of B_b is -eta J_t */
        double J[3];
        J[0] = grad[5][1] - grad[4][2];
        J[1] = grad[3][2] - grad[5][0];
        J[2] = grad[4][0] - grad[3][1];
        Pi[BX1 + t] += o->eta * J[b];
        Pi[BX1 + b] += -o->eta * J[t];
        /* energy: -(eta J x B)_n */
        double JxB_n = J[t] * Bf[b] - J[b] * Bf[t];
        Pi[ENG] += -o->eta * JxB_n;
    }
    if (o->parabolic_mask & PARAB_TC) {
        double B2 = Bf[0] * Bf[0] + Bf[1] * Bf[1] + Bf[2] * Bf[2];
        double bh[3] = { 0.0, 0.0, 0.0 };
        if (B2 > 0.0) {
            double Bm = sqrt(B2);
            for (int c = 0; c < 3; c++) bh[c] = Bf[c] / Bm;
        }
        double bgT = bh[0] * grad[6][0] + bh[1] * grad[6][1] + bh[2] * grad[6][2];
        double Fcl[3];
        for (int c = 0; c < 3; c++)
            Fcl[c] = o->kappa_par * bh[c] * bgT + o->kappa_perp * (grad[6][c] - bh[c] * bgT);
        double Fmag = sqrt(Fcl[0] * Fcl[0] + Fcl[1] * Fcl[1] + Fcl[2] * Fcl[2]);
        double Fc = Fcl[n];
        if (o->tc_phi > 0.0 && Fmag > 0.0) {
            /* Eq. sat_flux: upwinded saturated flux, then the harmonic blend */
            double tx = Fcl[n] / Fmag;
            double rh = 0.5 * (rL + rR);
            double pu = (tx < 0.0) ? pL : pR;
            double q = 5.0 * o->tc_phi * pu * sqrt(pu) / sqrt(rh);
            Fc = q / (Fmag + q) * Fcl[n];
        }
        Pi[ENG] += Fc;
    }
    (void)G;
}

/* Largest diffusion coefficient at a cell, entering Eq. Ca. */
static double diff_coeff(const orc_opts *o, const double *V)
{
    double D = 0.0;
    if (o->parabolic_mask & PARAB_VISC) D = fmax(D, o->nu);
    if (o->parabolic_mask & PARAB_RES) D = fmax(D, o->eta);
    if (o->parabolic_mask & PARAB_TC)
        D = fmax(D, (o->gamma - 1.0) * fmax(o->kappa_par, o->kappa_perp) / V[RHO]);
    return D;
}

/* ------------------------------------------------------------------------ */
/* Public helpers for the tests                                              */
/* ------------------------------------------------------------------------ */

void orc_prim2cons(const orc_opts *o, long ncell, const double *V, double *U)
{
    /* V, U are [9][ncell] */
    for (long c = 0; c < ncell; c++) {
        double v[NVAR], u[NVAR];
        for (int q = 0; q < NVAR; q++) v[q] = V[q * ncell + c];
        prim2cons(o, v, u);
        for (int q = 0; q < NVAR; q++) U[q * ncell + c] = u[q];
    }
}

void orc_cons2prim(const orc_opts *o, long ncell, const double *U, double *V, int *fails)
{
    for (long c = 0; c < ncell; c++) {
        double v[NVAR], u[NVAR];
        for (int q = 0; q < NVAR; q++) u[q] = U[q * ncell + c];
        cons2prim(o, u, v, fails);
        for (int q = 0; q < NVAR; q++) V[q * ncell + c] = v[q];
    }
}

void orc_flux(const orc_opts *o, const double *V, int d, double ch, double *F) { phys_flux(o, V, d, ch, F); }

void orc_riemann(const orc_opts *o, const double *VL, const double *VR, int d, double ch, double *F,
                 double *smax)
{
    riemann(o, VL, VR, d, ch, F, smax);
}

void orc_speeds(const orc_opts *o, const double *V, int d, double *lmin, double *lmax)
{
    signal_speeds(o, V, d, lmin, lmax);
}

void orc_eigen(const orc_opts *o, const double *V, int d, double *R, double *L, double *lam)
{
    double Rm[7][7], Lm[7][7];
    mhd_right_eigen(o, V, d, Rm, lam);
    ORC_SIDE_BEGIN;
    invert7(Rm, Lm);
    ORC_SIDE_END;
    memcpy(R, Rm, sizeof(Rm));
    memcpy(L, Lm, sizeof(Lm));
}

void orc_reconstruct(int recon, const double *w, double dx, double *wm, double *wp)
{
    reconstruct(recon, w, dx, wm, wp);
}

void orc_trace(int wref, double w0, double wm, double wp, double nu, double numax, double numin, double *wsm,
               double *wsp)
{
    trace_wave(wref, w0, wm, wp, nu, numax, numin, wsm, wsp);
}

void orc_predict(const orc_opts *o, const double *Vs /*[5][9]*/, const double *U0, int d, double dt, double ch,
                 double *Vm, double *Vp, int *fails)
{
    double S[5][NVAR];
    memcpy(S, Vs, sizeof(S));
    if (o->predictor == PRED_CHAR) predict_char(o, S, d, dt, ch, Vm, Vp);
    else predict_mh(o, S, U0, d, dt, ch, Vm, Vp, fails);
}

/* ------------------------------------------------------------------------ */
/* The CTU step on one ghosted box (Sec. 3.1)                                */
/* ------------------------------------------------------------------------ */

/* App. B: flag zones inside strong compressive pressure jumps,
 * sum_d |p_{+1} - p_{-1}| / min(p_{+1}, p_{-1}) > eps_q with div v < 0
 * (central differences), for the HLL solver (FLAG_HLL); every zone whose
 * reconstruction stencil (radius 2 for PPM, else 1) along an axis reaches
 * a flagged zone is flagged for MinMod linear reconstruction
 * (FLAG_MINMOD).  Zones without both neighbours along every axis are not
 * tested.  V: primitive [9][cells]. */
enum { FLAG_HLL = 1, FLAG_MINMOD = 2 };
static const int shock_offs[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };

static void shock_flags(const orc_opts *o, const grid_t *g, const double *V, const int N[3], unsigned char *flag)
{
    const int dim = o->dim;
    const long NC = g->NC;
    for (int k = 0; k < g->NZ; k++)
        for (int j = 0; j < g->NY; j++)
            for (int i = 0; i < g->NX; i++) {
                int ci[3] = { i, j, k }, ok = 1;
                for (int d = 0; d < dim; d++)
                    if (ci[d] < 1 || ci[d] > N[d] - 2) ok = 0;
                if (!ok) continue;
                double gradp = 0.0, divv = 0.0;
                for (int d = 0; d < dim; d++) {
                    const int *e = shock_offs[d];
                    long cp = cidx(g, i + e[0], j + e[1], k + e[2]);
                    long cm = cidx(g, i - e[0], j - e[1], k - e[2]);
                    double pp = V[PRS * NC + cp], pm = V[PRS * NC + cm];
                    gradp += fabs(pp - pm) / fmin(pp, pm);
                    divv += (V[(MX1 + d) * NC + cp] - V[(MX1 + d) * NC + cm]) / (2.0 * o->dx[d]);
                }
                if (gradp > o->shock_eps && divv < 0.0) flag[cidx(g, i, j, k)] |= FLAG_HLL;
            }
    int S = (o->recon == REC_PPM) ? 2 : 1;
    for (int k = 0; k < g->NZ; k++)
        for (int j = 0; j < g->NY; j++)
            for (int i = 0; i < g->NX; i++) {
                if (!(flag[cidx(g, i, j, k)] & FLAG_HLL)) continue;
                for (int d = 0; d < dim; d++) {
                    const int *e = shock_offs[d];
                    for (int s2 = -S; s2 <= S; s2++) {
                        int ii = i + s2 * e[0], jj = j + s2 * e[1], kk = k + s2 * e[2];
                        if (ii < 0 || ii >= g->NX || jj < 0 || jj >= g->NY || kk < 0 || kk >= g->NZ) continue;
                        flag[cidx(g, ii, jj, kk)] |= FLAG_MINMOD;
                    }
                }
            }
}

/* Exported for the pins: the App. B flags of a ghosted box (flags_out has
 * one byte per ghosted cell). */
int orc_shock_flags(const orc_opts *o, int nx, int ny, int nz, int ng, const double *U, unsigned char *flags_out)
{
    if (o->dim != 2 && o->dim != 3) return -1;
    grid_t g;
    int gz = (o->dim == 3) ? ng : 0;
    g.NX = nx + 2 * ng;
    g.NY = ny + 2 * ng;
    g.NZ = nz + 2 * gz;
    g.NC = (long)g.NX * g.NY * g.NZ;
    int N[3] = { g.NX, g.NY, g.NZ };
    double *V = malloc(sizeof(double) * NVAR * g.NC);
    for (long c = 0; c < g.NC; c++) {
        double u[NVAR], v[NVAR];
        for (int q = 0; q < NVAR; q++) u[q] = U[q * g.NC + c];
        cons2prim(o, u, v, NULL);
        for (int q = 0; q < NVAR; q++) V[q * g.NC + c] = v[q];
    }
    memset(flags_out, 0, g.NC);
    if (o->shock_eps > 0.0) shock_flags(o, &g, V, N, flags_out);
    free(V);
    return 0;
}

/*
 * orc_step: advance the interior of one ghosted box by dt.
 *   nx, ny, nz : interior extents (nz == 1 when dim == 2)
 *   ng         : ghost zones per side in active directions
 *   U_in       : [9][NZ][NY][NX] conserved, ghosts filled by the caller
 *   L0         : per-cell cooling coefficient on the same ghosted layout, or NULL
 *   U_out      : receives U^{n+1} in the interior (ghosts copied from U_in)
 *   face_flux  : optional [dim][9][NZ][NY][NX]; entry at cell c in direction d
 *                is dt*(F - Pi) on the face between c-e_d and c, interior
 *                faces only (others zero)
 *   out_scalars: [0] = CFL rate (Eq. Ca), [1] = max |dp/p| of the cooling step
 *                over the cells whose `leaf` entry is nonzero (all cells when
 *                leaf is NULL: the time-step estimate of Sec. 4.2 on
 *                unrefined cells only)
 *   leaf       : optional per-cell mask on the ghosted layout, or NULL
 *   fails      : [5] counters
 * Returns 0 on success, <0 on unsupported options.
 */
int orc_step(const orc_opts *o, int nx, int ny, int nz, int ng, const double *U_in, const double *L0, double dt,
             double ch, double *U_out, double *face_flux, double *out_scalars, int *fails,
             const unsigned char *leaf)
{
    if (o->dim != 2 && o->dim != 3) return -1;
    if (o->dim == 2 && nz != 1) return -1;
    if (o->predictor == PRED_CHAR && o->physics != PHYS_MHD) return -2;
    if (o->predictor == PRED_MH && (o->recon == REC_PPM || o->recon == REC_WENO3)) return -3;
    if (o->physics == PHYS_RMHD && (o->parabolic_mask || o->cooling)) return -4;
    if (o->glm && !(ch > 0.0)) return -5;
    int mt = (o->corner == CORNER_MT);
    if (mt && (o->parabolic_mask || o->hyperbolic_off || o->shock_eps > 0.0)) return -7;
    int need = (o->recon == REC_PPM ? 3 : 2) + (o->parabolic_mask ? 1 : 0);
    if (mt && need < 3) need = 3;
    if (ng < need) return -6;

    grid_t g;
    int gz = (o->dim == 3) ? ng : 0;
    g.NX = nx + 2 * ng;
    g.NY = ny + 2 * ng;
    g.NZ = nz + 2 * gz;
    g.NC = (long)g.NX * g.NY * g.NZ;
    long NC = g.NC;
    int N[3] = { g.NX, g.NY, g.NZ };
    int lo[3] = { ng, ng, gz };
    int hi[3] = { ng + nx, ng + ny, gz + nz }; /* exclusive */
    int offs[3][3] = { { 1, 0, 0 }, { 0, 1, 0 }, { 0, 0, 1 } };
    int dim = o->dim;
    int par = (o->parabolic_mask != 0);
    int hyp = !o->hyperbolic_off;

    double *V = calloc(NVAR * NC, sizeof(double));
    double *Fn = calloc(3 * NVAR * NC, sizeof(double)); /* t^n Godunov fluxes (MT: predictor fluxes) */
    double *PVm = mt ? calloc(NVAR * NC, sizeof(double)) : NULL; /* MT: normal-predictor states */
    double *PVp = mt ? calloc(NVAR * NC, sizeof(double)) : NULL;
    double *Pn = calloc(3 * NVAR * NC, sizeof(double)); /* t^n parabolic fluxes */
    double *Ln = calloc(3 * NVAR * NC, sizeof(double)); /* -dF/dx per direction */
    double *LPn = calloc(3 * NVAR * NC, sizeof(double)); /* +dPi/dx per direction */
    double *Uhm = calloc(3 * NVAR * NC, sizeof(double)); /* corner-coupled states, minus side */
    double *Uhp = calloc(3 * NVAR * NC, sizeof(double)); /* plus side */
    double *Fh = calloc(3 * NVAR * NC, sizeof(double));  /* F^{n+1/2} */
    double *Ph = calloc(3 * NVAR * NC, sizeof(double));  /* Pi^{n+1/2} */
    double *lamf = calloc(3 * NC, sizeof(double));       /* |S|max per face */
    double *pfL = calloc(3 * NC, sizeof(double));        /* Riemann input p, rho per face */
    double *pfR = calloc(3 * NC, sizeof(double));
    double *rfL = calloc(3 * NC, sizeof(double));
    double *rfR = calloc(3 * NC, sizeof(double));
    double *Uhalf = par ? calloc(NVAR * NC, sizeof(double)) : NULL;
    double *Vhalf = par ? calloc(NVAR * NC, sizeof(double)) : NULL;
    int lf[NFAIL] = { 0 };

    /* 1. primitive recovery on every cell */
#pragma omp parallel for schedule(static) reduction(+ : lf[:NFAIL])
    for (long c = 0; c < NC; c++) {
        double u[NVAR], v[NVAR];
        for (int q = 0; q < NVAR; q++) u[q] = U_in[q * NC + c];
        cons2prim(o, u, v, lf);
        for (int q = 0; q < NVAR; q++) V[q * NC + c] = v[q];
    }

    /* 1b. App. B shock flags (see shock_flags) */
    unsigned char *flag = calloc(NC, 1);
    if (o->shock_eps > 0.0) shock_flags(o, &g, V, N, flag);
    ORC_STAGE(1);
    orc_opts o_hll = *o, o_mm = *o;
    o_hll.riemann = RS_HLL;
    o_mm.recon = REC_LIN_MINMOD;

    /* 2-3. first-order Godunov fluxes and parabolic fluxes at t^n, on every
     * face whose stencil lies inside the ghosted box.  With the MT corner
     * coupling (no parabolic terms) the transverse fluxes are instead the
     * Riemann fluxes between the normal-predictor states of the two cells
     * of a face (the predictor of step 4), on the faces whose both cells
     * have their whole predictor stencil inside the box. */
    for (int d = 0; d < dim; d++) {
        if (mt) {
#pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < g.NZ; k++)
                for (int j = 0; j < g.NY; j++)
                    for (int i = 0; i < g.NX; i++) {
                        int ci[3] = { i, j, k };
                        if (ci[d] < 2 || ci[d] > N[d] - 3) continue;
                        long c = cidx(&g, i, j, k);
                        int dummy[NFAIL] = { 0 };
                        double Vs[5][NVAR], U0[NVAR], Vm[NVAR], Vp[NVAR];
                        for (int l = -2; l <= 2; l++) {
                            long cl = cidx(&g, i + l * offs[d][0], j + l * offs[d][1], k + l * offs[d][2]);
                            for (int q = 0; q < NVAR; q++) Vs[l + 2][q] = V[q * NC + cl];
                        }
                        for (int q = 0; q < NVAR; q++) U0[q] = U_in[q * NC + c];
                        if (o->predictor == PRED_CHAR) predict_char(o, Vs, d, dt, ch, Vm, Vp);
                        else predict_mh(o, Vs, U0, d, dt, ch, Vm, Vp, dummy);
                        for (int q = 0; q < NVAR; q++) {
                            PVm[q * NC + c] = Vm[q];
                            PVp[q * NC + c] = Vp[q];
                        }
                    }
#pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < g.NZ; k++)
                for (int j = 0; j < g.NY; j++)
                    for (int i = 0; i < g.NX; i++) {
                        int ci[3] = { i, j, k };
                        if (ci[d] < 3 || ci[d] > N[d] - 3) continue;
                        long cB = cidx(&g, i, j, k);
                        long cA = cidx(&g, i - offs[d][0], j - offs[d][1], k - offs[d][2]);
                        double VL[NVAR], VR[NVAR], F[NVAR], sm;
                        for (int q = 0; q < NVAR; q++) { VL[q] = PVp[q * NC + cA]; VR[q] = PVm[q * NC + cB]; }
                        riemann(o, VL, VR, d, ch, F, &sm);
                        for (int q = 0; q < NVAR; q++) Fn[(d * NVAR + q) * NC + cB] = F[q];
                    }
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < g.NZ; k++)
            for (int j = 0; j < g.NY; j++)
                for (int i = 0; i < g.NX; i++) {
                    int ci[3] = { i, j, k };
                    if (ci[d] < 1) continue;
                    long cB = cidx(&g, i, j, k);
                    long cA = cidx(&g, i - offs[d][0], j - offs[d][1], k - offs[d][2]);
                    double VL[NVAR], VR[NVAR], F[NVAR], sm;
                    for (int q = 0; q < NVAR; q++) { VL[q] = V[q * NC + cA]; VR[q] = V[q * NC + cB]; }
                    if (hyp && !mt) {
                        int hl = (flag[cA] | flag[cB]) & FLAG_HLL;
                        riemann(hl ? &o_hll : o, VL, VR, d, ch, F, &sm);
                        for (int q = 0; q < NVAR; q++) Fn[(d * NVAR + q) * NC + cB] = F[q];
                    }
                    if (par) {
                        int ok = 1;
                        for (int e = 0; e < dim; e++)
                            if (e != d && (ci[e] < 1 || ci[e] > N[e] - 2)) ok = 0;
                        if (ok) {
                            double Pi[NVAR];
                            parab_flux(o, &g, V, U_in, i, j, k, d, VL[PRS], VR[PRS], VL[RHO], VR[RHO], Pi);
                            for (int q = 0; q < NVAR; q++) Pn[(d * NVAR + q) * NC + cB] = Pi[q];
                        }
                    }
                }
        /* increment operators per cell (Eq. incrementop_hyp / incrementop_par) */
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < g.NZ; k++)
            for (int j = 0; j < g.NY; j++)
                for (int i = 0; i < g.NX; i++) {
                    int ci[3] = { i, j, k };
                    if (ci[d] < 1 || ci[d] > N[d] - 2) continue;
                    long c = cidx(&g, i, j, k);
                    long cp = cidx(&g, i + offs[d][0], j + offs[d][1], k + offs[d][2]);
                    for (int q = 0; q < NVAR; q++) {
                        Ln[(d * NVAR + q) * NC + c] = -(Fn[(d * NVAR + q) * NC + cp] - Fn[(d * NVAR + q) * NC + c]) / o->dx[d];
                        LPn[(d * NVAR + q) * NC + c] = (Pn[(d * NVAR + q) * NC + cp] - Pn[(d * NVAR + q) * NC + c]) / o->dx[d];
                    }
                }
    }

    ORC_STAGE(2);

    /* 4. normal predictors and corner coupling (Eq. transv) on cells one
     * zone beyond the interior along d, interior across d */
    for (int d = 0; d < dim; d++) {
        int rlo[3], rhi[3];
        for (int e = 0; e < 3; e++) { rlo[e] = lo[e]; rhi[e] = hi[e]; }
        rlo[d] = lo[d] - 1;
        rhi[d] = hi[d] + 1;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : lf[:NFAIL])
        for (int k = rlo[2]; k < rhi[2]; k++)
            for (int j = rlo[1]; j < rhi[1]; j++)
                for (int i = rlo[0]; i < rhi[0]; i++) {
                    long c = cidx(&g, i, j, k);
                    double Vm[NVAR], Vp[NVAR];
                    if (hyp) {
                        double Vs[5][NVAR], U0[NVAR];
                        for (int l = -2; l <= 2; l++) {
                            int ii = i + l * offs[d][0], jj = j + l * offs[d][1], kk = k + l * offs[d][2];
                            int inside = ii >= 0 && ii < g.NX && jj >= 0 && jj < g.NY && kk >= 0 && kk < g.NZ;
                            long cl = inside ? cidx(&g, ii, jj, kk) : c;
                            for (int q = 0; q < NVAR; q++) Vs[l + 2][q] = V[q * NC + cl];
                        }
                        for (int q = 0; q < NVAR; q++) U0[q] = U_in[q * NC + c];
                        const orc_opts *op = (flag[c] & FLAG_MINMOD) ? &o_mm : o;
                        if (o->predictor == PRED_CHAR) predict_char(op, Vs, d, dt, ch, Vm, Vp);
                        else predict_mh(op, Vs, U0, d, dt, ch, Vm, Vp, lf);
                    } else {
                        for (int q = 0; q < NVAR; q++) Vm[q] = Vp[q] = V[q * NC + c];
                    }
                    double Um[NVAR], Up[NVAR];
                    prim2cons(o, Vm, Um);
                    prim2cons(o, Vp, Up);
                    for (int q = 0; q < NVAR; q++) {
                        double tr = 0.0;
                        for (int e = 0; e < dim; e++) {
                            if (e != d) tr += Ln[(e * NVAR + q) * NC + c];
                            tr += LPn[(e * NVAR + q) * NC + c];
                        }
                        Uhm[(d * NVAR + q) * NC + c] = Um[q] + 0.5 * dt * tr;
                        Uhp[(d * NVAR + q) * NC + c] = Up[q] + 0.5 * dt * tr;
                    }
                }
    }

    ORC_STAGE(3);

    /* 5. time-centred Riemann fluxes (Eq. ctu_flux) on interior-adjacent faces */
    for (int d = 0; d < dim; d++) {
        int rlo[3], rhi[3];
        for (int e = 0; e < 3; e++) { rlo[e] = lo[e]; rhi[e] = hi[e]; }
        rhi[d] = hi[d] + 1;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : lf[:NFAIL])
        for (int k = rlo[2]; k < rhi[2]; k++)
            for (int j = rlo[1]; j < rhi[1]; j++)
                for (int i = rlo[0]; i < rhi[0]; i++) {
                    long cB = cidx(&g, i, j, k);
                    long cA = cidx(&g, i - offs[d][0], j - offs[d][1], k - offs[d][2]);
                    double UL[NVAR], UR[NVAR], VL[NVAR], VR[NVAR], F[NVAR], sm = 0.0;
                    for (int q = 0; q < NVAR; q++) {
                        UL[q] = Uhp[(d * NVAR + q) * NC + cA];
                        UR[q] = Uhm[(d * NVAR + q) * NC + cB];
                    }
                    /* an unphysical corner-coupled state falls back to the
                     * cell-centred primitive state of its cell (first order) */
                    int zl[NFAIL] = { 0 }, zr[NFAIL] = { 0 }, bl = 0, br = 0;
                    cons2prim(o, UL, VL, zl);
                    cons2prim(o, UR, VR, zr);
                    for (int q = 0; q < NFAIL; q++) {
                        lf[q] += zl[q] + zr[q];
                        bl |= zl[q];
                        br |= zr[q];
                    }
                    if (bl) for (int q = 0; q < NVAR; q++) VL[q] = V[q * NC + cA];
                    if (br) for (int q = 0; q < NVAR; q++) VR[q] = V[q * NC + cB];
                    if (hyp) {
                        int hl = (flag[cA] | flag[cB]) & FLAG_HLL;
                        riemann(hl ? &o_hll : o, VL, VR, d, ch, F, &sm);
                    } else {
                        for (int q = 0; q < NVAR; q++) F[q] = 0.0;
                    }
                    for (int q = 0; q < NVAR; q++) Fh[(d * NVAR + q) * NC + cB] = F[q];
                    lamf[d * NC + cB] = sm;
                    pfL[d * NC + cB] = VL[PRS];
                    pfR[d * NC + cB] = VR[PRS];
                    rfL[d * NC + cB] = VL[RHO];
                    rfR[d * NC + cB] = VR[RHO];
                }
    }

    ORC_STAGE(4);

    /* 6. parabolic fluxes at the half step from the cell-centred U^{n+1/2} */
    if (par) {
        memcpy(Uhalf, U_in, sizeof(double) * NVAR * NC);
        int rlo[3], rhi[3];
        for (int e = 0; e < 3; e++) {
            rlo[e] = lo[e] - (e < dim ? 1 : 0);
            rhi[e] = hi[e] + (e < dim ? 1 : 0);
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = rlo[2]; k < rhi[2]; k++)
            for (int j = rlo[1]; j < rhi[1]; j++)
                for (int i = rlo[0]; i < rhi[0]; i++) {
                    long c = cidx(&g, i, j, k);
                    for (int q = 0; q < NVAR; q++) {
                        double s = 0.0;
                        for (int e = 0; e < dim; e++) s += Ln[(e * NVAR + q) * NC + c] + LPn[(e * NVAR + q) * NC + c];
                        Uhalf[q * NC + c] = U_in[q * NC + c] + 0.5 * dt * s;
                    }
                }
#pragma omp parallel for schedule(static)
        for (long c = 0; c < NC; c++) {
            double u[NVAR], v[NVAR];
            for (int q = 0; q < NVAR; q++) u[q] = Uhalf[q * NC + c];
            cons2prim(o, u, v, NULL);
            for (int q = 0; q < NVAR; q++) Vhalf[q * NC + c] = v[q];
        }
        ORC_STAGE(5);
        for (int d = 0; d < dim; d++) {
            int flo[3], fhi[3];
            for (int e = 0; e < 3; e++) { flo[e] = lo[e]; fhi[e] = hi[e]; }
            fhi[d] = hi[d] + 1;
#pragma omp parallel for collapse(2) schedule(static)
            for (int k = flo[2]; k < fhi[2]; k++)
                for (int j = flo[1]; j < fhi[1]; j++)
                    for (int i = flo[0]; i < fhi[0]; i++) {
                        long cB = cidx(&g, i, j, k);
                        double Pi[NVAR];
                        parab_flux(o, &g, Vhalf, Uhalf, i, j, k, d, pfL[d * NC + cB], pfR[d * NC + cB],
                                   rfL[d * NC + cB], rfR[d * NC + cB], Pi);
                        for (int q = 0; q < NVAR; q++) Ph[(d * NVAR + q) * NC + cB] = Pi[q];
                    }
        }
    }

    ORC_STAGE(6);

    /* 7. conservative update (Eq. update), directions summed in order */
    memcpy(U_out, U_in, sizeof(double) * NVAR * NC);
    double rate = 0.0, dpp = 0.0;
    double dxmin = o->dx[0];
    for (int e = 1; e < dim; e++) dxmin = fmin(dxmin, o->dx[e]);
#pragma omp parallel for collapse(2) schedule(static) reduction(max : rate, dpp)
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++) {
                long c = cidx(&g, i, j, k);
                double u[NVAR];
                for (int q = 0; q < NVAR; q++) {
                    double s = 0.0;
                    for (int d = 0; d < dim; d++) {
                        long cp = cidx(&g, i + offs[d][0], j + offs[d][1], k + offs[d][2]);
                        double dF = Fh[(d * NVAR + q) * NC + cp] - Fh[(d * NVAR + q) * NC + c];
                        double dP = Ph[(d * NVAR + q) * NC + cp] - Ph[(d * NVAR + q) * NC + c];
                        s += (dF - dP) / o->dx[d];
                    }
                    u[q] = U_in[q * NC + c] - dt * s;
                }
                /* 8. operator-split point-local sources */
                if (o->glm) u[PSI] *= exp(-o->glm_alpha * ch * dt / dxmin);
                if (o->cooling && L0) {
                    double v[NVAR];
                    cons2prim(o, u, v, NULL);
                    double T = v[PRS] / v[RHO];
                    double beta = o->cool_beta;
                    if (T > o->T_floor) {
                        double x = pow(T, 1.0 - beta) - (1.0 - beta) * (o->gamma - 1.0) * v[RHO] * L0[c] * dt;
                        double xf = pow(o->T_floor, 1.0 - beta);
                        if (x < xf) x = xf;
                        double Tn = pow(x, 1.0 / (1.0 - beta));
                        double pn = v[RHO] * Tn;
                        u[ENG] += (pn - v[PRS]) / (o->gamma - 1.0);
                        if (!leaf || leaf[c]) dpp = fmax(dpp, fabs(pn - v[PRS]) / v[PRS]);
                    }
                }
                for (int q = 0; q < NVAR; q++) U_out[q * NC + c] = u[q];

                /* 9. CFL rate (Eq. Ca) */
                double lmax = 0.0;
                for (int d = 0; d < dim; d++) {
                    long cp = cidx(&g, i + offs[d][0], j + offs[d][1], k + offs[d][2]);
                    double lc = fmax(lamf[d * NC + c], lamf[d * NC + cp]);
                    lmax = fmax(lmax, lc / o->dx[d]);
                }
                double r = lmax;
                if (par) {
                    double vh[NVAR];
                    for (int q = 0; q < NVAR; q++) vh[q] = Vhalf[q * NC + c];
                    double D = diff_coeff(o, vh);
                    for (int d = 0; d < dim; d++) r += 2.0 * D / (o->dx[d] * o->dx[d]);
                }
                rate = fmax(rate, r);
            }

    if (face_flux) {
        memset(face_flux, 0, sizeof(double) * dim * NVAR * NC);
        for (int d = 0; d < dim; d++) {
            int rlo[3], rhi[3];
            for (int e = 0; e < 3; e++) { rlo[e] = lo[e]; rhi[e] = hi[e]; }
            rhi[d] = hi[d] + 1;
            for (int k = rlo[2]; k < rhi[2]; k++)
                for (int j = rlo[1]; j < rhi[1]; j++)
                    for (int i = rlo[0]; i < rhi[0]; i++) {
                        long c = cidx(&g, i, j, k);
                        for (int q = 0; q < NVAR; q++)
                            face_flux[(d * NVAR + q) * NC + c] =
                                dt * (Fh[(d * NVAR + q) * NC + c] - Ph[(d * NVAR + q) * NC + c]);
                    }
        }
    }
    ORC_STAGE(7);
    if (out_scalars) { out_scalars[0] = rate; out_scalars[1] = dpp; }
    if (fails) for (int k = 0; k < NFAIL; k++) fails[k] += lf[k];

    free(flag);
    free(V); free(Fn); free(Pn); free(Ln); free(LPn); free(Uhm); free(Uhp); free(Fh); free(Ph);
    free(PVm); free(PVp);
    free(lamf); free(pfL); free(pfR); free(rfL); free(rfR); free(Uhalf); free(Vhalf);
    return 0;
}

/* CFL rate from cell-centred states: max over cells of max_d (|v_d| + c_f)/dx_d
 * for MHD, max_d max(|lambda_-|, |lambda_+|)/dx_d for RMHD, plus the
 * diffusion term of Eq. Ca.  Interior cells only. */
double orc_cfl_rate(const orc_opts *o, int nx, int ny, int nz, int ng, const double *U)
{
    int gz = (o->dim == 3) ? ng : 0;
    grid_t g;
    g.NX = nx + 2 * ng;
    g.NY = ny + 2 * ng;
    g.NZ = nz + 2 * gz;
    g.NC = (long)g.NX * g.NY * g.NZ;
    double rate = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(max : rate)
    for (int k = gz; k < gz + nz; k++)
        for (int j = ng; j < ng + ny; j++)
            for (int i = ng; i < ng + nx; i++) {
                long c = cidx(&g, i, j, k);
                double u[NVAR], v[NVAR];
                for (int q = 0; q < NVAR; q++) u[q] = U[q * g.NC + c];
                cons2prim(o, u, v, NULL);
                double r = 0.0;
                for (int d = 0; d < o->dim; d++) {
                    double lm, lp;
                    signal_speeds(o, v, d, &lm, &lp);
                    r = fmax(r, fmax(fabs(lm), fabs(lp)) / o->dx[d]);
                }
                double D = diff_coeff(o, v);
                for (int d = 0; d < o->dim; d++) r += 2.0 * D / (o->dx[d] * o->dx[d]);
                rate = fmax(rate, r);
            }
    return rate;
}

/* Riemann solves counted since the last reset (reset != 0 clears it after
 * reading). */
long orc_riemann_count(int reset)
{
    long n;
#pragma omp atomic read
    n = orc_nsolve;
    if (reset) {
#pragma omp atomic write
        orc_nsolve = 0;
    }
    return n;
}

/* Threads used by the OpenMP loops of the next calls (n <= 0: the OpenMP
 * default of the process, OMP_NUM_THREADS or every core); returns the count
 * in force. */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_set_threads(int n)
{
#ifdef _OPENMP
    static int deflt = 0;
    if (deflt == 0) deflt = omp_get_max_threads();
    omp_set_num_threads(n > 0 ? n : deflt);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
