/*
 * ctu.h -- C ABI of the MI355X (gfx950) CTU-GLM step library (libctu.so).
 *
 * One call advances every patch of a batch by one dimensionally unsplit
 * Corner Transport Upwind step with GLM divergence cleaning, as defined in
 * Mignone et al. (ApJS 2012), Sec. 3.1 (Eq. update, ctu_flux, transv, Ca):
 * a conserved state U on ghosted boxes, dt, the EOS and the solver options
 * go in; the updated interior U, fine/coarse flux-register increments and the
 * maximum signal rate of Eq. Ca come out.  Ghost zones are filled by the
 * caller (Sec. 4: physical boundaries, same-level exchange, coarse
 * interpolation).
 *
 * Conventions shared by every entry point
 *  - A plan (and a hierarchy) belongs to one HIP device, named at creation;
 *    each call on it makes that device current for its duration and then
 *    restores the caller's current device.  Streams passed with a plan must
 *    belong to its device.
 *  - All pointers named *_dev are device pointers (hipMalloc / torch CUDA
 *    tensors) owned by the caller; the library never frees them.
 *  - Host pointers (options, box and register tables) are read during the
 *    call only.
 *  - Calls are asynchronous on the given HIP stream (NULL = default
 *    stream); results are valid after the stream is synchronised.
 *  - Every function returns a ctu_status: 0 on success, < 0 on a
 *    synchronous error (bad argument, unsupported option combination, HIP
 *    launch or allocation failure).  ctu_last_error() then returns a
 *    message (thread-local).  Physical failures inside kernels never abort:
 *    they are counted (see ctu_step).
 *  - A plan is used by one stream at a time: calls that overlap on two
 *    streams with the same plan race on its workspace.
 *
 * Variables (9 per cell, SoA):
 *   conserved   (rho | D, m_x, m_y, m_z, E, B_x, B_y, B_z, psi)
 *   primitive   (rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi)
 * MHD (Sec. 2.1): E = p/(Gamma-1) + rho v^2/2 + B^2/2.
 * RMHD (Sec. 2.2): D = rho gamma, m = w gamma^2 v + E x B,
 *   E = w gamma^2 - p + (B^2 + E_field^2)/2 - D, w = rho + Gamma p/(Gamma-1).
 *
 * State layout: box b occupies elements [offset_b, offset_b + 9*NX*NY*NZ)
 * of the state array as q[v][k][j][i] (i fastest) over its ghosted extent
 * NX = n_x + 2g, NY = n_y + 2g, NZ = n_z + 2g (NZ = n_z = 1 in 2D).  The
 * element type is double for CTU_FP64 and float for CTU_FP32.
 */
#ifndef CTU_H
#define CTU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ctu_status;
enum {
    CTU_OK = 0,
    CTU_ERR_ARG = -1,         /* invalid argument or table entry */
    CTU_ERR_UNSUPPORTED = -2, /* option combination not implemented */
    CTU_ERR_HIP = -3,         /* HIP runtime error (launch, copy) */
    CTU_ERR_NOMEM = -4        /* device allocation failed */
};

typedef enum { CTU_MHD = 0, CTU_RMHD = 1 } ctu_physics;
/* FP32: state, reconstruction, Riemann solves and update in float; the RMHD
 * conserved-to-primitive inversion, the CFL maximum and the flux registers
 * stay in double.  FP64: everything in double. */
typedef enum { CTU_FP64 = 0, CTU_FP32 = 1 } ctu_precision;
/* Sec. 3.2: linear with the MC (Eq. MClim), MinMod (Eq. minmod), harmonic
 * (Eq. harmonic_lim) or van Albada (Eq. vanalbada_lim) limiter; PPM (Eq.
 * ppm1 + Eq. ppm_parabolic_lim); improved WENO3 (Eq. WENO3, WENO3a). */
typedef enum {
    CTU_LIN_MC = 0, CTU_LIN_MINMOD = 1, CTU_LIN_VANLEER = 2, CTU_LIN_VANALBADA = 3,
    CTU_PPM = 4, CTU_WENO3 = 5
} ctu_recon;
/* Sec. 3.2 characteristic tracing (MHD only) or Sec. 3.3 MUSCL-Hancock
 * (linear reconstructions only; the RMHD predictor). */
typedef enum { CTU_PRED_CHAR = 0, CTU_PRED_MUSCL_HANCOCK = 1 } ctu_predictor;
/* Reference state of Eq. wnorm_predp/m: w_ref = w_{i,+-} (FACE, default),
 * w_{i,0} (CELL) or the nu_max / nu_min form (CW84). */
typedef enum { CTU_WREF_FACE = 0, CTU_WREF_CELL = 1, CTU_WREF_CW84 = 2 } ctu_wref;
/* Sec. 3.1: HLLD (MHD: Miyoshi & Kusano; RMHD: Mignone, Ugliano & Bodo 2009,
 * with a secant iteration on the total pressure and HLLC where its fan is not
 * admissible), HLL (MHD, RMHD), Rusanov, the local Lax-Friedrichs
 * flux (F_L + F_R)/2 - a (U_R - U_L)/2 with a the largest signal speed
 * magnitude of the two states (MHD, RMHD), HLLC (MHD: one contact at the
 * HLL-averaged normal velocity with the HLL-averaged transverse field in
 * both star states; RMHD: the contact speed from the quadratic of Mignone &
 * Bodo 2006 on the HLL averages, HLL where the star state is not
 * admissible), or Roe (MHD), the
 * linearised solver on the Cargo-Gallice averages (exact jump property,
 * seven waves, no entropy fix).  Rusanov, HLLC and Roe are not available
 * with shock_eps > 0. */
typedef enum { CTU_HLLD = 0, CTU_HLL = 1, CTU_RUSANOV = 2, CTU_HLLC = 3, CTU_ROE = 4 } ctu_riemann;

/* Sec. 2.2: the RMHD gas enthalpy w(rho, p) of the ideal EOS (Eq. gammaEos,
 * w = rho + Gamma p / (Gamma - 1)) or of the Taub-Matthews EOS (Eq. TMEos,
 * w = 5p/2 + sqrt(9p^2/4 + rho^2); gamma is then unused). */
typedef enum { CTU_EOS_IDEAL = 0, CTU_EOS_TM = 1 } ctu_eos;

/* Sec. 3.1 corner coupling of the face states: TN, Eq. transv with the
 * transverse increments of first-order Riemann fluxes between the t^n cell
 * states (every option set; the default), or MT, for runs without parabolic
 * terms, with the transverse increments of Riemann fluxes between the
 * normal-predictor states of the two cells of each face (the form the paper
 * takes from Mignone & Tzeferacos 2010 when Pi = 0; needs nghost >= 3, no
 * shock_eps, hyperbolic fluxes on). */
typedef enum { CTU_CORNER_TN = 0, CTU_CORNER_MT = 1 } ctu_corner;

#define CTU_PARAB_VISC 1u /* Eq. visc_tens */
#define CTU_PARAB_RES 2u  /* resistive term -curl(eta J) */
#define CTU_PARAB_TC 4u   /* Eq. tc_flux with the App. A saturated flux */

#define CTU_NFAIL 5 /* failure counters: rho<=0, p<=0, RMHD inversion, |v|>=1, NaN */

typedef struct {
    int32_t dim;           /* 2 or 3 (vectors always have 3 components) */
    int32_t physics;       /* ctu_physics */
    int32_t precision;     /* ctu_precision */
    int32_t recon;         /* ctu_recon */
    int32_t predictor;     /* ctu_predictor */
    int32_t wref;          /* ctu_wref */
    int32_t riemann;       /* ctu_riemann */
    int32_t glm;           /* 1: GLM cleaning (Eq. glm2x2); 0: B_n averaged at faces */
    double gamma;          /* specific heat ratio of the ideal EOS */
    double dx[3];          /* level-0 cell size; a box on level l uses dx / 2^l */
    double glm_alpha;      /* psi damping: psi *= exp(-alpha c_h dt / min dx) */
    uint32_t parabolic_mask; /* CTU_PARAB_* bits; 0 = no parabolic terms */
    int32_t cooling;       /* 1: optically thin cooling source (needs cool_L0) */
    double nu, eta;        /* kinematic viscosity, scalar resistivity */
    double kappa_par, kappa_perp; /* conduction coefficients along / across B */
    double tc_phi;         /* saturation parameter phi; <= 0: classical flux */
    double cool_beta;      /* Lambda = L0 rho^2 T^beta for T > T_floor, T = p/rho */
    double T_floor;
    int32_t hyperbolic_off; /* 1: skip hyperbolic fluxes (isolates Pi / sources) */
    int32_t pad;
    double shock_eps;      /* App. B shock detection threshold eps_q (5 is the paper's
                              default); 0 = off.  Zones with sum_d |p_{+1} - p_{-1}| /
                              min(p_{+1}, p_{-1}) > eps_q and div v < 0 at t^n take HLL
                              on their faces; zones whose reconstruction stencil along
                              an axis reaches one use MinMod linear reconstruction */
    int32_t eos;           /* ctu_eos: RMHD equation of state (MHD: CTU_EOS_IDEAL only) */
    int32_t exact_speeds;  /* RMHD signal speeds of HLL / Rusanov and the CFL rate: 0 = the
                              isotropic bound (a^2 = cs^2 + ca^2 - cs^2 ca^2 with relativistic
                              velocity addition), 1 = the exact fast magnetosonic speeds (the
                              outermost roots of the dispersion quartic); ignored for MHD,
                              whose fast speeds are exact */
    int32_t corner;        /* ctu_corner */
    int32_t pad2;
} ctu_opts;

/* One ghosted box: interior cells [lo, lo+n) in level-global indices.
 * Its block of nine ghosted planes must fit in 4 GiB (FP32: at most
 * 119,304,647 ghosted cells, FP64: 59,652,323); larger grids are split
 * into several boxes.  ctu_plan_create rejects a larger box (CTU_ERR_ARG). */
typedef struct {
    int32_t lo[3];
    int32_t n[3];   /* n[2] = 1 in 2D */
    int32_t level;  /* refinement level (cell size dx / 2^level) */
    int32_t pad;
    int64_t offset; /* element offset of the box's block in the state arrays */
} ctu_box;

/* A rectangle of faces of one box whose dt*A*(F - Pi) is accumulated into
 * the FP64 register array (Sec. 4, Eq. fluxcorr): the faces normal to
 * direction dir at level-global face index `face` (the face between cells
 * face-1 and face), covering transverse cells [tlo, tlo+tn) in the two other
 * directions (ordered by increasing direction index; in 2D tn[1] = 1).
 * Face (t0, t1) owns the 9 doubles at reg[9 * (slot + t1*tn[0] + t0) + v]. */
typedef struct {
    int32_t box, dir, face, pad;
    int32_t tlo[2], tn[2];
    int64_t slot;
} ctu_regface;

/* One coarse cell that receives a flux correction (Eq. addreflux):
 * U_coarse[cell] += -side * (sum of fine register slots - coarse slot) / V,
 * with V the coarse cell volume (so A/V = 1/dx_dir on the coarse level).
 * side = +1 when the refined region lies on the cell's high face along the
 * correction direction, -1 on its low face.  Several entries may name the
 * same cell; they are applied by one thread per cell in table order. */
typedef struct ctu_refluxface {
    int32_t box;        /* coarse box */
    int32_t i, j, k;    /* ghosted-local cell index inside that box */
    int32_t dir;        /* direction normal to the corrected face */
    int32_t side;       /* +1 / -1 */
    int32_t nfine;      /* number of fine slots (r^(dim-1), at most 4) */
    int32_t pad;
    int64_t coarse_slot;
    int64_t fine_slot[4];
} ctu_refluxface;

typedef struct ctu_plan ctu_plan;

/* ctu_plan_create_ex flags.
 * CTU_PLAN_CALLER_WORKSPACE: the library allocates no workspace; the caller
 *   supplies it with ctu_plan_set_workspace before the first step.
 * CTU_PLAN_LEVEL_DT: one plan over the boxes of several refinement levels
 *   (Sec. 4, ratio 2): params {dt, c_h} give the level-0 step, a box of
 *   level l steps by dt / 2^l (c_h, the same on every level for ratio 2, is
 *   shared), and the rate output is the largest rate / 2^l (the level-0 rate
 *   of the boxes' CFL numbers), so one launch chain advances every patch of
 *   the hierarchy by its own level step. */
#define CTU_PLAN_CALLER_WORKSPACE 1u
#define CTU_PLAN_LEVEL_DT 2u

/* Create a plan for a batch of boxes on HIP device hip_device (Sec. 3.1
 * applied to each patch of a level; Sec. 4 states the per-patch problem:
 * advance one patch by dt with ghost zones filled by the caller).
 * Validates the options, uploads the box, register and (optional, reflux /
 * nreflux, as for ctu_plan_set_reflux) reflux tables, reserves the tile
 * tables of every launch shape and, unless flags has
 * CTU_PLAN_CALLER_WORKSPACE, allocates the device workspace.  This is the
 * call that allocates; steps, launches, shape changes and the autotuner do
 * not.  nghost must be >= 3 (PPM needs 3, parabolic terms one more); box
 * blocks must not overlap.  Returns CTU_ERR_ARG for a device out of range
 * or unknown flags, CTU_ERR_UNSUPPORTED for PPM/WENO3 with MUSCL-Hancock,
 * characteristic tracing with RMHD, parabolic/cooling terms with RMHD, Roe
 * with RMHD, or the shock-adaptive hybrid with the Rusanov, HLLC or Roe
 * solver, CTU_ERR_NOMEM when an allocation fails. */
ctu_status ctu_plan_create_ex(int32_t hip_device, uint32_t flags, const ctu_opts *opts, const ctu_box *boxes,
                              int32_t nbox, int32_t nghost, const ctu_regface *regfaces, int32_t nreg,
                              const struct ctu_refluxface *reflux, int32_t nreflux, ctu_plan **plan_out);
/* ctu_plan_create_ex on the current device, library-owned workspace, no
 * reflux table. */
ctu_status ctu_plan_create(const ctu_opts *opts, const ctu_box *boxes, int32_t nbox, int32_t nghost,
                           const ctu_regface *regfaces, int32_t nreg, ctu_plan **plan_out);
void ctu_plan_destroy(ctu_plan *plan);
/* The plan's HIP device (-1 for a null plan). */
int32_t ctu_plan_device(const ctu_plan *plan);

/* Number of state elements the plan addresses: max over boxes of
 * offset + 9*NX*NY*NZ.  Bytes of device workspace the plan's option set
 * needs (held by the plan, or to be supplied by the caller): V^n and the
 * three corner-coupling increments T_d (9 values per ghosted cell each; in
 * the state's element type), with parabolic terms V^{n+1/2}, one rate per
 * cell and 8 parabolic face-flux values per face (one face per direction and
 * ghosted cell), with the MT corner coupling three predictor-flux fields, with
 * the App. B hybrid one flag byte per cell, each field 256-byte aligned. */
int64_t ctu_plan_state_elems(const ctu_plan *plan);
int64_t ctu_plan_workspace_bytes(const ctu_plan *plan);

/* Give a plan created with CTU_PLAN_CALLER_WORKSPACE its workspace: ws_dev
 * on the plan's device, 256-byte aligned, at least
 * ctu_plan_workspace_bytes; it stays owned by the caller, who keeps it
 * alive and unused by anything else while the plan steps.  May be called
 * again to move the plan to another buffer (waits for the device first).
 * Drops a captured graph.  CTU_ERR_ARG for a null, short or misaligned
 * buffer or a plan that owns its workspace.  Steps of a plan without a
 * workspace return CTU_ERR_ARG. */
ctu_status ctu_plan_set_workspace(ctu_plan *plan, void *ws_dev, int64_t bytes);

/* One CTU step (Sec. 3.1) of every box of the plan.
 *  U_in_dev   : state at t^n with ghosts filled (read only)
 *  U_out_dev  : receives U^{n+1} in every interior cell; ghost cells are left
 *               untouched; must not alias U_in_dev
 *  params_dev : device doubles {dt, c_h}; read by the kernels at run time, so
 *               a captured graph can be replayed with new values
 *  cool_L0_dev: per-cell cooling coefficient on the state layout (one
 *               element per cell, no variable index; same element type as
 *               the state), required when opts.cooling, else may be NULL
 *  reg_dev    : FP64 register array, accumulated (+=), NULL if nreg == 0
 *  rate_dev   : one double, set to the maximum over interior cells of
 *               max_d(lambda_d/dx_d) + sum_d 2 D/dx_d^2 (Eq. Ca); the next
 *               step is dt = C_a / rate
 *  dpp_dev    : one double, max |dp/p| of the cooling step (Eq. dt_cool), or NULL
 *  fails_dev  : CTU_NFAIL int32 counters, zeroed then incremented per failing
 *               conversion, or NULL */
ctu_status ctu_step(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                    const void *cool_L0_dev, double *reg_dev, double *rate_dev, double *dpp_dev,
                    int32_t *fails_dev, void *stream);

/* ctu_step without a workspace of the plan's: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Arguments, results and errors
 * are those of ctu_step; the plan may have been created with
 * CTU_PLAN_CALLER_WORKSPACE and never given one.  The workspace is instead
 * a fixed array of ctu_static_scratch_bytes() (64 MiB) that the library
 * holds on every GPU it runs on until the process ends; a plan whose
 * ctu_plan_workspace_bytes exceeds it is refused with CTU_ERR_ARG (its boxes
 * must be stepped with ctu_step or split into smaller plans).  The call
 * allocates nothing.  All calls on one GPU share that GPU's array, which
 * keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap on one GPU, on any streams or plans, race, so callers
 * serialise them (one stream, or events between streams). */
ctu_status ctu_step_static(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                           const void *cool_L0_dev, double *reg_dev, double *rate_dev, double *dpp_dev,
                           int32_t *fails_dev, void *stream);
/* Bytes of the fixed per-GPU array of ctu_step_static. */
int64_t ctu_static_scratch_bytes(void);

/* Launch shape of a plan's t^n and sweep kernels.  The per-cell arithmetic
 * does not depend on it: every shape gives the same results (bitwise in
 * FP64), only the speed differs.
 *  tc_layout : in-plane layout of the t^n kernel's blocks:
 *              CTU_TC_TILES   32 x 8 rectangles (256 x 1 in 2D);
 *              CTU_TC_FLAT    256 consecutive positions of each box's plane,
 *                             row by row (3D boxes with n[0] <= 37; others
 *                             keep the rectangles);
 *              CTU_TC_AUTO    per box, the one that needs fewer blocks
 *  tc_chunk  : planes per t^n block along the marching axis, 1..4096; 0 = 16
 *  x_pencils : x-sweep pencils per block, 1..64; 0 = the count that idles
 *              the fewest lanes
 *  xcd_order : 1 = launch order that gives each XCD a contiguous run of
 *              tiles (halo lines shared in one L2); 0 = place order
 *  yz_segments: blocks per y- and z-sweep column of 64 pencils, 1..8
 *              (0 = 1): each block updates a run of the line's cells and
 *              first recomputes the two predicted states below its run, so
 *              results do not depend on it; more, shorter blocks leave fewer
 *              compute units with a single block at the end of a launch */
typedef enum { CTU_TC_AUTO = 0, CTU_TC_TILES = 1, CTU_TC_FLAT = 2 } ctu_tc_layout;
typedef struct {
    int32_t tc_layout;
    int32_t tc_chunk;
    int32_t x_pencils;
    int32_t xcd_order;
    int32_t yz_segments;
} ctu_shape;

/* Rebuild the plan's tables for a shape (CTU_ERR_ARG for a field out of
 * range), in the buffers reserved at creation (no allocation; waits for the
 * device first, as a step in flight reads the tables); drops a captured
 * graph, which must be captured again.  A new plan starts with {AUTO, 0, 0, 1, 0}, or with the
 * shape that ctu_plan_autotune found for the same option set and box
 * extents earlier in the process. */
ctu_status ctu_plan_set_shape(ctu_plan *plan, const ctu_shape *shape);
/* The shape in use, and (if flat_boxes_out) how many boxes use the flat
 * t^n layout under it. */
ctu_status ctu_plan_get_shape(const ctu_plan *plan, ctu_shape *shape_out, int32_t *flat_boxes_out);

/* Measure candidate shapes on the caller's data and keep the fastest: the
 * t^n layout and chunk (4, 8, 16, 32), then the x-sweep pencils per block
 * (16, 8, 32, 4, auto),
 * then the y / z sweep segments (1, 2, 3, 4), then the launch order, one
 * coordinate at a time, starting from the plan's
 * shape; a candidate replaces the incumbent only when it is more than 1 %
 * faster.  Each candidate runs 1 + reps
 * steps of U_in_dev into U_out_dev on the stream (U_out_dev is overwritten;
 * no registers, rate, dpp or failure counts are written), timed with HIP
 * events; the call synchronizes the stream.  The winner is applied (as by
 * ctu_plan_set_shape), cached for plans of the same option set and box
 * extents created later in the process, and returned with its time per
 * step in ms.  cool_L0_dev is required when opts.cooling.  Allocates
 * nothing (its events and every shape's tables exist from creation). */
ctu_status ctu_plan_autotune(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                             const void *cool_L0_dev, int32_t reps, void *stream, ctu_shape *best_out,
                             double *best_ms_out);
/* Forget every shape found by ctu_plan_autotune in this process. */
ctu_status ctu_tune_cache_clear(void);

/* Capture ctu_step with the given arguments into a HIP graph owned by the
 * plan (replacing a previous one), and replay it.  The graph holds no
 * memset nodes; buffers are re-zeroed by kernels on every replay. */
ctu_status ctu_step_graph_capture(ctu_plan *plan, const void *U_in_dev, void *U_out_dev,
                                  const double *params_dev, const void *cool_L0_dev, double *reg_dev,
                                  double *rate_dev, double *dpp_dev, int32_t *fails_dev, void *stream);
ctu_status ctu_step_graph_launch(ctu_plan *plan, void *stream);

/* Signal rate of Eq. Ca from cell-centred states (for the first dt):
 * max over interior cells of max_d(|lambda_d|max / dx_d) + diffusion term. */
ctu_status ctu_cfl_rate(ctu_plan *plan, const void *U_dev, double *rate_dev, void *stream);

/* Elementwise maps over every ghosted cell of every box: primitive ->
 * conserved and conserved -> primitive (Sec. 2; RMHD inversion in FP64). */
ctu_status ctu_prim_to_cons(ctu_plan *plan, const void *V_dev, void *U_dev, void *stream);
ctu_status ctu_cons_to_prim(ctu_plan *plan, const void *U_dev, void *V_dev, int32_t *fails_dev, void *stream);

/* Refluxing at level synchronisation (Eq. fluxcorr, Eq. addreflux).
 * ctu_plan_set_reflux uploads (and groups per coarse cell) a table of
 * corrections for the boxes of this (coarse) plan, replacing any previous
 * table (the one given to ctu_plan_create_ex included); a setup call that
 * allocates device memory and waits for the device.  ctu_reflux applies them to the coarse
 * state in FP64 arithmetic; reg_dev holds both the coarse slots (dt*A*F of
 * the coarse step) and the fine slots (dt*A*F summed over the fine
 * substeps) that the table names. */
ctu_status ctu_plan_set_reflux(ctu_plan *coarse_plan, const ctu_refluxface *faces, int32_t nfaces);
ctu_status ctu_reflux(ctu_plan *coarse_plan, void *U_dev, const double *reg_dev, void *stream);

/* As ctu_reflux, then clears every register slot the table read (each slot
 * belongs to one face, hence to one corrected cell), ready for the next
 * accumulation; slots the table does not name are left as they are. */
ctu_status ctu_reflux_consume(ctu_plan *coarse_plan, void *U_dev, double *reg_dev, void *stream);

/* ---- AMR level cycle (Sec. 4) -------------------------------------------
 *
 * A hierarchy of boxes on a periodic cube of `base` level-0 cells per side
 * with refinement ratio 2: level l has base * 2^l cells per side.
 * level_nbox[l] boxes of level l follow each other in `boxes` (level-global
 * indices, `level` = l, `offset` = element offset of the box block in that
 * level's state array, the layout of ctu_plan_create).  3D only.  Checked at
 * creation (CTU_ERR_ARG): boxes inside their level, 2-aligned (even lo and n)
 * on levels >= 1, disjoint per level, level 0 covering the domain, every
 * fine box inside the coarser level's interiors, each box block below 4 GiB.
 * The ghost-fill tables are built on the host and uploaded once: per box,
 * the rectangles of its ghost cells that same-level interiors hold (under
 * the periodic shifts), and on levels >= 1 the coarse parents of the other
 * ghost cells with the coarse boxes holding their 7-cell stencils; also the
 * coarse boxes under each fine box for restriction.  Creation is the only
 * allocating call.  The hierarchy belongs to the device current at
 * creation; its plans must too. */
typedef struct ctu_hier ctu_hier;
ctu_status ctu_hier_create(int32_t precision, int32_t base, int32_t nlev, const int32_t *level_nbox,
                           const ctu_box *boxes, int32_t nghost, ctu_hier **out);
void ctu_hier_destroy(ctu_hier *hier);

/* Fill every ghost cell of every box of `level` in U_dev (that level's state
 * array; interiors are read, ghosts written).  A ghost cell whose periodic
 * image lies in a box interior of the same level is copied from it (level 0:
 * always).  Otherwise it is prolonged (Eq. prolong, ratio 2: the parent
 * value plus -+1/4 of the monotonised-central slope of the parent and its
 * face neighbours per direction, Eq. MClim) from the coarse state
 * (1 - alpha) Uc_old + alpha Uc_new (Eq. intalpha), read from coarse box
 * interiors only; alpha in [0, 1], Uc_new may be null when alpha = 0.  A
 * cell whose coarse stencil leaves the coarse interiors (insufficient
 * nesting) is set to NaN and counted in *missing_dev (nullable). */
ctu_status ctu_hier_fill_ghosts(ctu_hier *hier, int32_t level, void *U_dev, const void *Uc_old_dev,
                                const void *Uc_new_dev, double alpha, int32_t *missing_dev, void *stream);

/* Eq. avgdown (ratio 2, equal Cartesian volumes): every coarse cell under a
 * box interior of `fine_level` becomes the mean of its 8 children. */
ctu_status ctu_hier_average_down(ctu_hier *hier, int32_t fine_level, const void *U_fine_dev, void *U_coarse_dev,
                                 void *stream);

/* Leaf mask of `level` (one byte per ghosted cell, at offset / 9 of each box,
 * the layout of cool_L0): 1 on interior cells that no box of the next finer
 * level covers, 0 on covered and ghost cells. */
ctu_status ctu_hier_leaf_mask(ctu_hier *hier, int32_t level, uint8_t *leaf_dev, void *stream);

/* Refinement criterion (Eq. RefCrit, second-derivative error norm) with
 * sigma = conserved variable `var` of U_dev (ghosts filled), undivided
 * differences, sigma_ref,d = |s_{+1}| + 2|s_0| + |s_{-1}| weighted by eps;
 * evaluated in FP64, chi = 0 where its denominator vanishes.  tags_dev (the
 * layout of ctu_hier_leaf_mask) receives 1 on interior cells with
 * chi > chi_r and 0 on the other interior cells; *ntag_dev (nullable) is
 * increased by the number of tagged cells. */
ctu_status ctu_hier_tag(ctu_hier *hier, int32_t level, const void *U_dev, int32_t var, double eps, double chi_r,
                        uint8_t *tags_dev, int32_t *ntag_dev, void *stream);

/* Next level steps on the device (Eq. Ca, Eq. dt_cool, Eq. level_dt):
 * dt_l = min(cfl / rate_dev[l], eps_c dt_l / dpp_dev[l]) with dt_l read from
 * params_dev[l][0] (the cooling term only where dpp > 0; dpp_dev nullable),
 * dt_0 = min_l 2^l dt_l, and params_dev[l][0] <- dt_0 / 2^l (c_h in
 * params_dev[l][1] is left as it is).  One thread; no allocation. */
ctu_status ctu_hier_next_dt(ctu_hier *hier, const double *rate_dev, const double *dpp_dev, double cfl, double eps_c,
                            double *const *params_dev, void *stream);

/* Restrict the cooling time-step estimate of a plan's steps (dpp_dev of
 * ctu_step) to the cells whose byte in leaf_dev is nonzero (Sec. 4.2: the
 * source-term time step counts on leaf cells only); leaf_dev uses the layout
 * of cool_L0 and stays owned by the caller; null restores every cell.  The
 * cooling itself is applied on every cell. */
ctu_status ctu_plan_set_leaf_mask(ctu_plan *plan, const uint8_t *leaf_dev);

/* One level-0 step of the whole hierarchy with time subcycling (Sec. 4):
 * level l is filled (level 0 periodically; level l >= 1 at alpha = 0 and
 * 1/2 of its parent's step), advanced by ctu_step with plans[l], then level
 * l+1 takes two substeps, is averaged down into level l, and level l is
 * refluxed with ctu_reflux_consume.  plans[l] holds level l's boxes in the
 * same order and offsets, with its register faces and reflux table (the
 * caller builds both); params_dev[l] = {dt_l, c_h} on the device with
 * dt_l = dt_0 / 2^l.  Each level has two state arrays U_a[l], U_b[l];
 * cur[l] (host, 0 or 1) names the one holding the current state and is
 * updated on return.  cool_L0_dev (nullable; else per level, entries
 * nullable) gives each level's cooling coefficients.  reg_dev (FP64
 * registers, zero on the first call) is left with every slot it read
 * cleared.  rate_dev[l] / dpp_dev[l] (dpp nullable) receive the CFL rate and
 * max |dp/p| of level l's last substep; fails_dev[5] (nullable) accumulates
 * the failure counts of every step; missing_dev (nullable) as above.
 * Asynchronous on `stream`; allocation-free. */
ctu_status ctu_hier_advance(ctu_hier *hier, ctu_plan *const *plans, void *const *U_a, void *const *U_b,
                            int32_t *cur, const double *const *params_dev, const void *const *cool_L0_dev,
                            double *reg_dev, double *rate_dev, double *dpp_dev, int32_t *fails_dev,
                            int32_t *missing_dev, void *stream);

/* Per-stage kernel timing with HIP events recorded on the launch stream
 * around each kernel of ctu_step (eager launches only, not inside captured
 * graphs).  Enabling (re)starts the accumulation; up to 256 steps are
 * recorded.  The first enable creates the events (a profiling setup call).  ctu_plan_read_timing synchronises on the recorded events and
 * writes the total milliseconds per stage into ms_out[CTU_NSTAGE] and the
 * number of recorded steps into nsteps_out.  Stages: 0 primitive recovery,
 * 1 the t^n fluxes and transverse increments (with the half step), 2 and 3
 * the parabolic face fluxes of V^n and of V^{n+1/2} (parabolic runs), 4
 * unused, 5-7 direction sweeps x/y/z. */
#define CTU_NSTAGE 8
ctu_status ctu_plan_enable_timing(ctu_plan *plan, int32_t enable);
ctu_status ctu_plan_read_timing(ctu_plan *plan, double *ms_out, int32_t *nsteps_out);

/* Measurement helpers (not part of the step): the rates this build reaches
 * on the current device, for quoting roofline fractions against measured as
 * well as published peaks.  Both launch on the null stream and synchronise;
 * they create two HIP events (no device allocation).
 * ctu_measure_fma: nblocks x 256 threads, each running eight independent FMA
 * chains for iters x 16 steps (FP32: single-lane FMAs, as every kernel of
 * this build, which emits no packed FP32); out_dev holds nblocks * 256
 * elements of the precision (written, values meaningless); *tflops_out =
 * 2 FLOP per FMA over the timed launches.
 * ctu_measure_copy: a float4 device-to-device copy of `bytes` (a multiple of
 * 16) from src_dev to dst_dev, ten timed launches; *gbs_out = bytes read plus
 * bytes written per second, in GB/s. */
ctu_status ctu_measure_fma(int32_t precision, int32_t nblocks, int32_t iters, void *out_dev, double *tflops_out);
ctu_status ctu_measure_copy(const void *src_dev, void *dst_dev, int64_t bytes, double *gbs_out);

const char *ctu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CTU_H */
