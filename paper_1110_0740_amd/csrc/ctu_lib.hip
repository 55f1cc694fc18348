// ctu_lib.hip -- host side of libctu: plans, work tables, launches, graphs.
//
// Implements the C ABI declared in include/ctu.h.  A plan belongs to one
// device and owns the uploaded box / register / reflux tables and the tile
// tables of every kernel (sized at creation for every launch shape); its
// device workspace (V^n, the corner-coupling increments, V^{n+1/2}, the
// per-cell rate accumulator, predictor fluxes, shock flags) is one block,
// allocated at creation or supplied by the caller.  ctu_step enqueues the
// launch chain described in ctu_kernels.hpp on the caller's stream; nothing
// in it allocates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ctu.h"
#include "ctu_dispatch.hpp"
#include "ctu_hier.hpp"

using namespace ctu;

namespace {

thread_local std::string g_err;

ctu_status fail(ctu_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(CTU_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T> ctu_status upload(const std::vector<T> &h, T **d)
{
    *d = nullptr;
    if (h.empty()) return CTU_OK;
    if (hipMalloc((void **)d, h.size() * sizeof(T)) != hipSuccess) return fail(CTU_ERR_NOMEM, "hipMalloc of a table failed");
    HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return CTU_OK;
}

// copy a host table into a device buffer of `cap` entries reserved earlier
template <typename T> ctu_status upload_into(const std::vector<T> &h, T *d, size_t cap)
{
    if (h.size() > cap) return fail(CTU_ERR_ARG, "table larger than its reserved capacity");
    if (h.empty()) return CTU_OK;
    HIP_TRY(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return CTU_OK;
}

struct TileSet {
    std::vector<KTile> h;
    KTile *d = nullptr;
    size_t cap = 0;  // device entries reserved (shape tables: enough for every shape)
    int n() const { return (int)h.size(); }
};

// makes a plan's device current for the duration of a call and restores the
// caller's device afterwards
struct DevGuard {
    int old = -1;
    hipError_t err = hipSuccess;
    explicit DevGuard(int dev)
    {
        int cur = -1;
        err = hipGetDevice(&cur);
        if (err == hipSuccess && cur != dev) {
            err = hipSetDevice(dev);
            if (err == hipSuccess) old = cur;
        }
    }
    ~DevGuard()
    {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

// call f(std::integral_constant<int, PHYS>) for a plan's physics module
template <typename F> hipError_t with_phys(int phys, F &&f)
{
    if (phys == PHYS_MHD) return f(std::integral_constant<int, PHYS_MHD>{});
    if (phys == PHYS_RMHD) return f(std::integral_constant<int, PHYS_RMHD>{});
    return f(std::integral_constant<int, PHYS_RMHD_TM>{});
}

}  // namespace

struct ctu_plan {
    int dev = 0;  // HIP device of the tables, the workspace and every launch
    ctu_opts opts;
    KOpts ko;
    Combo combo;
    int nghost = 0;
    int esize = 8;
    std::vector<KBox> hboxes;
    KBox *dboxes = nullptr;
    std::vector<KReg> hregs;
    KReg *dregs = nullptr;
    bool has_regs = false;    // register faces were given (reg is then required)
    std::vector<int> hrface;  // per box and direction: n[d] + 2 range starts into hregs
    int *drface = nullptr;
    int64_t state_elems = 0;
    int64_t ws_cells = 0;  // sum of ghosted cells
    TileSet t_cells, t_tc, t_sweep[3], t_cfl;
    TileSet t_mt[3];  // MT corner coupling: 4 x 64 face tiles per direction
    TileSet t_pf, t_pd;  // parabolic fluxes: k_pflux / k_pdiv tiles (in-plane tiles by marching chunks)
    // workspace fields: V^n, the transverse increments T_d, V^{n+1/2}, rate
    void *wsV = nullptr, *wsT[3] = { nullptr, nullptr, nullptr };
    void *wsVh = nullptr, *wsLam = nullptr;
    void *wsPF = nullptr;  // parabolic face slots (NPF per face, dim faces per cell)
    void *wsF[3] = { nullptr, nullptr, nullptr };  // MT corner coupling: predictor fluxes per direction
    unsigned char *wsFlag = nullptr;  // App. B zone flags (one byte per cell) or null
    int64_t ws_bytes = 0;      // bytes of the workspace block the option set needs
    void *ws_block = nullptr;  // library-allocated workspace block (null: caller-owned or not yet set)
    bool has_ws = false;       // a workspace is in place
    // cells entering the cooling time-step estimate (caller-owned) or null
    const unsigned char *leaf = nullptr;
    // reflux
    KRefl *drefl = nullptr;
    int *dcell_start = nullptr;
    int nrefl_cells = 0;
    // launch shape of the t^n and sweep tables (see ctu_shape)
    ctu_shape shape{ CTU_TC_AUTO, 0, 0, 1, 0 };
    std::string tune_key;  // autotune cache key of the option set and box extents
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t tune_ev[2] = { nullptr, nullptr };  // autotuner timing events
    // per-stage event timing
    bool timing = false;
    int tsteps = 0;
    std::vector<hipEvent_t> tev;  // [step][stage][2]
    std::vector<char> tused;      // [step][stage]
};

static constexpr int kMaxTimedSteps = 256;

namespace {

void free_plan(ctu_plan *p)
{
    if (!p) return;
    DevGuard g(p->dev);
    for (hipEvent_t e : p->tev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->tune_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    void *ptrs[] = { p->dboxes, p->dregs, p->drface, p->t_cells.d, p->t_tc.d, p->t_sweep[0].d, p->t_sweep[1].d,
                     p->t_sweep[2].d, p->t_cfl.d, p->ws_block, p->drefl, p->dcell_start, p->t_mt[0].d, p->t_mt[1].d,
                     p->t_mt[2].d, p->t_pf.d, p->t_pd.d };
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

// pencils per block along x: the P that keeps P*(n+2) closest to a multiple
// of the block size (fewest idle lanes in the last round)
int pencils_per_block(int L, int npos)
{
    int best = 1;
    double best_eff = 0.0;
    for (int P = 1; P <= 64; P++) {
        if (P > npos && P > 1) break;
        long long items = (long long)P * L;
        long long rounds = (items + NT - 1) / NT;
        double eff = (double)items / (double)(rounds * NT);
        if (eff > best_eff + 1e-9 || (eff > best_eff - 1e-9 && P * L <= 16 * NT)) {
            if (eff >= best_eff - 1e-9) {
                best_eff = std::max(best_eff, eff);
                best = P;
            }
        }
    }
    return best;
}

// Launch order that gives each XCD a contiguous run of the tile list.  The
// dispatcher sends block b to XCD b % 8, and each XCD has its own L2: with
// the list in place order, tiles that share halo cache lines (neighbours in
// x and y) would run on different XCDs and fetch those lines once per XCD.
// Block b takes tile start[b % 8] + b / 8, where XCD x owns the run of
// n / 8 tiles (one more for the first n % 8 XCDs) from start[x].
constexpr int kXcds = 8;

void xcd_order(std::vector<KTile> &h)
{
    const size_t n = h.size(), q = n / kXcds, rem = n % kXcds;
    if (n < 2 * kXcds) return;
    std::vector<KTile> out(n);
    for (size_t b = 0; b < n; b++) {
        const size_t x = b % kXcds, r = b / kXcds;
        out[b] = h[x * q + std::min(x, rem) + r];
    }
    h.swap(out);
}

void add_linear_tiles(TileSet &ts, int box, long long count)
{
    for (long long s = 0; s < count; s += NT) ts.h.push_back(KTile{ box, (int)s, 0, 0 });
}

// Flat t^n layout (3D only): rows of at most MAXW1 positions.  AUTO picks it
// for a box when it needs fewer blocks per plane than the 32 x 8 tiles.
bool flat_allowed(const ctu_plan *p, const KBox &bx)
{
    return p->opts.dim == 3 && bx.n[0] + 3 <= TTile<3>::MAXW1;
}

// 3D rectangle layout: the region's W positions per row split into
// 32-wide rectangles, and a last part of at most SWMAX positions into strips
// of SH rows (a 33rd rectangle column would hold 2 of 32 active columns)
int rect_full_width(int W)
{
    const int r = W % TTile<3>::TX;
    return (r > 0 && r <= TTile<3>::SWMAX) ? W - r : W;
}

long long rect_tiles_per_plane(const KBox &bx)
{
    const int W = bx.n[0] + 2, H = bx.n[1] + 2, F = rect_full_width(W);
    long long t = (long long)((F + TTile<3>::TX - 1) / TTile<3>::TX) * ((H + TTile<3>::TY - 1) / TTile<3>::TY);
    if (F < W) t += (H + TTile<3>::SH - 1) / TTile<3>::SH;
    return t;
}

bool use_flat(const ctu_plan *p, const KBox &bx)
{
    if (!flat_allowed(p, bx) || p->shape.tc_layout == CTU_TC_TILES) return false;
    if (p->shape.tc_layout == CTU_TC_FLAT) return true;
    const long long W = bx.n[0] + 2, H = bx.n[1] + 2;
    const long long flat = ((W + 1) * (H + 1) + NT - 1) / NT;
    return flat < rect_tiles_per_plane(bx);
}

int tc_chunk(const ctu_plan *p) { return p->shape.tc_chunk > 0 ? p->shape.tc_chunk : TTile<3>::LM; }

// Entries of the shape-dependent tables for the largest shape: one-plane
// t^n chunks in the layout with more blocks per plane, one pencil per x-sweep
// block, eight y / z segments.
void shape_capacity(const ctu_plan *p, size_t cap[4])
{
    const int dim = p->opts.dim;
    for (int q = 0; q < 4; q++) cap[q] = 0;
    for (const KBox &bx : p->hboxes) {
        const long long em = bx.n[dim - 1] + 2;
        long long per = (dim == 3) ? rect_tiles_per_plane(bx) : (bx.n[0] + 2 + TTile<2>::TX - 1) / TTile<2>::TX;
        if (flat_allowed(p, bx)) per = std::max(per, ((long long)(bx.n[0] + 3) * (bx.n[1] + 3) + NT - 1) / NT);
        cap[0] += (size_t)(em * per);
        for (int D = 0; D < dim; D++) {
            int T0 = (D == 0) ? 1 : 0, T1 = (D == 2) ? 1 : 2;
            long long npos = (long long)bx.n[T0] * ((T1 < dim) ? bx.n[T1] : 1);
            cap[1 + D] += (size_t)(D == 0 ? npos : ((npos + 63) / 64) * 8);
        }
    }
}

// the tables that depend on the launch shape: t^n tiles and sweep columns,
// rebuilt on the host and copied into the buffers reserved at creation
ctu_status build_shape_tables(ctu_plan *p)
{
    const int dim = p->opts.dim;
    p->t_tc.h.clear();
    for (int D = 0; D < 3; D++) p->t_sweep[D].h.clear();
    const int LM = tc_chunk(p);
    for (int b = 0; b < (int)p->hboxes.size(); b++) {
        const KBox &bx = p->hboxes[b];
        // t^n marching kernel: in-plane tiles of the region [g-1, g+n]
        const int em = bx.n[dim - 1] + 2;
        if (use_flat(p, bx)) {
            const int npos = (bx.n[0] + 3) * (bx.n[1] + 3);
            for (int m0 = 0; m0 < em; m0 += LM)
                for (int p0 = 0; p0 < npos; p0 += NT) p->t_tc.h.push_back(KTile{ b, p0, -1, m0 });
        } else {
            const int TX = (dim == 3) ? TTile<3>::TX : TTile<2>::TX;
            const int TY = (dim == 3) ? TTile<3>::TY : TTile<2>::TY;
            const int ex = bx.n[0] + 2, ey = (dim == 3) ? bx.n[1] + 2 : 1;
            const int fx = (dim == 3) ? rect_full_width(ex) : ex;
            for (int m0 = 0; m0 < em; m0 += LM) {
                for (int y0 = 0; y0 < ey; y0 += TY)
                    for (int x0 = 0; x0 < fx; x0 += TX) p->t_tc.h.push_back(KTile{ b, x0, y0, m0 });
                if (fx < ex)
                    for (int y0 = 0; y0 < ey; y0 += TTile<3>::SH) p->t_tc.h.push_back(KTile{ b, fx, -2 - y0, m0 });
            }
        }
        for (int D = 0; D < dim; D++) {
            int T0 = (D == 0) ? 1 : 0, T1 = (D == 2) ? 1 : 2;
            int npos = bx.n[T0] * ((T1 < dim) ? bx.n[T1] : 1);
            if (D == 0) {
                int P = p->shape.x_pencils > 0 ? std::min(p->shape.x_pencils, npos)
                                               : pencils_per_block(bx.n[0] + 2, npos);
                for (int s = 0; s < npos; s += P) p->t_sweep[0].h.push_back(KTile{ b, s, P, 0 });
            } else {
                // rows [r0, r1) of the line of Lc items per tile: more, shorter
                // blocks, so that the last blocks of the launch keep more
                // waves per SIMD (each later segment re-runs two rows)
                const int Lc = bx.n[D] + 2;
                const int S = std::max(1, std::min(std::max(p->shape.yz_segments, 1), Lc / 2));
                const int L = (Lc + S - 1) / S;
                for (int s = 0; s < npos; s += 64)
                    for (int r0 = 0; r0 < Lc; r0 += L) p->t_sweep[D].h.push_back(KTile{ b, s, r0, std::min(Lc, r0 + L) });
            }
        }
    }
    if (p->shape.xcd_order) {
        xcd_order(p->t_tc.h);
        for (int D = 0; D < dim; D++) xcd_order(p->t_sweep[D].h);
    }
    ctu_status st;
    TileSet *all[] = { &p->t_tc, &p->t_sweep[0], &p->t_sweep[1], &p->t_sweep[2] };
    // a previous step may still read the tables being replaced
    HIP_TRY(hipDeviceSynchronize());
    for (TileSet *ts : all)
        if ((st = upload_into(ts->h, ts->d, ts->cap)) != CTU_OK) return st;
    return CTU_OK;
}

// reserve the shape tables' device buffers for every shape (creation only)
ctu_status reserve_shape_tables(ctu_plan *p)
{
    size_t cap[4];
    shape_capacity(p, cap);
    TileSet *all[] = { &p->t_tc, &p->t_sweep[0], &p->t_sweep[1], &p->t_sweep[2] };
    for (int q = 0; q < 4; q++) {
        all[q]->cap = cap[q];
        if (cap[q] == 0) continue;
        if (hipMalloc((void **)&all[q]->d, cap[q] * sizeof(KTile)) != hipSuccess)
            return fail(CTU_ERR_NOMEM, "hipMalloc of a tile table failed");
    }
    return CTU_OK;
}

// MT face tiles of direction D (see k_mtflux): D = 0: 63 x-faces from a
// (lanes from a-1) by 4 rows of y from b at z = c; D = 1, 2: 64 x-positions
// from a by 4 D-faces from b, the third axis at c.  Faces g..g+n along D,
// transverse positions g-1..g+n.
void add_mt_tiles(TileSet &ts, int b, const KBox &bx, int D, int dim)
{
    const int lo[3] = { bx.g[0] - 1, bx.g[1] - 1, dim == 3 ? bx.g[2] - 1 : 0 };
    const int hi[3] = { bx.g[0] + bx.n[0], bx.g[1] + bx.n[1], dim == 3 ? bx.g[2] + bx.n[2] : 0 };
    if (D == 0) {
        for (int z = lo[2]; z <= hi[2]; z++)
            for (int y = lo[1]; y <= hi[1]; y += 4)
                for (int x = bx.g[0]; x <= hi[0]; x += 63) ts.h.push_back({ b, x, y, z });
    } else {
        const int T = (D == 1) ? 2 : 1;
        for (int t = lo[T]; t <= hi[T]; t++)
            for (int f = bx.g[D]; f <= hi[D]; f += 4)
                for (int x = lo[0]; x <= hi[0]; x += 64) ts.h.push_back({ b, x, f, t });
    }
}

// Parabolic flux tiles: TX x TY in-plane cells by LM planes.  k_pflux: the
// n + 1 face cells g .. g+n per axis, tiles side by side; k_pdiv: the n + 2
// region cells g-1 .. g+n, tiles overlapping by one column (and row).
void add_pf_tiles(TileSet &ts, int b, const KBox &bx, int dim, bool div)
{
    const int TX = (dim == 3) ? PTile<3>::TX : PTile<2>::TX, TY = (dim == 3) ? PTile<3>::TY : PTile<2>::TY;
    const int LM = div ? ((dim == 3) ? PTile<3>::LM_DIV : PTile<2>::LM_DIV)
                       : ((dim == 3) ? PTile<3>::LM_FLUX : PTile<2>::LM_FLUX);
    const int k = div ? 2 : 1, sx = div ? TX - 1 : TX, sy = (div && dim == 3) ? TY - 1 : TY;
    const int ex = bx.n[0] + k, ey = (dim == 3) ? bx.n[1] + k : 1, em = bx.n[dim - 1] + k;
    for (int m0 = 0; m0 < em; m0 += LM)
        for (int y0 = 0; y0 < ey; y0 += sy)
            for (int x0 = 0; x0 < ex; x0 += sx) ts.h.push_back({ b, x0, y0, m0 });
}

ctu_status build_tables(ctu_plan *p)
{
    const int dim = p->opts.dim;
    const bool mt = p->opts.corner == CTU_CORNER_MT;
    for (int b = 0; b < (int)p->hboxes.size(); b++) {
        const KBox &bx = p->hboxes[b];
        add_linear_tiles(p->t_cells, b, bx.cells);
        add_linear_tiles(p->t_cfl, b, (long long)bx.n[0] * bx.n[1] * bx.n[2]);
        if (mt)
            for (int D = 0; D < dim; D++) add_mt_tiles(p->t_mt[D], b, bx, D, dim);
        if (p->opts.parabolic_mask) {
            add_pf_tiles(p->t_pf, b, bx, dim, false);
            add_pf_tiles(p->t_pd, b, bx, dim, true);
        }
    }
    xcd_order(p->t_pf.h);
    xcd_order(p->t_pd.h);
    ctu_status st;
    TileSet *all[] = { &p->t_cells, &p->t_cfl, &p->t_mt[0], &p->t_mt[1], &p->t_mt[2], &p->t_pf, &p->t_pd };
    for (TileSet *ts : all)
        if (!ts->h.empty() && (st = upload(ts->h, &ts->d)) != CTU_OK) return st;
    if ((st = reserve_shape_tables(p)) != CTU_OK) return st;
    return build_shape_tables(p);
}

// Workspace fields of the option set, in block order, each starting on a
// 256-byte boundary: V^n (9 per cell), T_d per direction, with parabolic
// terms V^{n+1/2}, the per-cell rate and the face slots (NPF per face, one
// face per direction and cell), with the MT coupling the predictor fluxes
// per direction, with the App. B hybrid one flag byte per cell.
// With base == null only the size is computed.
int64_t carve_ws(ctu_plan *p, char *base)
{
    const int64_t f9 = (int64_t)NV * p->ws_cells * p->esize;
    int64_t off = 0;
    auto take = [&](void **ptr, int64_t bytes) {
        if (base) *ptr = base + off;
        off += (bytes + 255) / 256 * 256;
    };
    void *dummy = nullptr;
    take(base ? &p->wsV : &dummy, f9);
    for (int d = 0; d < p->opts.dim; d++) take(base ? &p->wsT[d] : &dummy, f9);
    if (p->opts.parabolic_mask) {
        take(base ? &p->wsVh : &dummy, f9);
        take(base ? &p->wsLam : &dummy, p->ws_cells * p->esize);
        take(base ? &p->wsPF : &dummy, (int64_t)NPF * p->opts.dim * p->ws_cells * p->esize);
    }
    if (p->opts.corner == CTU_CORNER_MT)
        for (int d = 0; d < p->opts.dim; d++) take(base ? &p->wsF[d] : &dummy, f9);
    if (p->combo.shk) take(base ? (void **)&p->wsFlag : &dummy, p->ws_cells);
    return off;
}

// drop a captured graph (it refers to the old tables or workspace)
ctu_status drop_graph(ctu_plan *p)
{
    if (p->gexec) {
        HIP_TRY(hipGraphExecDestroy(p->gexec));
        p->gexec = nullptr;
    }
    if (p->graph) {
        HIP_TRY(hipGraphDestroy(p->graph));
        p->graph = nullptr;
    }
    return CTU_OK;
}

// event pair of (current step, stage) or null when timing is off / full
hipEvent_t *timer(ctu_plan *p, int stage)
{
    if (!p->timing || p->tsteps >= kMaxTimedSteps) return nullptr;
    size_t idx = (size_t)p->tsteps * CTU_NSTAGE + stage;
    p->tused[idx] = 1;
    return &p->tev[2 * idx];
}

struct StageTimer {
    hipEvent_t *ev;
    hipStream_t s;
    StageTimer(ctu_plan *p, int stage, hipStream_t st) : ev(timer(p, stage)), s(st)
    {
        if (ev) (void)hipEventRecord(ev[0], s);
    }
    ~StageTimer()
    {
        if (ev) (void)hipEventRecord(ev[1], s);
    }
};

// the parabolic fluxes over the plan's boxes: div = 1, k_pdiv on V^n (the
// Pi^n divergence per cell of the t^n region); div = 0, k_pflux on
// V^{n+1/2} (the sweeps' face slots).  Both write the wsPF field.
template <typename R> hipError_t launch_pflux(ctu_plan *p, const R *V, int div, hipStream_t s)
{
    PArgs<R> pa;
    const TileSet &ts = div ? p->t_pd : p->t_pf;
    pa.boxes = p->dboxes;
    pa.tiles = ts.d;
    pa.V = V;
    pa.PF = (R *)p->wsPF;
    pa.o = p->ko;
    if constexpr (sizeof(R) == 4) return launch_pflux_f32(p->opts.dim, div, (int)ts.n(), pa, s);
    else return launch_pflux_f64(p->opts.dim, div, (int)ts.n(), pa, s);
}

template <typename R>
ctu_status enqueue_step(ctu_plan *p, const void *U_in, void *U_out, const double *params, const void *L0, double *reg,
                        double *rate, double *dpp, int32_t *fails, hipStream_t s)
{
    const int dim = p->opts.dim;
    const bool par = p->opts.parabolic_mask != 0;
    hipLaunchKernelGGL(k_reset<0>, dim3(1), dim3(64), 0, s, rate, dpp, (int *)fails);
    HIP_TRY(hipGetLastError());
    const R gam = (R)p->opts.gamma;
    {
        StageTimer tm(p, 0, s);
        HIP_TRY(with_phys(p->combo.phys, [&](auto P) {
            hipLaunchKernelGGL((k_cons2prim<decltype(P)::value, R>), dim3(p->t_cells.n()), dim3(NT), 0, s,
                               p->dboxes, p->t_cells.d, (const R *)U_in, (R *)p->wsV, (int *)fails, gam, 1);
            return hipGetLastError();
        }));
        if (p->wsFlag) {
            HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL((k_shock_hll<R>), dim3(p->t_cells.n()), dim3(NT), 0, s, p->dboxes, p->t_cells.d,
                               (const R *)p->wsV, p->wsFlag, p->opts.shock_eps, dim);
            HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(k_shock_mm<0>, dim3(p->t_cells.n()), dim3(NT), 0, s, p->dboxes, p->t_cells.d, p->wsFlag,
                               p->ko.shock_r, dim);
        }
    }
    HIP_TRY(hipGetLastError());
    if (p->opts.corner == CTU_CORNER_MT) {
        StageTimer tm(p, 1, s);
        MtArgs<R> ma;
        ma.boxes = p->dboxes;
        ma.tiles = p->t_cells.d;
        ma.U = (const R *)U_in;
        ma.V = (const R *)p->wsV;
        for (int d = 0; d < 3; d++) {
            ma.F[d] = (R *)p->wsF[d];
            ma.T[d] = (R *)p->wsT[d];
        }
        ma.params = params;
        ma.o = p->ko;
        for (int D = 0; D < dim; D++) {
            hipError_t e;
            ma.tiles = p->t_mt[D].d;
            if constexpr (sizeof(R) == 4)
                e = launch_mtflux_f32(D, p->combo, p->t_mt[D].n(), ma, s);
            else
                e = launch_mtflux_f64(D, p->combo, p->t_mt[D].n(), ma, s);
            if (e != hipSuccess) return fail(CTU_ERR_HIP, std::string("MT flux launch: ") + hipGetErrorString(e));
        }
        ma.tiles = p->t_cells.d;
        if (dim == 3) hipLaunchKernelGGL((k_mtT<3, R>), dim3(p->t_cells.n()), dim3(NT), 0, s, ma);
        else hipLaunchKernelGGL((k_mtT<2, R>), dim3(p->t_cells.n()), dim3(NT), 0, s, ma);
        HIP_TRY(hipGetLastError());
    } else {
        if (par) {
            StageTimer tm(p, 2, s);
            HIP_TRY(launch_pflux(p, (const R *)p->wsV, 1, s));
        }
        StageTimer tm(p, 1, s);
        TArgs<R> ta;
        ta.boxes = p->dboxes;
        ta.tiles = p->t_tc.d;
        ta.U = (const R *)U_in;
        ta.V = (const R *)p->wsV;
        for (int d = 0; d < 3; d++) ta.T[d] = (R *)p->wsT[d];
        ta.Vh = (R *)p->wsVh;
        ta.PF = (const R *)p->wsPF;
        ta.flag = p->wsFlag;
        ta.params = params;
        ta.o = p->ko;
        ta.lm = tc_chunk(p);
        hipError_t e;
        if constexpr (sizeof(R) == 4)
            e = launch_tcouple_f32(dim, par ? 1 : 0, p->combo, p->t_tc.n(), ta, s);
        else
            e = launch_tcouple_f64(dim, par ? 1 : 0, p->combo, p->t_tc.n(), ta, s);
        if (e != hipSuccess) return fail(CTU_ERR_HIP, std::string("t^n kernel launch: ") + hipGetErrorString(e));
    }
    if (par) {
        StageTimer tm(p, 3, s);
        HIP_TRY(launch_pflux(p, (const R *)p->wsVh, 0, s));
    }
    SweepArgs<R> a;
    a.boxes = p->dboxes;
    a.regs = p->dregs;
    a.rface = p->drface;
    a.U = (const R *)U_in;
    a.Uout = (R *)U_out;
    a.V = (const R *)p->wsV;
    for (int d = 0; d < 3; d++) a.T[d] = (const R *)p->wsT[d];
    a.Vh = (const R *)p->wsVh;
    a.PF = (const R *)p->wsPF;
    a.lam = (R *)p->wsLam;
    a.L0 = (const R *)L0;
    a.leaf = p->leaf;
    a.flag = p->wsFlag;
    a.reg = p->hregs.empty() ? nullptr : reg;  // no entry lies on a box face: nothing to write
    a.params = params;
    a.rate = rate;
    a.dpp = dpp;
    a.fails = (int *)fails;
    a.o = p->ko;
    for (int D = 0; D < dim; D++) {
        a.tiles = p->t_sweep[D].d;
        a.first = (D == 0);
        a.last = (D == dim - 1);
        hipError_t e;
        {
            StageTimer tm(p, 5 + D, s);
            e = launch_sweep<R>(D, p->combo, p->t_sweep[D].n(), a, s);
        }
        if (e != hipSuccess) return fail(CTU_ERR_HIP, std::string("sweep launch: ") + hipGetErrorString(e));
    }
    if (p->timing && p->tsteps < kMaxTimedSteps) p->tsteps++;
    return CTU_OK;
}

// Autotune cache: the best shape found per option set and box extents,
// for the life of the process; ctu_plan_create applies a cached shape.
std::mutex g_tune_mu;
std::map<std::string, ctu_shape> g_tune_cache;

std::string tune_key(const ctu_plan *p)
{
    const ctu_opts &o = p->opts;
    std::vector<std::array<int, 3>> ext;
    for (const KBox &b : p->hboxes) ext.push_back({ b.n[0], b.n[1], b.n[2] });
    std::sort(ext.begin(), ext.end());
    unsigned long long h = 1469598103934665603ULL;  // FNV-1a over the sorted extents
    for (auto &e : ext)
        for (int v : e) {
            h ^= (unsigned)v;
            h *= 1099511628211ULL;
        }
    char buf[256];
    std::snprintf(buf, sizeof buf, "p%d d%d ph%d r%d pr%d rs%d w%d g%d pb%u c%d s%d h%u ng%d nb%zu k%d x%016llx",
                  p->esize, o.dim, o.physics, o.recon, o.predictor, o.riemann, o.wref, o.glm, o.parabolic_mask,
                  o.cooling, o.shock_eps > 0.0 ? 1 : 0, o.hyperbolic_off, p->nghost, p->hboxes.size(), o.corner, h);
    return buf;
}

ctu_status check_shape(const ctu_shape *sh)
{
    if (!sh) return fail(CTU_ERR_ARG, "null shape");
    if (sh->tc_layout < CTU_TC_AUTO || sh->tc_layout > CTU_TC_FLAT) return fail(CTU_ERR_ARG, "bad tc_layout");
    if (sh->tc_chunk < 0 || sh->tc_chunk > 4096) return fail(CTU_ERR_ARG, "tc_chunk must be 0 (default) or 1..4096");
    if (sh->x_pencils < 0 || sh->x_pencils > 64) return fail(CTU_ERR_ARG, "x_pencils must be 0 (auto) or 1..64");
    if (sh->xcd_order != 0 && sh->xcd_order != 1) return fail(CTU_ERR_ARG, "xcd_order must be 0 or 1");
    if (sh->yz_segments < 0 || sh->yz_segments > 8) return fail(CTU_ERR_ARG, "yz_segments must be 0 (one) or 1..8");
    return CTU_OK;
}

// rebuild the shape's tables; a captured graph refers to the old ones
ctu_status apply_shape(ctu_plan *p, const ctu_shape &sh)
{
    ctu_status st = drop_graph(p);
    if (st != CTU_OK) return st;
    p->shape = sh;
    return build_shape_tables(p);
}

ctu_status check_step_args(ctu_plan *p, const void *U_in, void *U_out, const double *params, const void *L0,
                           double *reg, double *rate, bool need_ws = true)
{
    if (!p) return fail(CTU_ERR_ARG, "null plan");
    if (need_ws && !p->has_ws) return fail(CTU_ERR_ARG, "the plan has no workspace: call ctu_plan_set_workspace first");
    if (!U_in || !U_out || !params || !rate) return fail(CTU_ERR_ARG, "U_in, U_out, params and rate are required");
    if (U_in == U_out) return fail(CTU_ERR_ARG, "U_out must not alias U_in");
    if (p->opts.cooling && !L0) return fail(CTU_ERR_ARG, "cooling needs cool_L0");
    if (p->has_regs && !reg) return fail(CTU_ERR_ARG, "the plan has register faces: reg is required");
    return CTU_OK;
}

}  // namespace

extern "C" {

const char *ctu_last_error(void) { return g_err.c_str(); }

static ctu_status set_reflux_table(ctu_plan *plan, const ctu_refluxface *faces, int32_t nfaces);

static ctu_status create_plan(int32_t dev, uint32_t flags, const ctu_opts *opts, const ctu_box *boxes, int32_t nbox,
                              int32_t nghost, const ctu_regface *regfaces, int32_t nreg, const ctu_refluxface *reflux,
                              int32_t nreflux, ctu_plan **plan_out)
{
    if (!plan_out) return fail(CTU_ERR_ARG, "plan_out is null");
    *plan_out = nullptr;
    if (!opts || !boxes || nbox <= 0) return fail(CTU_ERR_ARG, "options and at least one box are required");
    if (flags & ~(uint32_t)(CTU_PLAN_CALLER_WORKSPACE | CTU_PLAN_LEVEL_DT)) return fail(CTU_ERR_ARG, "unknown plan flags");
    if (nreflux < 0 || (nreflux > 0 && !reflux)) return fail(CTU_ERR_ARG, "bad reflux table");
    const ctu_opts &o = *opts;
    if (o.dim != 2 && o.dim != 3) return fail(CTU_ERR_ARG, "dim must be 2 or 3");
    if (o.physics != CTU_MHD && o.physics != CTU_RMHD) return fail(CTU_ERR_ARG, "bad physics");
    if (o.precision != CTU_FP64 && o.precision != CTU_FP32) return fail(CTU_ERR_ARG, "bad precision");
    if (o.recon < CTU_LIN_MC || o.recon > CTU_WENO3) return fail(CTU_ERR_ARG, "bad recon");
    if (o.predictor != CTU_PRED_CHAR && o.predictor != CTU_PRED_MUSCL_HANCOCK) return fail(CTU_ERR_ARG, "bad predictor");
    if (o.wref < CTU_WREF_FACE || o.wref > CTU_WREF_CW84) return fail(CTU_ERR_ARG, "bad wref");
    if (o.riemann != CTU_HLLD && o.riemann != CTU_HLL && o.riemann != CTU_RUSANOV && o.riemann != CTU_HLLC &&
        o.riemann != CTU_ROE)
        return fail(CTU_ERR_ARG, "bad riemann");
    if (o.eos != CTU_EOS_IDEAL && o.eos != CTU_EOS_TM) return fail(CTU_ERR_ARG, "bad eos");
    if (o.exact_speeds != 0 && o.exact_speeds != 1) return fail(CTU_ERR_ARG, "exact_speeds must be 0 or 1");
    if (o.corner != CTU_CORNER_TN && o.corner != CTU_CORNER_MT) return fail(CTU_ERR_ARG, "bad corner");
    if (o.corner == CTU_CORNER_MT && (o.parabolic_mask || o.hyperbolic_off || o.shock_eps > 0.0))
        return fail(CTU_ERR_UNSUPPORTED, "the MT corner coupling needs hyperbolic fluxes without parabolic terms "
                                         "or shock flags");
    if (o.eos == CTU_EOS_TM && o.physics != CTU_RMHD)
        return fail(CTU_ERR_UNSUPPORTED, "the Taub-Matthews EOS belongs to the RMHD module");
    if (!(o.gamma > 1.0)) return fail(CTU_ERR_ARG, "gamma must exceed 1");
    for (int d = 0; d < o.dim; d++)
        if (!(o.dx[d] > 0.0)) return fail(CTU_ERR_ARG, "dx must be positive");
    if (o.parabolic_mask & ~7u) return fail(CTU_ERR_ARG, "unknown parabolic bits");
    if (!(o.shock_eps >= 0.0)) return fail(CTU_ERR_ARG, "shock_eps must be >= 0");
    Combo c;
    c.phys = (o.physics == CTU_RMHD && o.eos == CTU_EOS_TM) ? PHYS_RMHD_TM : o.physics;
    c.pred = o.predictor;
    c.rk = (o.recon == CTU_PPM) ? RK_PPM : (o.recon == CTU_WENO3 ? RK_WENO : RK_LIN);
    c.rs = o.riemann;
    c.shk = o.shock_eps > 0.0 ? 1 : 0;
    const bool fixed = o.wref == CTU_WREF_FACE && o.glm && !o.hyperbolic_off && !c.shk;
    c.fast = (fixed && !o.parabolic_mask && !o.cooling) ? 1 : 0;
    c.par = (fixed && (o.parabolic_mask || o.cooling)) ? 1 : 0;
    if ((o.riemann == CTU_RUSANOV || o.riemann == CTU_HLLC || o.riemann == CTU_ROE) && c.shk)
        return fail(CTU_ERR_UNSUPPORTED, "the shock-adaptive hybrid (HLL on flagged faces) needs HLLD or HLL");
    if (o.physics == CTU_RMHD && o.riemann == CTU_ROE)
        return fail(CTU_ERR_UNSUPPORTED, "the Roe solver belongs to the MHD module");
    if (!combo_supported(c))
        return fail(CTU_ERR_UNSUPPORTED, "unsupported combination (characteristic tracing is MHD only; "
                                         "MUSCL-Hancock needs a linear reconstruction)");
    if (o.physics == CTU_RMHD && (o.parabolic_mask || o.cooling))
        return fail(CTU_ERR_UNSUPPORTED, "parabolic terms and cooling are MHD only");
    int need = (o.recon == CTU_PPM ? 3 : 2) + (o.parabolic_mask ? 1 : 0);
    if (o.corner == CTU_CORNER_MT && need < 3) need = 3;
    if (nghost < 3 || nghost < need) return fail(CTU_ERR_ARG, "nghost too small for the stencil");
    if (nreg > 0 && !regfaces) return fail(CTU_ERR_ARG, "regfaces is null");

    // the option checks above run on the host; the device is needed from here
    {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
        if (dev < 0 || dev >= ndev) return fail(CTU_ERR_ARG, "hip_device out of range (no such HIP device)");
    }
    DevGuard guard(dev);
    HIP_TRY(guard.err);
    ctu_plan *p = new ctu_plan();
    p->dev = dev;
    p->opts = o;
    p->combo = c;
    p->nghost = nghost;
    p->esize = (o.precision == CTU_FP32) ? 4 : 8;
    KOpts &k = p->ko;
    k.dim = o.dim;
    k.limiter = (o.recon <= CTU_LIN_VANALBADA) ? o.recon : LIM_MC;
    k.wref = o.wref;
    k.glm = o.glm ? 1 : 0;
    k.parab = (int)o.parabolic_mask;
    k.cooling = o.cooling ? 1 : 0;
    k.hyp_off = o.hyperbolic_off ? 1 : 0;
    k.shock_r = (o.recon == CTU_PPM) ? 2 : 1;
    k.xspeeds = (o.physics == CTU_RMHD && o.exact_speeds) ? 1 : 0;
    k.pad = 0;
    k.shock_eps = o.shock_eps;
    k.gamma = o.gamma;
    k.glm_alpha = o.glm_alpha;
    k.nu = o.nu;
    k.eta = o.eta;
    k.kpar = o.kappa_par;
    k.kperp = o.kappa_perp;
    k.phi = o.tc_phi;
    k.cool_beta = o.cool_beta;
    k.T_floor = o.T_floor;

    // boxes: validate, workspace offsets
    int64_t woff = 0;
    std::vector<std::pair<int64_t, int64_t>> spans;
    for (int b = 0; b < nbox; b++) {
        const ctu_box &B = boxes[b];
        KBox kb;
        std::memset(&kb, 0, sizeof(kb));
        for (int d = 0; d < 3; d++) {
            bool act = d < o.dim;
            kb.n[d] = act ? B.n[d] : 1;
            kb.g[d] = act ? nghost : 0;
            kb.N[d] = kb.n[d] + 2 * kb.g[d];
            kb.lo[d] = act ? B.lo[d] : 0;
            kb.dx[d] = act ? o.dx[d] / (double)(1LL << B.level) : 1.0;
            if (act && B.n[d] < 1) {
                free_plan(p);
                return fail(CTU_ERR_ARG, "box extents must be positive");
            }
        }
        if (o.dim == 2 && B.n[2] != 1) {
            free_plan(p);
            return fail(CTU_ERR_ARG, "2D boxes must have n[2] == 1");
        }
        if (B.level < 0 || B.level > 30 || B.offset < 0 || (B.offset % NV) != 0) {
            free_plan(p);
            return fail(CTU_ERR_ARG, "bad box level or offset (offsets are multiples of 9)");
        }
        kb.cells = (long long)kb.N[0] * kb.N[1] * kb.N[2];
        // the kernels address one box's nine planes with 32-bit byte offsets
        if (NV * kb.cells * p->esize > 0xFFFFFFFFLL) {
            free_plan(p);
            return fail(CTU_ERR_ARG,
                        "a box's nine variable planes must fit in 4 GiB of ghosted cells (split larger grids into boxes)");
        }
        kb.uoff = B.offset;
        kb.woff = woff;
        woff += NV * kb.cells;
        spans.push_back({ B.offset, B.offset + NV * kb.cells });
        p->state_elems = std::max<int64_t>(p->state_elems, B.offset + NV * kb.cells);
        p->ws_cells += kb.cells;
        kb.reg0 = kb.reg1 = 0;
        kb.rface[0] = kb.rface[1] = kb.rface[2] = 0;
        kb.lshift = (flags & CTU_PLAN_LEVEL_DT) ? B.level : 0;
        p->hboxes.push_back(kb);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t q = 1; q < spans.size(); q++)
        if (spans[q].first < spans[q - 1].second) {
            free_plan(p);
            return fail(CTU_ERR_ARG, "box blocks overlap in the state array");
        }

    // register faces grouped per box
    std::vector<std::vector<KReg>> per(nbox);
    for (int r = 0; r < nreg; r++) {
        const ctu_regface &R = regfaces[r];
        if (R.box < 0 || R.box >= nbox || R.dir < 0 || R.dir >= o.dim || R.tn[0] < 1 || R.tn[1] < 1 || R.slot < 0 ||
            (o.dim == 2 && R.tn[1] != 1)) {
            free_plan(p);
            return fail(CTU_ERR_ARG, "bad register face entry");
        }
        KReg kr;
        kr.dir = R.dir;
        kr.face = R.face;
        kr.tlo0 = R.tlo[0];
        kr.tlo1 = (o.dim == 2) ? 0 : R.tlo[1];
        kr.tn0 = R.tn[0];
        kr.tn1 = R.tn[1];
        kr.pad0 = kr.pad1 = 0;
        kr.slot = R.slot;
        per[R.box].push_back(kr);
    }
    // each box's entries sorted by (dir, face), with per-face ranges so that a
    // sweep reads only the rectangles on its own face plane; entries off the
    // box's faces lo[d] .. lo[d] + n[d] are never written and are dropped
    for (int b = 0; b < nbox; b++) {
        KBox &kb = p->hboxes[b];
        std::stable_sort(per[b].begin(), per[b].end(), [](const KReg &x, const KReg &y) {
            return x.dir != y.dir ? x.dir < y.dir : x.face < y.face;
        });
        kb.reg0 = (int)p->hregs.size();
        for (int d = 0; d < o.dim; d++) {
            kb.rface[d] = (int)p->hrface.size();
            for (int f = 0; f <= kb.n[d]; f++) {
                p->hrface.push_back((int)p->hregs.size());
                for (auto &r : per[b])
                    if (r.dir == d && r.face == kb.lo[d] + f) p->hregs.push_back(r);
            }
            p->hrface.push_back((int)p->hregs.size());
        }
        kb.reg1 = (int)p->hregs.size();
    }
    if (p->hrface.empty()) p->hrface.push_back(0);
    p->has_regs = nreg > 0;

    ctu_status st;
    if ((st = upload(p->hboxes, &p->dboxes)) != CTU_OK || (st = upload(p->hregs, &p->dregs)) != CTU_OK ||
        (st = upload(p->hrface, &p->drface)) != CTU_OK ||
        (st = build_tables(p)) != CTU_OK) {
        free_plan(p);
        return st;
    }
    p->tune_key = tune_key(p);
    {
        ctu_shape cached;
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(p->tune_key);
            if (it != g_tune_cache.end()) {
                cached = it->second;
                hit = true;
            }
        }
        if (hit && (st = apply_shape(p, cached)) != CTU_OK) {
            free_plan(p);
            return st;
        }
    }
    if (nreflux > 0 && (st = set_reflux_table(p, reflux, nreflux)) != CTU_OK) {
        free_plan(p);
        return st;
    }
    if (hipEventCreate(&p->tune_ev[0]) != hipSuccess || hipEventCreate(&p->tune_ev[1]) != hipSuccess) {
        free_plan(p);
        return fail(CTU_ERR_HIP, "hipEventCreate failed");
    }
    p->ws_bytes = carve_ws(p, nullptr);
    if (!(flags & CTU_PLAN_CALLER_WORKSPACE)) {
        if (hipMalloc(&p->ws_block, p->ws_bytes) != hipSuccess) {
            free_plan(p);
            return fail(CTU_ERR_NOMEM, "hipMalloc of the workspace failed");
        }
        carve_ws(p, (char *)p->ws_block);
        p->has_ws = true;
    }
    *plan_out = p;
    return CTU_OK;
}

ctu_status ctu_plan_create(const ctu_opts *opts, const ctu_box *boxes, int32_t nbox, int32_t nghost,
                           const ctu_regface *regfaces, int32_t nreg, ctu_plan **plan_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;  // no device: the option checks still report first
    return create_plan(dev, 0u, opts, boxes, nbox, nghost, regfaces, nreg, nullptr, 0, plan_out);
}

ctu_status ctu_plan_create_ex(int32_t hip_device, uint32_t flags, const ctu_opts *opts, const ctu_box *boxes,
                              int32_t nbox, int32_t nghost, const ctu_regface *regfaces, int32_t nreg,
                              const ctu_refluxface *reflux, int32_t nreflux, ctu_plan **plan_out)
{
    return create_plan(hip_device, flags, opts, boxes, nbox, nghost, regfaces, nreg, reflux, nreflux, plan_out);
}

ctu_status ctu_plan_set_workspace(ctu_plan *plan, void *ws_dev, int64_t bytes)
{
    if (!plan) return fail(CTU_ERR_ARG, "null plan");
    if (!ws_dev) return fail(CTU_ERR_ARG, "null workspace");
    if (plan->ws_block) return fail(CTU_ERR_ARG, "the plan owns its workspace (created without CTU_PLAN_CALLER_WORKSPACE)");
    if (bytes < plan->ws_bytes) return fail(CTU_ERR_ARG, "workspace smaller than ctu_plan_workspace_bytes");
    if (((uintptr_t)ws_dev & 255u) != 0) return fail(CTU_ERR_ARG, "workspace must be 256-byte aligned");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    ctu_status st = drop_graph(plan);
    if (st != CTU_OK) return st;
    // a previous step may still use the old workspace
    HIP_TRY(hipDeviceSynchronize());
    carve_ws(plan, (char *)ws_dev);
    plan->has_ws = true;
    return CTU_OK;
}

int32_t ctu_plan_device(const ctu_plan *plan) { return plan ? plan->dev : -1; }

void ctu_plan_destroy(ctu_plan *plan) { free_plan(plan); }

int64_t ctu_plan_state_elems(const ctu_plan *plan) { return plan ? plan->state_elems : 0; }
int64_t ctu_plan_workspace_bytes(const ctu_plan *plan) { return plan ? plan->ws_bytes : 0; }

ctu_status ctu_plan_set_shape(ctu_plan *plan, const ctu_shape *shape)
{
    if (!plan) return fail(CTU_ERR_ARG, "null plan");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    ctu_status st = check_shape(shape);
    if (st != CTU_OK) return st;
    return apply_shape(plan, *shape);
}

ctu_status ctu_plan_get_shape(const ctu_plan *plan, ctu_shape *shape_out, int32_t *flat_boxes_out)
{
    if (!plan || !shape_out) return fail(CTU_ERR_ARG, "null plan or shape");
    *shape_out = plan->shape;
    if (flat_boxes_out) {
        int nf = 0;
        for (const KBox &b : plan->hboxes) nf += use_flat(plan, b) ? 1 : 0;
        *flat_boxes_out = nf;
    }
    return CTU_OK;
}

ctu_status ctu_plan_autotune(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                             const void *cool_L0_dev, int32_t reps, void *stream, ctu_shape *best_out,
                             double *best_ms_out)
{
    if (!plan) return fail(CTU_ERR_ARG, "null plan");
    if (!U_in_dev || !U_out_dev || !params_dev) return fail(CTU_ERR_ARG, "U_in, U_out and params are required");
    if (U_in_dev == U_out_dev) return fail(CTU_ERR_ARG, "U_out must not alias U_in");
    if (plan->opts.cooling && !cool_L0_dev) return fail(CTU_ERR_ARG, "cooling needs cool_L0");
    if (reps < 1 || reps > 1000) return fail(CTU_ERR_ARG, "reps must be in 1..1000");
    if (!plan->has_ws) return fail(CTU_ERR_ARG, "the plan has no workspace: call ctu_plan_set_workspace first");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    hipStream_t s = (hipStream_t)stream;
    const bool timing = plan->timing;
    plan->timing = false;
    hipEvent_t e0 = plan->tune_ev[0], e1 = plan->tune_ev[1];
    ctu_status st = CTU_OK;
    auto run = [&](double &ms) -> ctu_status {
        ctu_status r;
        for (int k = 0; k <= reps; k++) {
            if (k == 1) HIP_TRY(hipEventRecord(e0, s));
            // no registers, rate, dpp or failure counts: only the timing matters
            r = (plan->esize == 4) ? enqueue_step<float>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, nullptr,
                                                         nullptr, nullptr, nullptr, s)
                                   : enqueue_step<double>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev,
                                                          nullptr, nullptr, nullptr, nullptr, s);
            if (r != CTU_OK) return r;
        }
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float f = 0.0f;
        HIP_TRY(hipEventElapsedTime(&f, e0, e1));
        ms = f / reps;
        return CTU_OK;
    };
    auto body = [&]() -> ctu_status {
        bool any_flat = false;
        for (const KBox &b : plan->hboxes) any_flat = any_flat || flat_allowed(plan, b);
        ctu_shape best = plan->shape;
        double best_ms = 0.0;
        ctu_status r;
        if ((r = apply_shape(plan, best)) != CTU_OK || (r = run(best_ms)) != CTU_OK) return r;
        auto consider = [&](const ctu_shape &c) -> ctu_status {
            double ms;
            ctu_status q;
            if ((q = apply_shape(plan, c)) != CTU_OK || (q = run(ms)) != CTU_OK) return q;
            // a candidate must beat the incumbent by 1 %, so that timing
            // noise does not flip between shapes of equal speed
            if (ms < 0.99 * best_ms) {
                best_ms = ms;
                best = c;
            }
            return CTU_OK;
        };
        // coordinate descent: t^n layout and chunk, x-sweep pencils, y / z
        // sweep segments, launch order
        const int layouts[] = { CTU_TC_AUTO, CTU_TC_TILES, CTU_TC_FLAT };
        const int chunks[] = { 4, 8, 16, 32 };
        for (int L : layouts) {
            if (L != CTU_TC_TILES && !any_flat) continue;
            for (int ch : chunks) {
                ctu_shape c = best;
                c.tc_layout = L;
                c.tc_chunk = ch;
                if ((r = consider(c)) != CTU_OK) return r;
            }
        }
        // the counts that measure fastest on a full line first: a later one
        // must win by the 1 % margin against them, not against a slow start
        const int pencils[] = { 16, 8, 32, 4, 0 };
        for (int P : pencils) {
            ctu_shape c = best;
            c.x_pencils = P;
            if ((r = consider(c)) != CTU_OK) return r;
        }
        const int segs[] = { 0, 2, 3, 4 };
        for (int S : segs) {
            ctu_shape c = best;
            c.yz_segments = S;
            if ((r = consider(c)) != CTU_OK) return r;
        }
        {
            ctu_shape c = best;
            c.xcd_order = 1 - c.xcd_order;
            if ((r = consider(c)) != CTU_OK) return r;
        }
        if ((r = apply_shape(plan, best)) != CTU_OK) return r;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[plan->tune_key] = best;
        }
        if (best_out) *best_out = best;
        if (best_ms_out) *best_ms_out = best_ms;
        return CTU_OK;
    };
    st = body();
    plan->timing = timing;
    return st;
}

ctu_status ctu_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
    return CTU_OK;
}

ctu_status ctu_step(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                    const void *cool_L0_dev, double *reg_dev, double *rate_dev, double *dpp_dev, int32_t *fails_dev,
                    void *stream)
{
    ctu_status st = check_step_args(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev);
    if (st != CTU_OK) return st;
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    hipStream_t s = (hipStream_t)stream;
    if (plan->esize == 4)
        return enqueue_step<float>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev, dpp_dev,
                                   fails_dev, s);
    return enqueue_step<double>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev, dpp_dev,
                                fails_dev, s);
}

ctu_status ctu_step_graph_capture(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                                  const void *cool_L0_dev, double *reg_dev, double *rate_dev, double *dpp_dev,
                                  int32_t *fails_dev, void *stream)
{
    ctu_status st = check_step_args(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev);
    if (st != CTU_OK) return st;
    if (!stream) return fail(CTU_ERR_ARG, "graph capture needs a non-default stream");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    hipStream_t s = (hipStream_t)stream;
    if ((st = drop_graph(plan)) != CTU_OK) return st;
    bool was_timing = plan->timing;
    plan->timing = false;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ctu_status st2 = (plan->esize == 4)
                         ? enqueue_step<float>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev,
                                               dpp_dev, fails_dev, s)
                         : enqueue_step<double>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev,
                                                dpp_dev, fails_dev, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    plan->timing = was_timing;
    if (st2 != CTU_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st2;
    }
    if (e != hipSuccess) return fail(CTU_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    plan->graph = g;
    HIP_TRY(hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0));
    HIP_TRY(hipGraphLaunch(plan->gexec, s));
    return CTU_OK;
}

ctu_status ctu_step_graph_launch(ctu_plan *plan, void *stream)
{
    if (!plan || !plan->gexec) return fail(CTU_ERR_ARG, "no captured graph");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    HIP_TRY(hipGraphLaunch(plan->gexec, (hipStream_t)stream));
    return CTU_OK;
}

ctu_status ctu_plan_enable_timing(ctu_plan *plan, int32_t enable)
{
    if (!plan) return fail(CTU_ERR_ARG, "null plan");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    if (enable && plan->tev.empty()) {
        plan->tev.assign(2 * (size_t)kMaxTimedSteps * CTU_NSTAGE, nullptr);
        for (auto &e : plan->tev) HIP_TRY(hipEventCreate(&e));
    }
    plan->tused.assign((size_t)kMaxTimedSteps * CTU_NSTAGE, 0);
    plan->tsteps = 0;
    plan->timing = enable != 0;
    return CTU_OK;
}

ctu_status ctu_plan_read_timing(ctu_plan *plan, double *ms_out, int32_t *nsteps_out)
{
    if (!plan || !ms_out) return fail(CTU_ERR_ARG, "plan and ms_out are required");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    for (int st = 0; st < CTU_NSTAGE; st++) ms_out[st] = 0.0;
    for (int step = 0; step < plan->tsteps; step++)
        for (int st = 0; st < CTU_NSTAGE; st++) {
            size_t idx = (size_t)step * CTU_NSTAGE + st;
            if (idx >= plan->tused.size() || !plan->tused[idx]) continue;
            HIP_TRY(hipEventSynchronize(plan->tev[2 * idx + 1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, plan->tev[2 * idx], plan->tev[2 * idx + 1]));
            ms_out[st] += ms;
        }
    if (nsteps_out) *nsteps_out = plan->tsteps;
    return CTU_OK;
}

ctu_status ctu_cfl_rate(ctu_plan *plan, const void *U_dev, double *rate_dev, void *stream)
{
    if (!plan || !U_dev || !rate_dev) return fail(CTU_ERR_ARG, "plan, U and rate are required");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_reset<0>, dim3(1), dim3(64), 0, s, rate_dev, (double *)nullptr, (int *)nullptr);
    HIP_TRY(hipGetLastError());
    int nb = plan->t_cfl.n();
    HIP_TRY(with_phys(plan->combo.phys, [&](auto P) {
        constexpr int PH = decltype(P)::value;
        if (plan->esize == 4)
            hipLaunchKernelGGL((k_cfl<PH, float>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->t_cfl.d,
                               (const float *)U_dev, rate_dev, plan->ko);
        else
            hipLaunchKernelGGL((k_cfl<PH, double>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->t_cfl.d,
                               (const double *)U_dev, rate_dev, plan->ko);
        return hipGetLastError();
    }));
    return CTU_OK;
}

ctu_status ctu_prim_to_cons(ctu_plan *plan, const void *V_dev, void *U_dev, void *stream)
{
    if (!plan || !V_dev || !U_dev) return fail(CTU_ERR_ARG, "plan, V and U are required");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    hipStream_t s = (hipStream_t)stream;
    int nb = plan->t_cells.n();
    HIP_TRY(with_phys(plan->combo.phys, [&](auto P) {
        constexpr int PH = decltype(P)::value;
        if (plan->esize == 4)
            hipLaunchKernelGGL((k_prim2cons<PH, float>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->t_cells.d,
                               (const float *)V_dev, (float *)U_dev, (float)plan->opts.gamma);
        else
            hipLaunchKernelGGL((k_prim2cons<PH, double>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->t_cells.d,
                               (const double *)V_dev, (double *)U_dev, plan->opts.gamma);
        return hipGetLastError();
    }));
    return CTU_OK;
}

ctu_status ctu_cons_to_prim(ctu_plan *plan, const void *U_dev, void *V_dev, int32_t *fails_dev, void *stream)
{
    if (!plan || !V_dev || !U_dev) return fail(CTU_ERR_ARG, "plan, U and V are required");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    hipStream_t s = (hipStream_t)stream;
    if (fails_dev) {
        hipLaunchKernelGGL(k_reset<0>, dim3(1), dim3(64), 0, s, (double *)nullptr, (double *)nullptr, (int *)fails_dev);
        HIP_TRY(hipGetLastError());
    }
    int nb = plan->t_cells.n();
    HIP_TRY(with_phys(plan->combo.phys, [&](auto P) {
        constexpr int PH = decltype(P)::value;
        if (plan->esize == 4)
            hipLaunchKernelGGL((k_cons2prim<PH, float>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->t_cells.d,
                               (const float *)U_dev, (float *)V_dev, (int *)fails_dev, (float)plan->opts.gamma, 0);
        else
            hipLaunchKernelGGL((k_cons2prim<PH, double>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->t_cells.d,
                               (const double *)U_dev, (double *)V_dev, (int *)fails_dev, plan->opts.gamma, 0);
        return hipGetLastError();
    }));
    return CTU_OK;
}

ctu_status ctu_plan_set_reflux(ctu_plan *plan, const ctu_refluxface *faces, int32_t nfaces)
{
    if (!plan) return fail(CTU_ERR_ARG, "null plan");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    HIP_TRY(hipDeviceSynchronize());  // a previous reflux may still read the old table
    return set_reflux_table(plan, faces, nfaces);
}

static ctu_status set_reflux_table(ctu_plan *plan, const ctu_refluxface *faces, int32_t nfaces)
{
    if (nfaces > 0 && !faces) return fail(CTU_ERR_ARG, "faces is null");
    // group the entries per coarse cell, keeping table order inside a cell
    std::map<std::pair<int, long long>, std::vector<int>> groups;
    std::vector<std::pair<int, long long>> order;
    for (int e = 0; e < nfaces; e++) {
        const ctu_refluxface &f = faces[e];
        if (f.box < 0 || f.box >= (int)plan->hboxes.size() || (f.side != 1 && f.side != -1) || f.nfine < 1 ||
            f.nfine > 4 || f.dir < 0 || f.dir >= plan->opts.dim || f.coarse_slot < 0)
            return fail(CTU_ERR_ARG, "bad reflux entry");
        const KBox &bx = plan->hboxes[f.box];
        if (f.i < 0 || f.i >= bx.N[0] || f.j < 0 || f.j >= bx.N[1] || f.k < 0 || f.k >= bx.N[2])
            return fail(CTU_ERR_ARG, "reflux cell outside its box");
        long long c = ((long long)f.k * bx.N[1] + f.j) * bx.N[0] + f.i;
        auto key = std::make_pair(f.box, c);
        if (!groups.count(key)) order.push_back(key);
        groups[key].push_back(e);
    }
    std::vector<KRefl> ents;
    std::vector<int> starts;
    for (auto &key : order) {
        starts.push_back((int)ents.size());
        for (int e : groups[key]) {
            const ctu_refluxface &f = faces[e];
            KRefl r;
            r.box = f.box;
            r.i = f.i;
            r.j = f.j;
            r.k = f.k;
            r.dir = f.dir;
            r.side = f.side;
            r.nfine = f.nfine;
            r.pad = 0;
            r.cslot = f.coarse_slot;
            for (int q = 0; q < 4; q++) r.fslot[q] = (q < f.nfine) ? f.fine_slot[q] : 0;
            // the correction per unit of register difference: -side / (face
            // area) / dx_dir (the register holds dt A F; A / V = 1 / dx_dir)
            const KBox &bx = plan->hboxes[f.box];
            double area = 1.0;
            for (int d = 0; d < 3; d++)
                if (d != f.dir && bx.n[d] > 0 && !(d == 2 && bx.N[2] == 1)) area *= bx.dx[d];
            r.scale = -(double)f.side / area * (1.0 / bx.dx[f.dir]);
            ents.push_back(r);
        }
    }
    starts.push_back((int)ents.size());
    if (plan->drefl) (void)hipFree(plan->drefl);
    if (plan->dcell_start) (void)hipFree(plan->dcell_start);
    plan->drefl = nullptr;
    plan->dcell_start = nullptr;
    plan->nrefl_cells = (int)order.size();
    ctu_status st;
    if ((st = upload(ents, &plan->drefl)) != CTU_OK) return st;
    if ((st = upload(starts, &plan->dcell_start)) != CTU_OK) return st;
    return CTU_OK;
}

static ctu_status reflux_launch(ctu_plan *plan, void *U_dev, double *reg_dev, int consume, void *stream)
{
    if (!plan || !U_dev || !reg_dev) return fail(CTU_ERR_ARG, "plan, U and reg are required");
    if (plan->nrefl_cells == 0) return CTU_OK;
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    int nb = (plan->nrefl_cells + NT - 1) / NT;
    hipStream_t s = (hipStream_t)stream;
    if (plan->esize == 4)
        hipLaunchKernelGGL((k_reflux<float>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->drefl, plan->dcell_start,
                           plan->nrefl_cells, (float *)U_dev, reg_dev, consume);
    else
        hipLaunchKernelGGL((k_reflux<double>), dim3(nb), dim3(NT), 0, s, plan->dboxes, plan->drefl,
                           plan->dcell_start, plan->nrefl_cells, (double *)U_dev, reg_dev, consume);
    HIP_TRY(hipGetLastError());
    return CTU_OK;
}

ctu_status ctu_reflux(ctu_plan *plan, void *U_dev, const double *reg_dev, void *stream)
{
    return reflux_launch(plan, U_dev, const_cast<double *>(reg_dev), 0, stream);
}

ctu_status ctu_reflux_consume(ctu_plan *plan, void *U_dev, double *reg_dev, void *stream)
{
    return reflux_launch(plan, U_dev, reg_dev, 1, stream);
}

ctu_status ctu_plan_set_leaf_mask(ctu_plan *plan, const uint8_t *leaf_dev)
{
    if (!plan) return fail(CTU_ERR_ARG, "null plan");
    plan->leaf = leaf_dev;
    return CTU_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free step: the workspace is a fixed device array of the library
// ---------------------------------------------------------------------------

namespace {

// The array is a per-device object of the code object: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.  Its
// name is only a host-side stand-in; launches use the address returned by
// hipGetSymbolAddress for the current device.
constexpr int64_t kScratchBytes = 64LL << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of its copy of `scratch`

// the device address of `scratch` on `dev`, which must be current
ctu_status scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return CTU_OK;
    }
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(CTU_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return CTU_OK;
}

// workspace pointers of a plan, saved around a step on the scratch
struct WsPtrs {
    void *V, *T[3], *Vh, *Lam, *F[3];
    unsigned char *Flag;
    explicit WsPtrs(const ctu_plan *p)
        : V(p->wsV), T{ p->wsT[0], p->wsT[1], p->wsT[2] }, Vh(p->wsVh), Lam(p->wsLam),
          F{ p->wsF[0], p->wsF[1], p->wsF[2] }, Flag(p->wsFlag)
    {
    }
    void restore(ctu_plan *p) const
    {
        p->wsV = V;
        p->wsVh = Vh;
        p->wsLam = Lam;
        p->wsFlag = Flag;
        for (int d = 0; d < 3; d++) {
            p->wsT[d] = T[d];
            p->wsF[d] = F[d];
        }
    }
};

}  // namespace

extern "C" {

int64_t ctu_static_scratch_bytes(void) { return kScratchBytes; }

ctu_status ctu_step_static(ctu_plan *plan, const void *U_in_dev, void *U_out_dev, const double *params_dev,
                           const void *cool_L0_dev, double *reg_dev, double *rate_dev, double *dpp_dev,
                           int32_t *fails_dev, void *stream)
{
    ctu_status st = check_step_args(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev, rate_dev, false);
    if (st != CTU_OK) return st;
    if (plan->ws_bytes > kScratchBytes)
        return fail(CTU_ERR_ARG, "the plan's workspace (" + std::to_string(plan->ws_bytes) +
                                     " bytes) exceeds the static scratch (" + std::to_string(kScratchBytes) +
                                     " bytes): step it with ctu_step, or split its boxes into smaller plans");
    DevGuard guard(plan->dev);
    HIP_TRY(guard.err);
    void *ptr = nullptr;
    if ((st = scratch_address(plan->dev, &ptr)) != CTU_OK) return st;
    // every scratch field is written before it is read within the step, so
    // nothing needs clearing; the previous call's contents are overwritten
    const WsPtrs saved(plan);
    carve_ws(plan, (char *)ptr);
    hipStream_t s = (hipStream_t)stream;
    st = (plan->esize == 4) ? enqueue_step<float>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev,
                                                  rate_dev, dpp_dev, fails_dev, s)
                            : enqueue_step<double>(plan, U_in_dev, U_out_dev, params_dev, cool_L0_dev, reg_dev,
                                                   rate_dev, dpp_dev, fails_dev, s);
    saved.restore(plan);
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// AMR hierarchy: ghost filling, restriction and the subcycled level cycle
// ---------------------------------------------------------------------------

namespace {

struct HierLevel {
    int N = 0;  // cells per side of the periodic level
    std::vector<HBox> hb;
    std::vector<int> nb_start, nb_list, cb_start, cb_list, pb_start, pb_list, ch_start, ch_list;
    std::vector<HTile> fill_t, avg_t, copy_t;
    std::vector<HCopy> copies;  // same-level ghost copy rectangles
    std::vector<HPar> pars;     // coarse parents of ghosts to prolong (levels >= 1)
    std::vector<int> multi;     // seven coarse boxes per parent whose stencil spans several
    HBox *db = nullptr;
    int *d_pb_start = nullptr, *d_pb_list = nullptr, *d_ch_start = nullptr, *d_ch_list = nullptr;
    HTile *d_fill_t = nullptr, *d_avg_t = nullptr, *d_copy_t = nullptr;
    HCopy *d_copies = nullptr;
    HPar *d_pars = nullptr;
    int *d_multi = nullptr;
};

int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// do [a0, a1) and [b0, b1) + s meet for a shift s in {-N, 0, N}?
bool meets_periodic(int a0, int a1, int b0, int b1, int N)
{
    for (int s = -N; s <= N; s += N)
        if (std::max(a0, b0 + s) < std::min(a1, b1 + s)) return true;
    return false;
}

// boxes whose interior meets the region [lo, hi) (per axis) under the
// periodic shifts of an N-cell level (or without shifts when N == 0)
void candidates(const std::vector<HBox> &boxes, const int lo[3], const int hi[3], int N, std::vector<int> &out)
{
    for (int c = 0; c < (int)boxes.size(); c++) {
        const HBox &b = boxes[c];
        bool ok = true;
        for (int d = 0; d < 3 && ok; d++) {
            if (N > 0) ok = meets_periodic(lo[d], hi[d], b.lo[d], b.lo[d] + b.n[d], N);
            else ok = std::max(lo[d], b.lo[d]) < std::min(hi[d], b.lo[d] + b.n[d]);
        }
        if (ok) out.push_back(c);
    }
}

long long overlap_volume(const HBox &a, const int lo[3], const int hi[3])
{
    long long v = 1;
    for (int d = 0; d < 3; d++) {
        int e = std::min(a.lo[d] + a.n[d], hi[d]) - std::max(a.lo[d], lo[d]);
        if (e <= 0) return 0;
        v *= e;
    }
    return v;
}

}  // namespace

struct ctu_hier {
    int dev = 0;  // the device current at creation: tables, counters and launches
    int esize = 8, base = 0, nlev = 0, ng = 0;
    std::vector<HierLevel> lev;
    int *dfails = nullptr;  // per-step failure counts inside the cycle
};

namespace {

void free_hier(ctu_hier *h)
{
    if (!h) return;
    DevGuard g(h->dev);
    for (HierLevel &L : h->lev) {
        void *ptrs[] = { L.db, L.d_pb_start, L.d_pb_list,
                         L.d_ch_start, L.d_ch_list, L.d_fill_t, L.d_avg_t, L.d_copy_t, L.d_copies, L.d_pars,
                         L.d_multi };
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
    }
    if (h->dfails) (void)hipFree(h->dfails);
    delete h;
}

bool holds_h(const HBox &b, int i, int j, int k)
{
    return i >= b.lo[0] && i < b.lo[0] + b.n[0] && j >= b.lo[1] && j < b.lo[1] + b.n[1] && k >= b.lo[2] &&
           k < b.lo[2] + b.n[2];
}

int wrap_h(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// The ghost-fill tables of one level (after its candidate lists): for each
// box, the rectangles of its ghosted extent that a same-level interior holds
// under a periodic shift, and on levels >= 1 the coarse parents of the ghost
// cells left over, each with its child mask and the coarse box that holds
// its whole 7-cell stencil (-1: several boxes, -2: not all held).
ctu_status build_fill_tables(ctu_hier *h, int l)
{
    HierLevel &L = h->lev[l];
    const int g = h->ng, N = L.N;
    for (int b = 0; b < (int)L.hb.size(); b++) {
        const HBox &B = L.hb[b];
        int lo[3], hi[3];
        for (int d = 0; d < 3; d++) {
            lo[d] = B.lo[d] - g;
            hi[d] = B.lo[d] + B.n[d] + g;
        }
        std::vector<unsigned char> cov((size_t)B.cells, 0);
        auto at = [&](int x, int y, int z) -> unsigned char & {
            return cov[((size_t)z * B.N[1] + y) * B.N[0] + x];
        };
        for (int z = g; z < g + B.n[2]; z++)
            for (int y = g; y < g + B.n[1]; y++)
                for (int x = g; x < g + B.n[0]; x++) at(x, y, z) = 1;
        // every periodic image of every candidate (all boxes of the level when
        // the ghost width reaches past the neighbouring images)
        const bool all = N <= 2 * g;
        const int ne = all ? (int)L.hb.size() : L.nb_start[b + 1] - L.nb_start[b];
        for (int e = 0; e < ne; e++) {
            const int c = all ? e : L.nb_list[L.nb_start[b] + e];
            const HBox &C = L.hb[c];
            int k0[3], k1[3];
            for (int d = 0; d < 3; d++) {
                k0[d] = floor_div(lo[d] - (C.lo[d] + C.n[d]), N) + 1;
                k1[d] = floor_div(hi[d] - 1 - C.lo[d], N);
            }
            for (int kz = k0[2]; kz <= k1[2]; kz++)
                for (int ky = k0[1]; ky <= k1[1]; ky++)
                    for (int kx = k0[0]; kx <= k1[0]; kx++) {
                        if (c == b && kx == 0 && ky == 0 && kz == 0) continue;
                        const int sh[3] = { kx * N, ky * N, kz * N };
                        HCopy cp{};
                        bool empty = false;
                        for (int d = 0; d < 3 && !empty; d++) {
                            const int a0 = std::max(lo[d], C.lo[d] + sh[d]);
                            const int a1 = std::min(hi[d], C.lo[d] + C.n[d] + sh[d]);
                            empty = a1 <= a0;
                            cp.dlo[d] = a0 - lo[d];
                            cp.slo[d] = a0 - sh[d] - (C.lo[d] - g);
                            cp.ext[d] = a1 - a0;
                        }
                        if (empty) continue;
                        cp.dst = b;
                        cp.src = c;
                        for (int z = 0; z < cp.ext[2]; z++)
                            for (int y = 0; y < cp.ext[1]; y++)
                                for (int x = 0; x < cp.ext[0]; x++) {
                                    unsigned char &m = at(cp.dlo[0] + x, cp.dlo[1] + y, cp.dlo[2] + z);
                                    if (m) return fail(CTU_ERR_ARG, "same-level boxes overlap under the periodic shifts");
                                    m = 1;
                                }
                        const int ncell = cp.ext[0] * cp.ext[1] * cp.ext[2];
                        const int id = (int)L.copies.size();
                        L.copies.push_back(cp);
                        for (int s0 = 0; s0 < ncell; s0 += NT) L.copy_t.push_back(HTile{ id, s0 });
                    }
        }
        if (l == 0) {
            for (unsigned char m : cov)
                if (!m) return fail(CTU_ERR_ARG, "a level-0 ghost cell lies in no box (level 0 must cover the domain)");
            continue;
        }
        const HierLevel &Cl = h->lev[l - 1];
        const int Nc = N / 2;
        int p0[3], p1[3];
        for (int d = 0; d < 3; d++) {
            p0[d] = floor_div(lo[d], 2);
            p1[d] = floor_div(hi[d] - 1, 2);
        }
        for (int pz = p0[2]; pz <= p1[2]; pz++)
            for (int py = p0[1]; py <= p1[1]; py++)
                for (int px = p0[0]; px <= p1[0]; px++) {
                    HPar P{};
                    P.box = b;
                    const int pu[3] = { px, py, pz };
                    for (int d = 0; d < 3; d++) P.f0[d] = 2 * pu[d] - lo[d];
                    for (int c8 = 0; c8 < 8; c8++) {
                        const int x = P.f0[0] + (c8 & 1), y = P.f0[1] + ((c8 >> 1) & 1), z = P.f0[2] + ((c8 >> 2) & 1);
                        if (x < 0 || y < 0 || z < 0 || x >= B.N[0] || y >= B.N[1] || z >= B.N[2]) continue;
                        if (!at(x, y, z)) P.mask |= 1u << c8;
                    }
                    if (!P.mask) continue;
                    for (int d = 0; d < 3; d++) P.pc[d] = wrap_h(pu[d], Nc);
                    // the coarse boxes of the parent and its six face
                    // neighbours (-x, +x, -y, +y, -z, +z)
                    int ob[7];
                    bool held_all = true, one = true;
                    for (int t = 0; t < 7 && held_all; t++) {
                        int q[3] = { P.pc[0], P.pc[1], P.pc[2] };
                        if (t > 0) q[(t - 1) / 2] = wrap_h(q[(t - 1) / 2] + ((t & 1) ? -1 : 1), Nc);
                        ob[t] = -1;
                        for (int e = L.cb_start[b]; e < L.cb_start[b + 1] && ob[t] < 0; e++)
                            if (holds_h(Cl.hb[L.cb_list[e]], q[0], q[1], q[2])) ob[t] = L.cb_list[e];
                        held_all = ob[t] >= 0;
                        one = one && held_all && ob[t] == ob[0];
                    }
                    if (!held_all) {
                        P.cbox = HPAR_MISSING;
                    } else if (one) {
                        P.cbox = ob[0];
                    } else {
                        P.cbox = -1 - (int)(L.multi.size() / 7);
                        L.multi.insert(L.multi.end(), ob, ob + 7);
                    }
                    L.pars.push_back(P);
                }
    }
    return CTU_OK;
}

template <typename R>
ctu_status hier_fill(ctu_hier *h, int level, void *U, const void *Uo, const void *Un, double alpha, int32_t *missing,
                     hipStream_t s)
{
    HierLevel &L = h->lev[level];
    // same-level copies (and, on level 0, the periodic images), then on
    // finer levels the remaining ghosts, prolonged one coarse parent per
    // thread; the two write disjoint cells and read no cell the other writes
    if (!L.copy_t.empty()) {
        hipLaunchKernelGGL((k_hcopy<R>), dim3((unsigned)L.copy_t.size()), dim3(NT), 0, s, L.db, L.d_copies,
                           L.d_copy_t, (R *)U);
        HIP_TRY(hipGetLastError());
    }
    if (level > 0 && !L.pars.empty()) {
        const unsigned nb = (unsigned)((L.pars.size() + NT - 1) / NT);
        hipLaunchKernelGGL((k_hprolong<R>), dim3(nb), dim3(NT), 0, s, L.db, L.d_pars, (int)L.pars.size(),
                           L.d_multi, h->lev[level - 1].db, L.N, h->ng, (R *)U, (const R *)Uo,
                           (const R *)(Un ? Un : Uo), alpha, (int *)missing);
        HIP_TRY(hipGetLastError());
    }
    return CTU_OK;
}

template <typename R>
ctu_status hier_avg(ctu_hier *h, int fine, const void *Uf, void *Uc, hipStream_t s)
{
    HierLevel &F = h->lev[fine];
    if (F.avg_t.empty()) return CTU_OK;
    hipLaunchKernelGGL((k_havg<R>), dim3((unsigned)F.avg_t.size()), dim3(NT), 0, s, F.db, F.d_avg_t, F.d_pb_start,
                       F.d_pb_list, h->lev[fine - 1].db, h->ng, (const R *)Uf, (R *)Uc, (int *)nullptr);
    HIP_TRY(hipGetLastError());
    return CTU_OK;
}

ctu_status hier_fill_any(ctu_hier *h, int level, void *U, const void *Uo, const void *Un, double alpha,
                         int32_t *missing, hipStream_t s)
{
    return h->esize == 4 ? hier_fill<float>(h, level, U, Uo, Un, alpha, missing, s)
                         : hier_fill<double>(h, level, U, Uo, Un, alpha, missing, s);
}

ctu_status hier_avg_any(ctu_hier *h, int fine, const void *Uf, void *Uc, hipStream_t s)
{
    return h->esize == 4 ? hier_avg<float>(h, fine, Uf, Uc, s) : hier_avg<double>(h, fine, Uf, Uc, s);
}

struct CycleArgs {
    ctu_hier *h;
    ctu_plan *const *plans;
    void *const *Ua;
    void *const *Ub;
    int32_t *cur;
    const double *const *params;
    double *reg, *rate, *dpp;
    int32_t *fails, *missing;
    const void *const *L0;
    hipStream_t s;
};

// advance `lev` by its dt; then, when a finer level exists, advance it twice
// (ghosts from this level's old / new states at alpha = 0 and 1/2),
// restrict it and reflux this level
ctu_status advance_level(const CycleArgs &c, int lev, const void *pold, const void *pnew, double alpha)
{
    ctu_hier *h = c.h;
    void *in = c.cur[lev] ? c.Ub[lev] : c.Ua[lev];
    void *out = c.cur[lev] ? c.Ua[lev] : c.Ub[lev];
    ctu_status st = hier_fill_any(h, lev, in, pold, pnew, alpha, c.missing, c.s);
    if (st != CTU_OK) return st;
    st = ctu_step(c.plans[lev], in, out, c.params[lev], c.L0 ? c.L0[lev] : nullptr, c.reg, c.rate + lev,
                  c.dpp ? c.dpp + lev : nullptr, h->dfails, c.s);
    if (st != CTU_OK) return st;
    if (c.fails) {
        hipLaunchKernelGGL(k_add_fails, dim3(1), dim3(64), 0, c.s, (int *)c.fails, (const int *)h->dfails);
        HIP_TRY(hipGetLastError());
    }
    c.cur[lev] ^= 1;
    if (lev + 1 < h->nlev) {
        for (int q = 0; q < 2; q++)
            if ((st = advance_level(c, lev + 1, in, out, 0.5 * q)) != CTU_OK) return st;
        const void *fine_now = c.cur[lev + 1] ? c.Ub[lev + 1] : c.Ua[lev + 1];
        if ((st = hier_avg_any(h, lev + 1, fine_now, out, c.s)) != CTU_OK) return st;
        if ((st = reflux_launch(c.plans[lev], out, c.reg, 1, (void *)c.s)) != CTU_OK) return st;
    }
    return CTU_OK;
}

}  // namespace

extern "C" {

ctu_status ctu_hier_create(int32_t precision, int32_t base, int32_t nlev, const int32_t *level_nbox,
                           const ctu_box *boxes, int32_t nghost, ctu_hier **out)
{
    if (!out) return fail(CTU_ERR_ARG, "out is required");
    *out = nullptr;
    if (precision != CTU_FP32 && precision != CTU_FP64) return fail(CTU_ERR_ARG, "bad precision");
    if (base < 2 || nlev < 1 || nlev > 16 || nghost < 1 || !level_nbox || !boxes)
        return fail(CTU_ERR_ARG, "need base >= 2, 1 <= nlev <= 16, nghost >= 1, level_nbox and boxes");
    if ((long long)base << (nlev - 1) > (1LL << 30)) return fail(CTU_ERR_ARG, "finest level too large");
    ctu_hier *h = new ctu_hier();
    if (hipGetDevice(&h->dev) != hipSuccess) h->dev = 0;  // host checks below report first; uploads then fail
    h->esize = (precision == CTU_FP32) ? 4 : 8;
    h->base = base;
    h->nlev = nlev;
    h->ng = nghost;
    h->lev.resize(nlev);
    int pos = 0;
    for (int l = 0; l < nlev; l++) {
        HierLevel &L = h->lev[l];
        L.N = base << l;
        if (level_nbox[l] < 0) {
            free_hier(h);
            return fail(CTU_ERR_ARG, "negative box count");
        }
        for (int b = 0; b < level_nbox[l]; b++, pos++) {
            const ctu_box &B = boxes[pos];
            HBox hb{};
            long long cells = 1;
            for (int d = 0; d < 3; d++) {
                hb.lo[d] = B.lo[d];
                hb.n[d] = B.n[d];
                hb.N[d] = B.n[d] + 2 * nghost;
                cells *= hb.N[d];
                if (B.n[d] < 1 || B.lo[d] < 0 || B.lo[d] + B.n[d] > L.N || (l > 0 && ((B.lo[d] | B.n[d]) & 1))) {
                    free_hier(h);
                    return fail(CTU_ERR_ARG, "box outside its level, empty, or (levels >= 1) not 2-aligned");
                }
            }
            if (B.level != l || B.offset < 0) {
                free_hier(h);
                return fail(CTU_ERR_ARG, "box level must match its position; offsets must be >= 0");
            }
            if (NV * cells * h->esize > 0xFFFFFFFFLL) {
                free_hier(h);
                return fail(CTU_ERR_ARG, "a box's nine variable planes must fit in 4 GiB");
            }
            hb.off = B.offset;
            hb.cells = cells;
            L.hb.push_back(hb);
        }
        // disjoint interiors; level 0 covers the domain
        long long vol = 0;
        for (size_t a = 0; a < L.hb.size(); a++) {
            int hi[3];
            for (int d = 0; d < 3; d++) hi[d] = L.hb[a].lo[d] + L.hb[a].n[d];
            vol += (long long)L.hb[a].n[0] * L.hb[a].n[1] * L.hb[a].n[2];
            for (size_t c = a + 1; c < L.hb.size(); c++)
                if (overlap_volume(L.hb[c], L.hb[a].lo, hi) > 0) {
                    free_hier(h);
                    return fail(CTU_ERR_ARG, "boxes of one level overlap");
                }
        }
        if (l == 0 && vol != (long long)L.N * L.N * L.N) {
            free_hier(h);
            return fail(CTU_ERR_ARG, "level 0 must cover the periodic domain");
        }
    }
    for (int l = 0; l < nlev; l++) {
        HierLevel &L = h->lev[l];
        L.nb_start.push_back(0);
        L.cb_start.push_back(0);
        L.pb_start.push_back(0);
        for (int b = 0; b < (int)L.hb.size(); b++) {
            const HBox &B = L.hb[b];
            int lo[3], hi[3];
            for (int d = 0; d < 3; d++) {
                lo[d] = B.lo[d] - nghost;
                hi[d] = B.lo[d] + B.n[d] + nghost;
            }
            candidates(L.hb, lo, hi, L.N, L.nb_list);
            L.nb_start.push_back((int)L.nb_list.size());
            if (l > 0) {
                const HierLevel &C = h->lev[l - 1];
                int clo[3], chi[3], flo[3], fhi[3];
                for (int d = 0; d < 3; d++) {
                    clo[d] = floor_div(lo[d], 2) - 1;
                    chi[d] = floor_div(hi[d] - 1, 2) + 2;
                    flo[d] = B.lo[d] / 2;
                    fhi[d] = (B.lo[d] + B.n[d]) / 2;
                }
                candidates(C.hb, clo, chi, C.N, L.cb_list);
                size_t p0 = L.pb_list.size();
                candidates(C.hb, flo, fhi, 0, L.pb_list);
                long long cover = 0;
                for (size_t e = p0; e < L.pb_list.size(); e++) cover += overlap_volume(C.hb[L.pb_list[e]], flo, fhi);
                if (cover != (long long)(fhi[0] - flo[0]) * (fhi[1] - flo[1]) * (fhi[2] - flo[2])) {
                    free_hier(h);
                    return fail(CTU_ERR_ARG, "a fine box is not covered by the coarser level (nesting)");
                }
            }
            L.cb_start.push_back((int)L.cb_list.size());
            L.pb_start.push_back((int)L.pb_list.size());
            for (long long s0 = 0; s0 < B.cells; s0 += NT) L.fill_t.push_back(HTile{ b, (int)s0 });
            if (l > 0) {
                long long fc = (long long)(B.n[0] / 2) * (B.n[1] / 2) * (B.n[2] / 2);
                for (long long s0 = 0; s0 < fc; s0 += NT) L.avg_t.push_back(HTile{ b, (int)s0 });
            }
        }
    }
    // ghost-fill tables
    for (int l = 0; l < nlev; l++) {
        ctu_status st = build_fill_tables(h, l);
        if (st != CTU_OK) {
            free_hier(h);
            return st;
        }
    }
    // children: boxes of the next finer level whose footprint meets each box
    for (int l = 0; l < nlev; l++) {
        HierLevel &L = h->lev[l];
        L.ch_start.push_back(0);
        for (const HBox &B : L.hb) {
            if (l + 1 < nlev) {
                int lo[3], hi[3];
                for (int d = 0; d < 3; d++) {
                    lo[d] = 2 * B.lo[d];
                    hi[d] = 2 * (B.lo[d] + B.n[d]);
                }
                candidates(h->lev[l + 1].hb, lo, hi, 0, L.ch_list);
            }
            L.ch_start.push_back((int)L.ch_list.size());
        }
    }
    // every check passed: upload the tables
    for (int l = 0; l < nlev; l++) {
        HierLevel &L = h->lev[l];
        ctu_status st;
        if ((st = upload(L.ch_start, &L.d_ch_start)) != CTU_OK || (st = upload(L.ch_list, &L.d_ch_list)) != CTU_OK) {
            free_hier(h);
            return st;
        }
        if ((st = upload(L.hb, &L.db)) != CTU_OK || (st = upload(L.pb_start, &L.d_pb_start)) != CTU_OK ||
            (st = upload(L.pb_list, &L.d_pb_list)) != CTU_OK || (st = upload(L.fill_t, &L.d_fill_t)) != CTU_OK ||
            (st = upload(L.copy_t, &L.d_copy_t)) != CTU_OK || (st = upload(L.copies, &L.d_copies)) != CTU_OK ||
            (st = upload(L.pars, &L.d_pars)) != CTU_OK || (st = upload(L.multi, &L.d_multi)) != CTU_OK ||
            (st = upload(L.avg_t, &L.d_avg_t)) != CTU_OK) {
            free_hier(h);
            return st;
        }
    }
    if (hipMalloc((void **)&h->dfails, 8 * sizeof(int)) != hipSuccess) {
        free_hier(h);
        return fail(CTU_ERR_NOMEM, "hipMalloc of the cycle counters failed");
    }
    *out = h;
    return CTU_OK;
}

void ctu_hier_destroy(ctu_hier *h) { free_hier(h); }

ctu_status ctu_hier_fill_ghosts(ctu_hier *h, int32_t level, void *U_dev, const void *Uc_old_dev,
                                const void *Uc_new_dev, double alpha, int32_t *missing_dev, void *stream)
{
    if (!h || !U_dev || level < 0 || level >= h->nlev) return fail(CTU_ERR_ARG, "bad hierarchy, level or U");
    if (level > 0 && !Uc_old_dev) return fail(CTU_ERR_ARG, "levels >= 1 need the coarse state");
    if (level > 0 && alpha != 0.0 && !Uc_new_dev) return fail(CTU_ERR_ARG, "alpha != 0 needs the new coarse state");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(CTU_ERR_ARG, "alpha must lie in [0, 1]");
    DevGuard guard(h->dev);
    HIP_TRY(guard.err);
    return hier_fill_any(h, level, U_dev, Uc_old_dev, Uc_new_dev, alpha, missing_dev, (hipStream_t)stream);
}

ctu_status ctu_hier_average_down(ctu_hier *h, int32_t fine_level, const void *U_fine_dev, void *U_coarse_dev,
                                 void *stream)
{
    if (!h || fine_level < 1 || fine_level >= h->nlev || !U_fine_dev || !U_coarse_dev)
        return fail(CTU_ERR_ARG, "bad hierarchy, level or states");
    DevGuard guard(h->dev);
    HIP_TRY(guard.err);
    return hier_avg_any(h, fine_level, U_fine_dev, U_coarse_dev, (hipStream_t)stream);
}

ctu_status ctu_hier_advance(ctu_hier *h, ctu_plan *const *plans, void *const *U_a, void *const *U_b, int32_t *cur,
                            const double *const *params_dev, const void *const *cool_L0_dev, double *reg_dev,
                            double *rate_dev, double *dpp_dev, int32_t *fails_dev, int32_t *missing_dev, void *stream)
{
    if (!h || !plans || !U_a || !U_b || !cur || !params_dev || !rate_dev)
        return fail(CTU_ERR_ARG, "hierarchy, plans, states, cur, params and rate are required");
    for (int l = 0; l < h->nlev; l++) {
        if (!plans[l] || !U_a[l] || !U_b[l] || !params_dev[l] || (cur[l] != 0 && cur[l] != 1))
            return fail(CTU_ERR_ARG, "every level needs a plan, two state buffers, params and cur in {0, 1}");
        if (plans[l]->esize != h->esize) return fail(CTU_ERR_ARG, "plan and hierarchy precisions differ");
        if (plans[l]->hboxes.size() != h->lev[l].hb.size())
            return fail(CTU_ERR_ARG, "plan of a level must hold that level's boxes");
        if (plans[l]->dev != h->dev) return fail(CTU_ERR_ARG, "plans and hierarchy belong to different devices");
        if (!plans[l]->has_ws) return fail(CTU_ERR_ARG, "a level's plan has no workspace");
    }
    DevGuard guard(h->dev);
    HIP_TRY(guard.err);

    CycleArgs c{ h,       plans,     U_a,       U_b,         cur,         params_dev,         reg_dev,
                 rate_dev, dpp_dev, fails_dev, missing_dev, cool_L0_dev, (hipStream_t)stream };
    return advance_level(c, 0, nullptr, nullptr, 0.0);
}

ctu_status ctu_hier_leaf_mask(ctu_hier *h, int32_t level, uint8_t *leaf_dev, void *stream)
{
    if (!h || !leaf_dev || level < 0 || level >= h->nlev) return fail(CTU_ERR_ARG, "bad hierarchy, level or mask");
    DevGuard guard(h->dev);
    HIP_TRY(guard.err);
    HierLevel &L = h->lev[level];
    if (L.fill_t.empty()) return CTU_OK;
    const HBox *fbox = (level + 1 < h->nlev) ? h->lev[level + 1].db : nullptr;
    hipLaunchKernelGGL(k_hleaf, dim3((unsigned)L.fill_t.size()), dim3(NT), 0, (hipStream_t)stream, L.db, L.d_fill_t,
                       L.d_ch_start, L.d_ch_list, fbox, h->ng, (unsigned char *)leaf_dev);
    HIP_TRY(hipGetLastError());
    return CTU_OK;
}

ctu_status ctu_hier_tag(ctu_hier *h, int32_t level, const void *U_dev, int32_t var, double eps, double chi_r,
                        uint8_t *tags_dev, int32_t *ntag_dev, void *stream)
{
    if (!h || !U_dev || !tags_dev || level < 0 || level >= h->nlev) return fail(CTU_ERR_ARG, "bad hierarchy, level or arrays");
    if (var < 0 || var >= NV || !(eps >= 0.0)) return fail(CTU_ERR_ARG, "var must name a conserved variable; eps >= 0");
    DevGuard guard(h->dev);
    HIP_TRY(guard.err);
    HierLevel &L = h->lev[level];
    if (L.fill_t.empty()) return CTU_OK;
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 4)
        hipLaunchKernelGGL((k_htag<float>), dim3((unsigned)L.fill_t.size()), dim3(NT), 0, s, L.db, L.d_fill_t, h->ng,
                           (const float *)U_dev, var, eps, chi_r, (unsigned char *)tags_dev, (int *)ntag_dev);
    else
        hipLaunchKernelGGL((k_htag<double>), dim3((unsigned)L.fill_t.size()), dim3(NT), 0, s, L.db, L.d_fill_t, h->ng,
                           (const double *)U_dev, var, eps, chi_r, (unsigned char *)tags_dev, (int *)ntag_dev);
    HIP_TRY(hipGetLastError());
    return CTU_OK;
}

ctu_status ctu_hier_next_dt(ctu_hier *h, const double *rate_dev, const double *dpp_dev, double cfl, double eps_c,
                            double *const *params_dev, void *stream)
{
    if (!h || !rate_dev || !params_dev || !(cfl > 0.0) || !(eps_c > 0.0))
        return fail(CTU_ERR_ARG, "hierarchy, rate and params are required; cfl, eps_c > 0");
    HDtArgs a{};
    for (int l = 0; l < h->nlev; l++) {
        if (!params_dev[l]) return fail(CTU_ERR_ARG, "params of every level are required");
        a.params[l] = params_dev[l];
    }
    a.rate = rate_dev;
    a.dpp = dpp_dev;
    a.nlev = h->nlev;
    a.cfl = cfl;
    a.eps_c = eps_c;
    DevGuard guard(h->dev);
    HIP_TRY(guard.err);
    hipLaunchKernelGGL(k_next_dt, dim3(1), dim3(64), 0, (hipStream_t)stream, a);
    HIP_TRY(hipGetLastError());
    return CTU_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Measurement helpers: the rates this build can reach on the device, timed
// with HIP events (the roofline fractions are quoted against them beside the
// published peaks).
// ---------------------------------------------------------------------------

namespace {

// eight independent FMA chains per lane, 16 steps per iteration; the chains
// converge to c / (1 - b) and their sum is stored so that none is removed
template <typename R>
__global__ __launch_bounds__(NT) void k_fma_peak(R *out, int iters, R b, R c)
{
    R a0 = R(threadIdx.x) * R(1e-3), a1 = a0 + R(1), a2 = a0 + R(2), a3 = a0 + R(3), a4 = a0 + R(4),
      a5 = a0 + R(5), a6 = a0 + R(6), a7 = a0 + R(7);
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int u = 0; u < 16; u++) {
            a0 = fma(a0, b, c);
            a1 = fma(a1, b, c);
            a2 = fma(a2, b, c);
            a3 = fma(a3, b, c);
            a4 = fma(a4, b, c);
            a5 = fma(a5, b, c);
            a6 = fma(a6, b, c);
            a7 = fma(a7, b, c);
        }
    }
    out[(size_t)blockIdx.x * NT + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

__global__ __launch_bounds__(NT) void k_copy_peak(const float4 *src, float4 *dst, long long n)
{
    for (long long k = (long long)blockIdx.x * NT + threadIdx.x; k < n; k += (long long)gridDim.x * NT) dst[k] = src[k];
}

// milliseconds of `reps` launches of f on the current device's null stream
template <typename F> ctu_status time_launches(F f, int reps, double *ms)
{
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CTU_ERR_HIP, "hipEventCreate failed");
    }
    f();  // warm-up
    hipError_t e = hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && e == hipSuccess; r++) {
        f();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(CTU_ERR_HIP, std::string("peak measurement: ") + hipGetErrorString(e));
    *ms = t;
    return CTU_OK;
}

}  // namespace

extern "C" {

ctu_status ctu_measure_fma(int32_t precision, int32_t nblocks, int32_t iters, void *out_dev, double *tflops_out)
{
    if ((precision != CTU_FP32 && precision != CTU_FP64) || nblocks < 1 || iters < 1 || !out_dev || !tflops_out)
        return fail(CTU_ERR_ARG, "precision FP32 or FP64, nblocks >= 1, iters >= 1, out and tflops_out required");
    const int reps = 5;
    double ms = 0.0;
    ctu_status st;
    if (precision == CTU_FP32)
        st = time_launches([&] { hipLaunchKernelGGL(k_fma_peak<float>, dim3(nblocks), dim3(NT), 0, nullptr,
                                                    (float *)out_dev, iters, 0.999f, 1e-3f); }, reps, &ms);
    else
        st = time_launches([&] { hipLaunchKernelGGL(k_fma_peak<double>, dim3(nblocks), dim3(NT), 0, nullptr,
                                                    (double *)out_dev, iters, 0.999, 1e-3); }, reps, &ms);
    if (st != CTU_OK) return st;
    const double flop = 2.0 * 8.0 * 16.0 * (double)iters * (double)nblocks * NT * reps;
    *tflops_out = flop / (ms * 1e-3) / 1e12;
    return CTU_OK;
}

ctu_status ctu_measure_copy(const void *src_dev, void *dst_dev, int64_t bytes, double *gbs_out)
{
    if (!src_dev || !dst_dev || bytes < 16 || (bytes & 15) || !gbs_out)
        return fail(CTU_ERR_ARG, "src, dst and gbs_out required; bytes a positive multiple of 16");
    const int reps = 10;
    const long long n = bytes / 16;
    double ms = 0.0;
    ctu_status st = time_launches([&] { hipLaunchKernelGGL(k_copy_peak, dim3(256 * 16), dim3(NT), 0, nullptr,
                                                           (const float4 *)src_dev, (float4 *)dst_dev, n); }, reps, &ms);
    if (st != CTU_OK) return st;
    *gbs_out = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return CTU_OK;
}

}  // extern "C"
