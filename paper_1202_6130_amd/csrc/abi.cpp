// C-ABI implementation of lbm.h: parameter validation, workspace layout,
// kernel launches on the caller's stream, diagnostics and the small host-side
// least-squares solves of the contact-angle and slip measurements.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "copy.hpp"
#include "launch.hpp"

using namespace lbmwet;

namespace {

thread_local std::string g_err;
// Message slot of the context whose entry point is running on this thread
// (set by CtxScope), so that an error is also kept with its context.
thread_local std::string *g_ctx_err = nullptr;

lbm_status fail(lbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    if (g_ctx_err) *g_ctx_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                            \
    do {                                     \
        lbm_status s_ = (expr);              \
        if (s_ != LBM_OK) return s_;         \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t storage_bytes(int st) { return st == LBM_STORE_F16DEV ? 2 : (st == LBM_STORE_F64 ? 8 : 4); }
size_t compute_bytes(int st) { return (st == LBM_STORE_F64 || st == LBM_STORE_F32X) ? 8 : 4; }
int kernel_storage(int st) {
    switch (st) {
    case LBM_STORE_F16DEV: return STORE_F16;
    case LBM_STORE_F64: return STORE_F64;
    case LBM_STORE_F32X: return STORE_F32X;
    default: return STORE_F32;
    }
}
int compute_is_f64(int st) { return compute_bytes(st) == 8; }

uint32_t default_seg_rows(uint32_t nx, uint32_t ny) {
    // enough waves to fill 256 CUs several times over, without making the
    // halo rows (2 per segment) a large share of the loads
    const uint32_t strips = (nx + kStripColsHost - 1) / kStripColsHost;
    uint64_t want = 16384;
    uint32_t rows = 64;
    while (rows > 8 && uint64_t(strips) * ((ny + rows - 1) / rows) < want) rows /= 2;
    return rows < ny ? rows : ny;
}

struct Layout {
    size_t fa, fb, mom, uprev, row_tab, node_tab, phi_raw, partials, iso_part, small, profile, total;
    uint32_t strips, segs, seg_rows, waves, iso_blocks;
    uint32_t tiles;                // largest step-tile count over the tile shapes
    uint32_t pstride;              // population plane stride (elements)
};

#ifndef LBM_PLANE_PAD_BYTES
#define LBM_PLANE_PAD_BYTES 3840
#endif

// Population plane stride.  Planes of a lattice above 1 MiB per plane are
// spaced by nx*ny plus a pad of LBM_PLANE_PAD_BYTES (a multiple of 256, so
// rows keep their alignment): the nine load and nine store streams of a tile
// then do not all start at one offset modulo large powers of two, which costs
// the tiled step several percent of bandwidth on MI355X.
uint32_t plane_stride(const lbm_params &p) {
    const size_t N = size_t(p.nx) * p.ny, s = storage_bytes(p.storage);
    if (N * s < (size_t(1) << 20)) return uint32_t(N);
    return uint32_t(N + LBM_PLANE_PAD_BYTES / s);
}

// Populations per node of the parameters' velocity set.
int pop_count(const lbm_params &p) { return p.lattice == LBM_D2Q21 ? 21 : 9; }

// Offsets (bytes) into one lattice's workspace.  fb and mom are adjacent: the
// pair doubles as staging for host float64 arrays at creation.  For D2Q21 the
// diagnostic partial rows follow its own tiling (one per workgroup).
Layout make_layout(const lbm_params &p) {
    Layout L{};
    const size_t N = size_t(p.nx) * p.ny, s = storage_bytes(p.storage), cb = compute_bytes(p.storage);
    L.seg_rows = p.seg_rows > 0 ? uint32_t(p.seg_rows) : default_seg_rows(p.nx, p.ny);
    if (L.seg_rows > uint32_t(p.ny)) L.seg_rows = p.ny;
    L.strips = (uint32_t(p.nx) + kStripColsHost - 1) / kStripColsHost;
    L.segs = (uint32_t(p.ny) + L.seg_rows - 1) / L.seg_rows;
    L.waves = L.strips * L.segs;
    // batch work-list capacity: the largest tile count over the shapes plus
    // the largest block count over the two-step variants (both lists are kept)
    uint32_t t1 = 0, t2 = 0;
    for (int s = 0; s < kNumTileShapes; ++s) t1 = std::max(t1, step_tiles(uint32_t(p.nx), uint32_t(p.ny), s));
    for (int v = 0; v < kPass2Variants; ++v) t2 = std::max(t2, pass2_blocks(uint32_t(p.nx), uint32_t(p.ny), v));
    L.tiles = t1 + t2;
    L.iso_blocks = isoline_blocks(uint32_t(N));
    size_t o = 0;
    L.pstride = plane_stride(p);
    const size_t P = L.pstride, nq = size_t(pop_count(p));
    // D2Q21: one row of diagnostic partials per workgroup
    if (p.lattice == LBM_D2Q21) L.waves = q21_tiles(uint32_t(p.nx), uint32_t(p.ny));
    L.fa = o; o = align_up(o + nq * P * s);
    L.fb = o; o = o + nq * P * s;                      // no padding: fb+mom contiguous
    L.mom = o; o = align_up(o + 3 * N * cb);
    L.uprev = o; o = align_up(o + 2 * N * cb);
    const bool node = p.wall_kind == LBM_WALL_FIELDS || p.wall_kind == LBM_WALL_MASK;
    L.row_tab = o; o = align_up(o + 2 * size_t(p.ny) * cb);
    L.node_tab = o; o = align_up(o + (node ? 3 * N * cb : 0));
    L.phi_raw = o; o = align_up(o + (node ? N : size_t(p.ny)) * sizeof(double));
    L.partials = o; o = align_up(o + size_t(L.waves) * 8 * sizeof(double));
    L.iso_part = o; o = align_up(o + size_t(L.iso_blocks) * 10 * sizeof(double));
    L.small = o; o = align_up(o + 64 * sizeof(double));
    L.profile = o; o = align_up(o + size_t(p.ny) * sizeof(double));
    L.total = o;
    return L;
}

lbm_status validate(const lbm_params *p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1) return fail(LBM_EINVAL, "nx, ny must be >= 1 (got %d, %d)", p->nx, p->ny);
    if (p->storage != LBM_STORE_F32 && p->storage != LBM_STORE_F16DEV && p->storage != LBM_STORE_F64 &&
        p->storage != LBM_STORE_F32X)
        return fail(LBM_EINVAL, "unknown storage %d", p->storage);
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D2Q21) return fail(LBM_EINVAL, "unknown lattice %d", p->lattice);
    if ((int64_t(p->nx) * p->ny + LBM_PLANE_PAD_BYTES) * pop_count(*p) * int64_t(storage_bytes(p->storage)) >=
        (int64_t(1) << 32))
        return fail(LBM_EINVAL, "lattice too large: Q*(nx*ny + pad)*bytes must be < 2^32");
    if (p->psi_kind != LBM_PSI_EXP && p->psi_kind != LBM_PSI_EOS)
        return fail(LBM_EINVAL, "unknown psi_kind %d", p->psi_kind);
    if (p->collision != LBM_COLL_BGK && p->collision != LBM_COLL_PROJECTED)
        return fail(LBM_EINVAL, "unknown collision %d", p->collision);
    if (p->lattice == LBM_D2Q21 && p->storage != LBM_STORE_F32 && p->storage != LBM_STORE_F64)
        return fail(LBM_EINVAL, "D2Q21 takes storage F32 or F64");
    if (p->psi_kind == LBM_PSI_EOS) {
        if (p->lattice != LBM_D2Q21) return fail(LBM_EINVAL, "the EOS pseudo-potential is built for D2Q21");
        for (double v : p->eos)
            if (!isfinite(v)) return fail(LBM_EINVAL, "non-finite eos parameter");
        if (!(p->eos[3] > 0) || !(p->eos[4] > p->eos[3]))
            return fail(LBM_EINVAL, "eos needs 0 < rho_1 < rho_2");
    }
    if (p->wall_kind == LBM_WALL_MASK &&
        !(p->filter_wall >= 1 && p->filter_wall <= 1000 && p->filter_core >= 0 && p->filter_core <= p->filter_wall))
        return fail(LBM_EINVAL, "mask walls need 0 <= filter_core <= filter_wall <= 1000, filter_wall >= 1 (got %d, %d)",
                    p->filter_core, p->filter_wall);
    if (p->wall_kind < LBM_WALL_NONE || p->wall_kind > LBM_WALL_MASK)
        return fail(LBM_EINVAL, "unknown wall_kind %d", p->wall_kind);
    if (!(p->tau > 0.5) || !isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be > 0.5");
    if (!(p->eps >= 1.0) || !isfinite(p->eps)) return fail(LBM_EINVAL, "eps must be >= 1");
    const double vals[] = {p->G, p->G_R, p->G_A, p->U_wall[0], p->U_wall[1], p->F_ext[0], p->F_ext[1]};
    for (double v : vals)
        if (!isfinite(v)) return fail(LBM_EINVAL, "non-finite model parameter");
    if (p->wall_kind == LBM_WALL_FLAT_SLAB) {
        if (p->slab_rows < 1 || p->slab_rows >= p->ny)
            return fail(LBM_EINVAL, "slab_rows must be in [1, ny) (got %d)", p->slab_rows);
        if (!(p->wall_width > 0) || !(p->core_range > 0) || !(p->tail_range > 0))
            return fail(LBM_EINVAL, "wall_width, core_range, tail_range must be > 0");
    }
    if (p->storage == LBM_STORE_F16DEV && !(p->rho_ref > 0) ) return fail(LBM_EINVAL, "rho_ref must be > 0");
    if (p->seg_rows < 0) return fail(LBM_EINVAL, "seg_rows must be >= 0");
    if (p->diag_interval < 0) return fail(LBM_EINVAL, "diag_interval must be >= 0");
    if (p->reserved != 0) return fail(LBM_EINVAL, "reserved must be 0");
    return LBM_OK;
}

// 3x3 solve by Gaussian elimination with partial pivoting; false if singular.
bool solve3(double A[3][3], double b[3], double z[3]) {
    double big = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) big = fmax(big, fabs(A[i][j]));
    if (!(big > 0)) return false;
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (!(fabs(A[p][c]) > 1e-14 * big)) return false;
        for (int j = 0; j < 3; ++j) { double t = A[c][j]; A[c][j] = A[p][j]; A[p][j] = t; }
        { double t = b[c]; b[c] = b[p]; b[p] = t; }
        for (int r = c + 1; r < 3; ++r) {
            const double m = A[r][c] / A[c][c];
            for (int j = c; j < 3; ++j) A[r][j] -= m * A[c][j];
            b[r] -= m * b[c];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double acc = b[r];
        for (int j = r + 1; j < 3; ++j) acc -= A[r][j] * z[j];
        z[r] = acc / A[r][r];
    }
    return true;
}

}  // namespace

struct lbm_ctx {
    std::string err;               // last error message of a call on this context
    int device;                    // HIP device current at lbm_create
    lbm_params p;
    Layout lay;
    hipStream_t stream;
    char *ws;
    LatDevAny L;
    int wall_mode;                 // 0 = per-row tables, 1 = per-node
    int own_cur;
    int64_t own_step;
    int *cur;                      // which buffer holds the state (0: fa, 1: fb)
    int64_t *step;
    int shape;                     // step tile shape (index into kShapeWaves/kShapeRows)
    int pass2;                     // two-steps-per-pass variant, -1: single steps
    bool view;                     // lives inside a batch (lbm_step/lbm_set_state refused)
    bool attached;                 // an lbm_ctx of the caller grouped by lbm_batch_attach
    // diagnostics bookkeeping
    bool have_prev;                // a snapshot exists for the residual
    int64_t last_diag_step;
    bool last_diag_compared;
    double *d_small;               // [0..7] diag totals, [8..15] moment totals,
                                   // [16..25] isoline sums, [32..35] ranges (u32)
    uint32_t *d_ranges;
};

struct lbm_batch {
    std::vector<lbm_ctx *> lat;
    bool owned;                    // contexts created (and freed) by the batch
    hipStream_t stream;
    int cur;
    int64_t step;
    void *d_lats;
    uint4 *d_work;                 // per-wave (lattice, strip, segment): diagnostics
    uint32_t nwork;
    uint4 *d_twork;                // per-tile (lattice, strip, tile row), grouped by tile shape
    uint32_t ntiles;               // capacity of d_twork (largest tile count of every lattice)
    std::vector<int> shapes;       // tile shape of each lattice
    uint32_t toff[kNumTileShapes + 1];   // d_twork[toff[s], toff[s+1]): tiles of shape s
    int pass2;                     // two-steps-per-pass variant, -1: single steps
    uint32_t poff, pcnt;           // d_twork[poff, poff + pcnt): blocks of that variant
    std::vector<uint4> h_twork;    // host image of d_twork (kept until the next upload)
    double *d_part;
    uint32_t *d_ranges;
    double *d_res;
    hipGraphExec_t graph[2];
    int graph_chunk[2];
};

namespace {

// Routes the error messages of one entry point into its context as well
// (nested entry points restore the outer context's slot on return).
struct CtxScope {
    std::string *prev;
    explicit CtxScope(const lbm_ctx *c) : prev(g_ctx_err) { g_ctx_err = c ? &const_cast<lbm_ctx *>(c)->err : nullptr; }
    ~CtxScope() { g_ctx_err = prev; }
};

lbm_status launch_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(LBM_EDEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
    return LBM_OK;
}

// Runs the diagnostic kernel over the current state and reduces it into
// d_small[slot*8 .. +6].
// partials: where the per-wave partial sums go (nullptr: the workspace's).
lbm_status run_diag(lbm_ctx *c, int write_mom, int compare, int update, int slot, double *partials = nullptr) {
    LatDevAny L = c->L;
    if (partials) L.partials = partials;
    if (c->p.lattice == LBM_D2Q21)
        TRY(launch_ok(launch_diag_q21(kernel_storage(c->p.storage), L, c->wall_mode, *c->cur, write_mom, compare,
                                      update, c->stream),
                      "diag_q21"));
    else
        TRY(launch_ok(launch_diag(kernel_storage(c->p.storage), nullptr, nullptr, 0, L, c->wall_mode, *c->cur,
                                  write_mom, compare, update, c->stream),
                      "diag"));
    TRY(launch_ok(launch_reduce(L.partials, c->d_ranges, 1, 8, 6, c->d_small + 8 * slot, 8, c->stream),
                  "reduce"));
    return LBM_OK;
}

lbm_status sync(lbm_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Builds a context inside `ws` (layout already checked).  Synchronises.
lbm_status init_ctx(lbm_ctx *c, const lbm_params *p, const double *rho0, const double *u0,
                    const double *wall_fields, char *ws, hipStream_t stream) {
    c->p = *p;
    HIPCHK(hipGetDevice(&c->device));
    c->lay = make_layout(*p);
    c->stream = stream;
    c->ws = ws;
    c->own_cur = 0;
    c->own_step = 0;
    c->cur = &c->own_cur;
    c->step = &c->own_step;
    c->shape = 0;
    c->pass2 = -1;
    c->view = false;
    c->attached = false;
    c->have_prev = false;
    c->last_diag_step = -1;
    c->last_diag_compared = false;
    c->wall_mode = (p->wall_kind == LBM_WALL_FIELDS || p->wall_kind == LBM_WALL_MASK) ? 1 : 0;
    const Layout &Y = c->lay;
    const size_t N = size_t(p->nx) * p->ny;
    c->d_small = (double *)(ws + Y.small);
    c->d_ranges = (uint32_t *)(c->d_small + 32);

    LatDevAny &L = c->L;
    L.nx = p->nx; L.ny = p->ny; L.plane = uint32_t(N); L.pstride = Y.pstride;
    L.strips = Y.strips; L.segs = Y.segs; L.seg_rows = Y.seg_rows; L.wave0 = 0;
    L.fa = ws + Y.fa; L.fb = ws + Y.fb;
    L.row_tab = ws + Y.row_tab;
    L.node_tab = c->wall_mode ? (const void *)(ws + Y.node_tab) : nullptr;
    L.mom = ws + Y.mom;
    L.uprev = ws + Y.uprev;
    L.partials = (double *)(ws + Y.partials);
    L.G = p->G; L.omega = 1.0 / p->tau;
    L.Ux = p->U_wall[0]; L.Uy = p->U_wall[1];
    L.Fx = p->F_ext[0]; L.Fy = p->F_ext[1];
    L.rho_ref = p->storage == LBM_STORE_F16DEV ? p->rho_ref : 1.0;
    L.lattice = pop_count(*p);
    L.psi_kind = p->psi_kind;
    L.collision = p->collision;
    // D2Q21: marching step where it applies and the lattice fills the chip
    // with marching workgroups, else one-row tiles (measured on MI355X: never
    // slower than two-row tiles except binary32 at tau != 1 on lattices that
    // march; faster on lattices of few tiles, and in binary64, where the
    // two-row tile at tau != 1 spills registers)
    if (p->lattice == LBM_D2Q21)
        c->shape = (q21_march_ok(kernel_storage(p->storage), L.omega) &&
                    q21_march_blocks(uint32_t(p->nx), uint32_t(p->ny)) >= kQ21FillBlocks) ? 1 : 2;
    {
        // eq. EOS with branch slopes s_b theta (s_b = eos[0..2]), pressure
        // continuous at rho_1 = eos[3] and rho_2 = eos[4].  The pseudo-potential
        // 2 (rho theta - p) / theta is linear on each branch; it is evaluated as
        // k_b (rho - rho_b) + a_b so that a branch of slope theta (the paper's
        // liquid) gives exactly the same psi at every density.
        const double sV = p->eos[0], sU = p->eos[1], sL = p->eos[2], r1 = p->eos[3], r2 = p->eos[4];
        L.eos_kV = 2.0 * (1.0 - sV);
        L.eos_kU = 2.0 * (1.0 - sU);
        L.eos_kL = 2.0 * (1.0 - sL);
        L.eos_aU = 2.0 * r1 * (1.0 - sV);
        L.eos_aL = L.eos_aU + 2.0 * (r2 - r1) * (1.0 - sU);
        L.eos_r1 = r1;
        L.eos_r2 = r2;
    }

    const uint32_t ranges[4] = {0, Y.waves, 0, Y.iso_blocks};
    HIPCHK(hipMemcpyAsync(c->d_ranges, ranges, sizeof ranges, hipMemcpyHostToDevice, stream));

    const int f64 = compute_is_f64(p->storage);
    double *stage = (double *)(ws + Y.fb);   // >= 3N doubles (fb + mom)
    double *phi_raw = (double *)(ws + Y.phi_raw);
    if (c->wall_mode == 0) {
        const int P = p->wall_kind == LBM_WALL_FLAT_SLAB ? p->slab_rows : 0;
        TRY(launch_ok(launch_walls_row(f64, L.lattice, p->ny, P, p->wall_width, p->core_range, p->tail_range, p->eps,
                                       p->G_R, p->G_A, ws + Y.row_tab, phi_raw, stream),
                      "walls_row"));
    } else {
        if (p->wall_kind == LBM_WALL_MASK) {
            // solid indicator into the first field slot, held nodes into
            // population buffer A (free until the initial state is written)
            double *bnd = (double *)(ws + Y.fa);
            HIPCHK(hipMemcpyAsync(stage, wall_fields, N * sizeof(double), hipMemcpyHostToDevice, stream));
            HIPCHK(hipMemcpyAsync(bnd, wall_fields + N, N * sizeof(double), hipMemcpyHostToDevice, stream));
            TRY(launch_ok(launch_filter_walls(L.lattice, uint32_t(p->nx), uint32_t(p->ny), stage, bnd, p->filter_core,
                                              p->filter_wall, stream),
                          "filter_walls"));
        } else {
            HIPCHK(hipMemcpyAsync(stage, wall_fields, 3 * N * sizeof(double), hipMemcpyHostToDevice, stream));
        }
        TRY(launch_ok(launch_walls_node(f64, L.lattice, p->nx, p->ny, stage, p->eps, p->G_R, p->G_A, ws + Y.node_tab,
                                        phi_raw, stream),
                      "walls_node"));
    }
    HIPCHK(hipStreamSynchronize(stream));   // staging is reused below
    HIPCHK(hipMemcpyAsync(stage, rho0, N * sizeof(double), hipMemcpyHostToDevice, stream));
    const double *dux = nullptr, *duy = nullptr;
    if (u0) {
        HIPCHK(hipMemcpyAsync(stage + N, u0, 2 * N * sizeof(double), hipMemcpyHostToDevice, stream));
        dux = stage + N;
        duy = stage + 2 * N;
    }
    TRY(launch_ok(launch_init(kernel_storage(p->storage), L.lattice, p->nx, p->ny, L.pstride, stage, dux, duy, L.fa, L.rho_ref, stream),
                  "init"));
    HIPCHK(hipStreamSynchronize(stream));
    return LBM_OK;
}

lbm_status check_host_fields(const lbm_params *p, const double *rho0, const double *u0,
                             const double *wall_fields) {
    const size_t N = size_t(p->nx) * p->ny;
    if (!rho0) return fail(LBM_EINVAL, "rho0 is NULL");
    for (size_t i = 0; i < N; ++i)
        if (!(rho0[i] > 0) || !isfinite(rho0[i])) return fail(LBM_EINVAL, "rho0[%zu] must be finite and > 0", i);
    if (u0)
        for (size_t i = 0; i < 2 * N; ++i)
            if (!isfinite(u0[i])) return fail(LBM_EINVAL, "non-finite u0 at %zu", i);
    if (p->wall_kind == LBM_WALL_FIELDS) {
        if (!wall_fields) return fail(LBM_EINVAL, "wall_fields required for LBM_WALL_FIELDS");
        for (size_t i = 0; i < 3 * N; ++i)
            if (!isfinite(wall_fields[i])) return fail(LBM_EINVAL, "non-finite wall field at %zu", i);
        for (size_t i = 0; i < N; ++i)
            if (wall_fields[i] < 0 || wall_fields[i] > 1) return fail(LBM_EINVAL, "phi must be in [0,1]");
    } else if (p->wall_kind == LBM_WALL_MASK) {
        if (!wall_fields) return fail(LBM_EINVAL, "wall_fields (solid, boundary indicators) required for LBM_WALL_MASK");
        for (size_t i = 0; i < 2 * N; ++i)
            if (wall_fields[i] != 0.0 && wall_fields[i] != 1.0)
                return fail(LBM_EINVAL, "mask indicator at %zu must be 0 or 1", i);
    } else if (wall_fields) {
        return fail(LBM_EINVAL, "wall_fields must be NULL unless wall_kind is LBM_WALL_FIELDS or LBM_WALL_MASK");
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_params_default(lbm_params *p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    memset(p, 0, sizeof *p);
    p->storage = LBM_STORE_F32;
    p->wall_kind = LBM_WALL_NONE;
    p->tau = 1.0;
    p->G = -5.0;
    p->eps = 1.0;
    p->wall_width = 2.0;
    p->core_range = 1.0;
    p->tail_range = 3.0;
    p->rho_ref = 1.0;
    p->slab_rows = 8;
    p->lattice = LBM_D2Q9;
    p->psi_kind = LBM_PSI_EXP;
    p->collision = LBM_COLL_BGK;
    p->filter_core = 5;
    p->filter_wall = 22;
    const double eos[5] = {0.25, -0.25, 1.0, 0.222, 0.869};
    for (int i = 0; i < 5; ++i) p->eos[i] = eos[i];
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

lbm_status lbm_device_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(LBM_EINVAL, "NULL pointer");
    if (uintptr_t(src) % 16 || uintptr_t(dst) % 16 || bytes % 16)
        return fail(LBM_EINVAL, "src, dst and bytes must be multiples of 16");
    const uintptr_t s = uintptr_t(src), d = uintptr_t(dst);
    if (bytes && s < d + bytes && d < s + bytes) return fail(LBM_EINVAL, "src and dst overlap");
    HIPCHK(launch_copy16(src, dst, bytes, (hipStream_t)stream));
    return LBM_OK;
}

lbm_status lbm_workspace_bytes(const lbm_params *p, size_t *bytes) {
    TRY(validate(p));
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = make_layout(*p).total;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_params *p, const double *rho0, const double *u0, const double *wall_fields,
                      void *workspace, size_t workspace_bytes, void *stream, lbm_ctx **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(validate(p));
    TRY(check_host_fields(p, rho0, u0, wall_fields));
    const Layout Y = make_layout(*p);
    if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if (uintptr_t(workspace) % kAlign) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < Y.total)
        return fail(LBM_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, Y.total);
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ENOMEM, "host allocation failed");
    lbm_status st = init_ctx(c, p, rho0, u0, wall_fields, (char *)workspace, (hipStream_t)stream);
    if (st != LBM_OK) {
        delete c;
        return st;
    }
    *out = c;
    return LBM_OK;
}

// A diagnostic pass after the step just taken (every K-th step index).
static lbm_status diag_after_step(lbm_ctx *c, double *partials = nullptr) {
    TRY(run_diag(c, 0, c->have_prev ? 1 : 0, 1, 0, partials));
    c->last_diag_compared = c->have_prev;
    c->have_prev = true;
    c->last_diag_step = *c->step;
    return LBM_OK;
}

// Reads the last diagnostic pass (synchronising) into out[6] as
// lbm_diagnostics reports it; LBM_EUNSTABLE when it counted non-finite nodes.
static lbm_status read_diag(lbm_ctx *c, double out[6]) {
    double r[8];
    HIPCHK(hipMemcpyAsync(r, c->d_small, sizeof r, hipMemcpyDeviceToHost, c->stream));
    TRY(sync(c));
    out[0] = double(c->last_diag_step);
    out[1] = r[0];
    out[2] = r[1];
    out[3] = r[2];
    if (!c->last_diag_compared) out[4] = INFINITY;
    else out[4] = r[4] > 0 ? r[3] / r[4] : (r[3] > 0 ? INFINITY : 0.0);
    out[5] = r[5];
    if (r[5] > 0) return fail(LBM_EUNSTABLE, "%.0f nodes with non-finite density or velocity at step %lld", r[5],
                              (long long)c->last_diag_step);
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t nsteps, double *residual_out) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    CtxScope scope(c);
    if (c->view) return fail(LBM_ESTATE, "lbm_step on a batch lattice view; use lbm_batch_step");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    const int ks = kernel_storage(c->p.storage);
    const int K = c->p.diag_interval;
    double d[6];
    bool checked = false;
    for (int64_t s = 0; s < nsteps;) {
        // two steps in one pass unless a diagnostic falls after the first
        const bool pair = c->pass2 >= 0 && nsteps - s >= 2 && !(K > 0 && (*c->step + 1) % K == 0);
        if (c->p.lattice == LBM_D2Q21)
            TRY(launch_ok(launch_step_q21(ks, c->L, c->wall_mode, *c->cur, c->shape, c->stream), "step_q21"));
        else if (pair)
            TRY(launch_ok(launch_step_pass2(ks, c->L, c->wall_mode, c->pass2, *c->cur, c->stream), "step_pass2"));
        else
            TRY(launch_ok(launch_step(ks, c->L, c->wall_mode, c->shape, *c->cur, c->stream), "step"));
        *c->cur ^= 1;
        *c->step += pair ? 2 : 1;
        s += pair ? 2 : 1;
        if (K > 0 && *c->step % K == 0) {
            TRY(diag_after_step(c));
            if (residual_out) {
                TRY(read_diag(c, d));          // stops at the first pass with non-finite values
                *residual_out = d[4];
                checked = true;
            }
        }
    }
    if (residual_out && !checked) {
        if (K == 0 && c->last_diag_step != *c->step) TRY(diag_after_step(c));
        if (c->last_diag_step < 0) {
            *residual_out = INFINITY;          // K > 0 and no pass yet
        } else {
            TRY(read_diag(c, d));
            *residual_out = d[4];
        }
    }
    return LBM_OK;
}

lbm_status lbm_diagnostics(lbm_ctx *c, double out[6]) {
    if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    if (c->last_diag_step != *c->step) TRY(diag_after_step(c));
    return read_diag(c, out);
}

}  // extern "C"

// ------------------------------------------ diagnostics without workspace scratch
// The per-wave partial sums of lbm_diagnostics_noalloc live in this array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel: it is a host-side stand-in, not a device address;
// the device address on each GPU comes from hipGetSymbolAddress (scratch_on).
static __device__ __align__(256) double scratch[size_t(LBM_NOALLOC_MAX_ROWS) * 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, nullptr until resolved

// Device address of `scratch` on device dev, resolved once per device with
// that device current.
lbm_status scratch_on(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(LBM_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e2));
        if (!p) return fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

extern "C" {

lbm_status lbm_diagnostics_noalloc(lbm_ctx *c, double out[6]) {
    if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    if (c->lay.waves > uint32_t(LBM_NOALLOC_MAX_ROWS))
        return fail(LBM_EINVAL, "lattice needs %u partial rows; lbm_diagnostics_noalloc holds at most %d",
                    c->lay.waves, LBM_NOALLOC_MAX_ROWS);
    if (c->last_diag_step != *c->step) {
        double *part = nullptr;
        TRY(scratch_on(c->device, &part));
        TRY(diag_after_step(c, part));
    }
    return read_diag(c, out);
}

lbm_status lbm_moments(lbm_ctx *c, double *rho, double *ux, double *uy, double totals[3]) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    CtxScope scope(c);
    TRY(run_diag(c, 1, 0, 0, 1));
    const size_t N = size_t(c->p.nx) * c->p.ny;
    const int f64 = compute_is_f64(c->p.storage);
    double *outs[3] = {rho, ux, uy};
    std::vector<float> tmp(f64 ? 0 : N);
    for (int k = 0; k < 3; ++k) {
        if (!outs[k]) continue;
        if (f64) {
            HIPCHK(hipMemcpyAsync(outs[k], (double *)c->L.mom + k * N, N * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
            TRY(sync(c));
        } else {
            HIPCHK(hipMemcpyAsync(tmp.data(), (float *)c->L.mom + k * N, N * sizeof(float), hipMemcpyDeviceToHost,
                                  c->stream));
            TRY(sync(c));
            for (size_t i = 0; i < N; ++i) outs[k][i] = double(tmp[i]);
        }
    }
    double r[8];
    HIPCHK(hipMemcpyAsync(r, c->d_small + 8, sizeof r, hipMemcpyDeviceToHost, c->stream));
    TRY(sync(c));
    if (totals) {
        totals[0] = r[0];
        totals[1] = r[1];
        totals[2] = r[2];
    }
    return LBM_OK;
}

}  // extern "C"

namespace {

// One isoline pass; returns the 10 reduced sums.
lbm_status iso_pass(lbm_ctx *c, IsoParams ip, double sums[10]) {
    const int f64 = compute_is_f64(c->p.storage);
    double *part = (double *)(c->ws + c->lay.iso_part);
    TRY(launch_ok(launch_isoline(f64, ip, c->L.mom, (const double *)(c->ws + c->lay.phi_raw), part, c->stream),
                  "isoline"));
    TRY(launch_ok(launch_reduce(part, c->d_ranges + 2, 1, 10, 10, c->d_small + 16, 10, c->stream), "reduce"));
    HIPCHK(hipMemcpyAsync(sums, c->d_small + 16, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

// Least-squares circle through the region-III crossings selected by ip
// (side, unwrap): algebraic (Kasa) fit about the centroid, then up to 20
// Gauss-Newton steps of the geometric fit (Sec. III.B).
lbm_status fit_circle(lbm_ctx *c, IsoParams ip, double min_points, double &xc_out, double &yc_out, double &R_out) {
    double s[10];
    ip.mode = 0;
    TRY(iso_pass(c, ip, s));
    const double n = s[0];
    if (n < min_points) return fail(LBM_ENOFIT, "only %.0f isoline points in region III", n);
    ip.mx = s[1] / n;
    ip.my = s[2] / n;
    // algebraic fit about the centroid: x^2 + y^2 + D x + E y + F = 0
    ip.mode = 1;
    TRY(iso_pass(c, ip, s));
    double A[3][3] = {{s[3], s[4], s[1]}, {s[4], s[5], s[2]}, {s[1], s[2], s[0]}};
    double b[3] = {-s[6], -s[7], -s[8]}, z[3];
    if (!solve3(A, b, z)) return fail(LBM_ENOFIT, "degenerate algebraic circle fit");
    double xc = -0.5 * z[0], yc = -0.5 * z[1], R2 = xc * xc + yc * yc - z[2];
    if (!(R2 > 0)) return fail(LBM_ENOFIT, "degenerate algebraic circle fit");
    double R = sqrt(R2);
    // geometric refinement
    ip.mode = 2;
    for (int it = 0; it < 20; ++it) {
        ip.xc = xc; ip.yc = yc; ip.R = R;
        TRY(iso_pass(c, ip, s));
        double J[3][3] = {{s[1], s[2], s[3]}, {s[2], s[4], s[5]}, {s[3], s[5], s[6]}};
        double g[3] = {s[7], s[8], s[9]}, d[3];
        if (!solve3(J, g, d)) return fail(LBM_ENOFIT, "degenerate geometric circle fit");
        xc += d[0]; yc += d[1]; R += d[2];
        if (fabs(d[0]) + fabs(d[1]) + fabs(d[2]) < 1e-13 * (1.0 + fabs(R))) break;
    }
    if (!(R > 0) || !isfinite(R) || !isfinite(xc) || !isfinite(yc)) return fail(LBM_ENOFIT, "circle fit diverged");
    xc_out = xc + ip.mx;
    yc_out = yc + ip.my;
    R_out = R;
    return LBM_OK;
}

// theta = acos((y_ref - yc) / R), clamped, in degrees (Sec. III.B: h = yc + R - y_ref).
double contact_angle_deg(double xc, double yc, double R, double y_ref) {
    (void)xc;
    double cs = (y_ref - yc) / R;
    cs = cs > 1 ? 1 : (cs < -1 ? -1 : cs);
    return acos(cs) * (180.0 / M_PI);
}

}  // namespace

extern "C" {

lbm_status lbm_contact_angle(lbm_ctx *c, double iso, double y_ref, double out[4]) {
    if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    if (!isfinite(iso) || !isfinite(y_ref)) return fail(LBM_EINVAL, "iso and y_ref must be finite");
    TRY(run_diag(c, 1, 0, 0, 1));
    IsoParams ip{uint32_t(c->p.nx), uint32_t(c->p.ny), c->wall_mode, 0, iso, 0.01, 0, 0, 0, 0, 0};
    double xc, yc, R;
    TRY(fit_circle(c, ip, 16, xc, yc, R));
    out[0] = contact_angle_deg(xc, yc, R, y_ref);
    out[1] = R;
    out[2] = xc;
    out[3] = yc;
    return LBM_OK;
}

lbm_status lbm_dynamic_angles(lbm_ctx *c, double iso, double y_ref, double out[8]) {
    if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    if (!isfinite(iso) || !isfinite(y_ref)) return fail(LBM_EINVAL, "iso and y_ref must be finite");
    TRY(run_diag(c, 1, 0, 0, 1));
    const uint32_t nx = uint32_t(c->p.nx), ny = uint32_t(c->p.ny);
    IsoParams ip{nx, ny, c->wall_mode, 5, iso, 0.01, 0, 0, 0, 0, 0};
    double s[10];
    // the drop's position along the periodic x: circular mean of its crossings
    TRY(iso_pass(c, ip, s));
    if (s[0] < 16) return fail(LBM_ENOFIT, "only %.0f isoline points in region III", s[0]);
    if (!(fabs(s[1]) + fabs(s[2]) > 1e-9 * s[0]))
        return fail(LBM_ENOFIT, "isoline points spread evenly over the periodic x range");
    double xmid = atan2(s[1], s[2]) * (double(nx) / (2.0 * M_PI));
    if (xmid < 0) xmid += double(nx);
    ip.unwrap = 1;
    ip.xmid = xmid;
    // apex: the highest crossing
    ip.mode = 3;
    const int f64 = compute_is_f64(c->p.storage);
    double *part = (double *)(c->ws + c->lay.iso_part);
    TRY(launch_ok(launch_isoline(f64, ip, c->L.mom, (const double *)(c->ws + c->lay.phi_raw), part, c->stream),
                  "isoline top"));
    std::vector<double> top(size_t(c->lay.iso_blocks) * 10);
    HIPCHK(hipMemcpyAsync(top.data(), part, top.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    TRY(sync(c));
    bool found = false;
    double ax = 0, ay = -1;
    for (uint32_t b = 0; b < c->lay.iso_blocks; ++b) {
        const double f = top[10 * b], x = top[10 * b + 1], y = top[10 * b + 2];
        if (f != 0.0 && (!found || y > ay || (y == ay && x < ax))) {
            found = true;
            ax = x;
            ay = y;
        }
    }
    if (!found) return fail(LBM_ENOFIT, "no isoline points");
    // rear (x <= apex) and front (x >= apex) circles, each through the apex
    double cx[2], cy[2], cr[2];
    for (int k = 0; k < 2; ++k) {
        IsoParams sp = ip;
        sp.side = k == 0 ? -1 : 1;
        sp.xs = ax;
        TRY(fit_circle(c, sp, 8, cx[k], cy[k], cr[k]));
    }
    // mean velocity and density of the liquid in region III
    ip.mode = 4;
    ip.unwrap = 0;
    TRY(iso_pass(c, ip, s));
    if (!(s[1] > 0)) return fail(LBM_ENOFIT, "no liquid nodes in region III");
    const double U = s[2] / s[1];
    const int adv = U >= 0 ? 1 : 0;          // the side the drop moves towards
    out[0] = contact_angle_deg(cx[adv], cy[adv], cr[adv], y_ref);
    out[1] = contact_angle_deg(cx[1 - adv], cy[1 - adv], cr[1 - adv], y_ref);
    out[2] = U;
    out[3] = cr[adv];
    out[4] = cr[1 - adv];
    out[5] = ax - double(nx) * floor(ax / double(nx));
    out[6] = ay;
    out[7] = s[1] / s[0];
    return LBM_OK;
}

lbm_status lbm_slip_length(lbm_ctx *c, double out[3]) {
    if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    if (c->p.wall_kind != LBM_WALL_FLAT_SLAB) return fail(LBM_EINVAL, "slip length needs wall_kind FLAT_SLAB");
    TRY(run_diag(c, 1, 0, 0, 1));
    const int nx = c->p.nx, ny = c->p.ny, P = c->p.slab_rows;
    const int f64 = compute_is_f64(c->p.storage);
    const size_t N = size_t(nx) * ny;
    const void *ux = (const char *)c->L.mom + N * compute_bytes(c->p.storage);
    double *prof = (double *)(c->ws + c->lay.profile);
    TRY(launch_ok(launch_profile(f64, nx, ny, ux, prof, c->stream), "profile"));
    std::vector<double> rows(ny), phi(ny);
    HIPCHK(hipMemcpyAsync(rows.data(), prof, ny * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(phi.data(), c->ws + c->lay.phi_raw, ny * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    TRY(sync(c));
    const int top = ny - P;
    const double mid = 0.5 * top;
    double A[3][3] = {{0}}, b[3] = {0}, z[3];
    int used = 0;
    for (int y = 0; y <= top; ++y) {
        if (!(phi[y] < 0.01)) continue;       // region III only
        const double t = y - mid, u = rows[y] / nx;
        const double v[3] = {1.0, t, t * t};
        for (int i = 0; i < 3; ++i) {
            b[i] += v[i] * u;
            for (int j = 0; j < 3; ++j) A[i][j] += v[i] * v[j];
        }
        ++used;
    }
    if (used < 3 || !solve3(A, b, z)) return fail(LBM_ENOFIT, "not enough region-III rows for the slip fit");
    const double yw = c->p.wall_width * atanh(0.98);   // phi(y_w) = 0.01
    const double tb = yw - mid, tt = (top - yw) - mid;
    const double ub = z[0] + z[1] * tb + z[2] * tb * tb, ut = z[0] + z[1] * tt + z[2] * tt * tt;
    const double gb = fabs(z[1] + 2 * z[2] * tb), gt = fabs(z[1] + 2 * z[2] * tt);
    const double us = 0.5 * (ub + ut), g = 0.5 * (gb + gt);
    out[0] = g > 0 ? us / g : INFINITY;
    out[1] = us;
    out[2] = 2 * z[2];
    return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx *c, double *f) {
    if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    const size_t N = size_t(c->p.nx) * c->p.ny;
    void *pop = *c->cur ? c->L.fb : c->L.fa;
    double *stage = (double *)(*c->cur ? c->L.fa : c->L.fb);   // the other buffer is free between steps
    for (int q = 0; q < pop_count(c->p); ++q) {
        TRY(launch_ok(launch_plane(kernel_storage(c->p.storage), c->L.lattice, 0, c->p.nx, c->p.ny, c->L.pstride, q, pop, stage, c->L.rho_ref,
                                   c->stream),
                      "get_plane"));
        HIPCHK(hipMemcpyAsync(f + q * N, stage, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        TRY(sync(c));
    }
    return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx *c, const double *f, int64_t step_index) {
    if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
    CtxScope scope(c);
    if (c->view) return fail(LBM_ESTATE, "lbm_set_state on a batch lattice view");
    if (step_index < 0) return fail(LBM_EINVAL, "step_index must be >= 0");
    const size_t N = size_t(c->p.nx) * c->p.ny;
    void *pop = *c->cur ? c->L.fb : c->L.fa;
    double *stage = (double *)(*c->cur ? c->L.fa : c->L.fb);
    for (int q = 0; q < pop_count(c->p); ++q) {
        HIPCHK(hipMemcpyAsync(stage, f + q * N, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
        TRY(launch_ok(launch_plane(kernel_storage(c->p.storage), c->L.lattice, 1, c->p.nx, c->p.ny, c->L.pstride, q, pop, stage, c->L.rho_ref,
                                   c->stream),
                      "set_plane"));
        TRY(sync(c));
    }
    *c->step = step_index;
    c->have_prev = false;
    c->last_diag_step = -1;
    c->last_diag_compared = false;
    return LBM_OK;
}

int64_t lbm_step_index(const lbm_ctx *c) { return c ? *c->step : -1; }

lbm_status lbm_destroy(lbm_ctx *c) {
    CtxScope scope(c);
    if (c && c->attached) return fail(LBM_ESTATE, "context is attached to a batch; destroy the batch first");
    if (!c || c->view) return LBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    g_ctx_err = nullptr;                 // the context's slot goes with it
    delete c;
    if (e != hipSuccess) return fail(LBM_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return LBM_OK;
}

// ------------------------------------------------------------------ batches
static lbm_status batch_check(const lbm_params *ps, int32_t n) {
    if (!ps || n < 1) return fail(LBM_EINVAL, "need n >= 1 lattices");
    for (int32_t k = 0; k < n; ++k) {
        TRY(validate(&ps[k]));
        if (ps[k].storage != LBM_STORE_F32) return fail(LBM_EINVAL, "lattice %d: batches take F32 storage only", k);
        if (ps[k].lattice != LBM_D2Q9 || ps[k].psi_kind != LBM_PSI_EXP)
            return fail(LBM_EINVAL, "lattice %d: batches take D2Q9 with the exponential pseudo-potential", k);
        if (ps[k].wall_kind == LBM_WALL_FIELDS || ps[k].wall_kind == LBM_WALL_MASK)
            return fail(LBM_EINVAL, "lattice %d: batches take wall kinds NONE or FLAT_SLAB", k);
    }
    return LBM_OK;
}

// Device tables of a batch: lattice descriptors, the wave work list, the
// per-wave partial sums and per-lattice reduction ranges and results.
struct TablesLayout {
    size_t lats, work, twork, part, ranges, res, total;
};

static TablesLayout tables_layout(size_t base, int32_t n, uint32_t nwork, uint32_t ntiles) {
    TablesLayout T;
    size_t o = base;
    T.lats = o; o = align_up(o + size_t(n) * sizeof(LatDev<float>));
    T.work = o; o = align_up(o + size_t(nwork) * sizeof(uint4));
    T.twork = o; o = align_up(o + size_t(ntiles) * sizeof(uint4));
    T.part = o; o = align_up(o + size_t(nwork) * 8 * sizeof(double));
    T.ranges = o; o = align_up(o + size_t(n) * 2 * sizeof(uint32_t));
    T.res = o; o = align_up(o + size_t(n) * 8 * sizeof(double));
    T.total = o;
    return T;
}

struct BatchLayout {
    std::vector<size_t> off;
    size_t lats, work, part, ranges, res, total;
    uint32_t nwork, ntiles;
};

static BatchLayout batch_layout(const lbm_params *ps, int32_t n, int32_t seg_rows) {
    BatchLayout B;
    size_t o = 0;
    B.nwork = 0;
    B.ntiles = 0;
    for (int32_t k = 0; k < n; ++k) {
        lbm_params p = ps[k];
        p.seg_rows = seg_rows;
        Layout L = make_layout(p);
        B.off.push_back(o);
        o = align_up(o + L.total);
        B.nwork += L.waves;
        B.ntiles += L.tiles;
    }
    const TablesLayout T = tables_layout(o, n, B.nwork, B.ntiles);
    B.lats = T.lats;
    B.work = T.work;
    B.part = T.part;
    B.ranges = T.ranges;
    B.res = T.res;
    B.total = T.total;
    return B;
}

lbm_status lbm_batch_workspace_bytes(const lbm_params *ps, int32_t n, size_t *bytes) {
    TRY(batch_check(ps, n));
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = batch_layout(ps, n, ps[0].seg_rows).total;
    return LBM_OK;
}

static lbm_batch *new_batch(char *ws, const TablesLayout &T, uint32_t nwork, uint32_t ntiles, hipStream_t st,
                            bool owned) {
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return nullptr;
    b->owned = owned;
    b->stream = st;
    b->cur = 0;
    b->step = 0;
    b->graph[0] = b->graph[1] = nullptr;
    b->graph_chunk[0] = b->graph_chunk[1] = 0;
    b->nwork = nwork;
    b->ntiles = ntiles;
    for (int s = 0; s <= kNumTileShapes; ++s) b->toff[s] = 0;
    b->pass2 = -1;
    b->poff = b->pcnt = 0;
    b->d_lats = ws + T.lats;
    b->d_work = (uint4 *)(ws + T.work);
    b->d_twork = (uint4 *)(ws + T.twork);
    b->d_part = (double *)(ws + T.part);
    b->d_ranges = (uint32_t *)(ws + T.ranges);
    b->d_res = (double *)(ws + T.res);
    return b;
}

static void drop_graphs(lbm_batch *b) {
    for (int i = 0; i < 2; ++i) {
        if (b->graph[i]) (void)hipGraphExecDestroy(b->graph[i]);
        b->graph[i] = nullptr;
        b->graph_chunk[i] = 0;
    }
}

// Builds the step-tile list from b->shapes, grouped by shape (one launch per
// non-empty group), and uploads it.  Recorded graphs are dropped.  Synchronises.
static lbm_status upload_twork(lbm_batch *b) {
    const int32_t n = int32_t(b->lat.size());
    std::vector<uint4> &tw = b->h_twork;
    HIPCHK(hipStreamSynchronize(b->stream));     // the previous image may still be in flight
    tw.clear();
    for (int s = 0; s < kNumTileShapes; ++s) {
        b->toff[s] = uint32_t(tw.size());
        for (int32_t k = 0; k < n; ++k) {
            if (b->shapes[k] != s) continue;
            const lbm_ctx *c = b->lat[k];
            const uint32_t trows = tile_rows(uint32_t(c->p.ny), s), groups = tile_groups(uint32_t(c->p.nx), s);
            for (uint32_t tr = 0; tr < trows; ++tr)
                for (uint32_t gp = 0; gp < groups; ++gp) tw.push_back(make_uint4(uint32_t(k), gp, tr, 0));
        }
    }
    b->toff[kNumTileShapes] = uint32_t(tw.size());
    b->poff = uint32_t(tw.size());
    if (b->pass2 >= 0) {
        const int v = b->pass2;
        for (int32_t k = 0; k < n; ++k) {
            const lbm_ctx *c = b->lat[k];
            const uint32_t bands = (uint32_t(c->p.ny) + uint32_t(kPass2Rows[v]) - 1) / uint32_t(kPass2Rows[v]);
            const uint32_t groups = pass2_blocks(uint32_t(c->p.nx), uint32_t(c->p.ny), v) / bands;
            for (uint32_t tr = 0; tr < bands; ++tr)
                for (uint32_t gp = 0; gp < groups; ++gp) tw.push_back(make_uint4(uint32_t(k), gp, tr, 0));
        }
    }
    b->pcnt = uint32_t(tw.size()) - b->poff;
    if (tw.size() > b->ntiles) return fail(LBM_EINVAL, "internal: tile list exceeds its capacity");
    HIPCHK(hipMemcpyAsync(b->d_twork, tw.data(), tw.size() * sizeof(uint4), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    return LBM_OK;
}

// One time step of every lattice of the batch: one launch per tile shape in use.
static hipError_t batch_launch(lbm_batch *b, int parity) {
    for (int s = 0; s < kNumTileShapes; ++s) {
        const uint32_t cnt = b->toff[s + 1] - b->toff[s];
        if (!cnt) continue;
        hipError_t e = launch_step_batch(b->d_lats, b->d_twork + b->toff[s], cnt, s, parity, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Builds descriptors and the work list over b->lat (whose current buffer is
// fa, i.e. batch parity 0) and uploads them.  Synchronises.
static lbm_status upload_tables(lbm_batch *b) {
    const int32_t n = int32_t(b->lat.size());
    std::vector<LatDev<float>> lats(n);
    std::vector<uint4> work;
    std::vector<uint32_t> ranges(2 * size_t(n));
    work.reserve(b->nwork);
    b->shapes.resize(size_t(n));
    for (int32_t k = 0; k < n; ++k) b->shapes[k] = b->lat[k]->shape;
    uint32_t w0 = 0;
    for (int32_t k = 0; k < n; ++k) {
        lbm_ctx *c = b->lat[k];
        c->cur = &b->cur;
        const Layout &Y = c->lay;
        LatDevAny La = c->L;
        La.wave0 = w0;
        La.partials = b->d_part + 8 * size_t(w0);
        lats[k] = La.get<float>();
        for (uint32_t sg = 0; sg < Y.segs; ++sg)
            for (uint32_t sp = 0; sp < Y.strips; ++sp) work.push_back(make_uint4(uint32_t(k), sp, sg, 0));
        ranges[2 * k] = w0;
        ranges[2 * k + 1] = w0 + Y.waves;
        w0 += Y.waves;
    }
    if (w0 != b->nwork) return fail(LBM_EINVAL, "internal: work list size mismatch");
    HIPCHK(hipMemcpyAsync(b->d_lats, lats.data(), lats.size() * sizeof(LatDev<float>), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipMemcpyAsync(b->d_work, work.data(), work.size() * sizeof(uint4), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_ranges, ranges.data(), ranges.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return upload_twork(b);
}

lbm_status lbm_batch_create(const lbm_params *ps, int32_t n, const double *const *rho0s,
                            const double *const *u0s, int32_t seg_rows,
                            void *workspace, size_t workspace_bytes, void *stream, lbm_batch **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(batch_check(ps, n));
    if (!rho0s) return fail(LBM_EINVAL, "rho0s is NULL");
    if (seg_rows < 0) return fail(LBM_EINVAL, "seg_rows must be >= 0");
    if (!workspace || uintptr_t(workspace) % kAlign) return fail(LBM_EINVAL, "workspace NULL or not 256-byte aligned");
    BatchLayout B = batch_layout(ps, n, seg_rows);
    if (workspace_bytes < B.total) return fail(LBM_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, B.total);
    char *ws = (char *)workspace;
    hipStream_t st = (hipStream_t)stream;
    TablesLayout T = tables_layout(B.lats, n, B.nwork, B.ntiles);
    lbm_batch *b = new_batch(ws, T, B.nwork, B.ntiles, st, true);
    if (!b) return fail(LBM_ENOMEM, "host allocation failed");
    lbm_status stt = LBM_OK;
    for (int32_t k = 0; k < n && stt == LBM_OK; ++k) {
        lbm_params p = ps[k];
        p.seg_rows = seg_rows;
        stt = check_host_fields(&p, rho0s[k], u0s ? u0s[k] : nullptr, nullptr);
        if (stt != LBM_OK) break;
        lbm_ctx *c = new (std::nothrow) lbm_ctx();
        if (!c) { stt = fail(LBM_ENOMEM, "host allocation failed"); break; }
        stt = init_ctx(c, &p, rho0s[k], u0s ? u0s[k] : nullptr, nullptr, ws + B.off[k], st);
        if (stt != LBM_OK) { delete c; break; }
        c->view = true;
        b->lat.push_back(c);
    }
    if (stt == LBM_OK) stt = upload_tables(b);
    if (stt != LBM_OK) {
        for (lbm_ctx *c : b->lat) delete c;
        delete b;
        return stt;
    }
    *out = b;
    return LBM_OK;
}

static lbm_status attach_check(lbm_ctx *const *ctxs, int32_t n, uint32_t *nwork, uint32_t *ntiles) {
    if (!ctxs || n < 1) return fail(LBM_EINVAL, "need n >= 1 contexts");
    uint32_t w = 0, t = 0;
    for (int32_t k = 0; k < n; ++k) {
        const lbm_ctx *c = ctxs[k];
        if (!c) return fail(LBM_EINVAL, "context %d is NULL", k);
        if (c->view || c->attached) return fail(LBM_ESTATE, "context %d already belongs to a batch", k);
        if (c->p.storage != LBM_STORE_F32 || c->wall_mode != 0 || c->p.lattice != LBM_D2Q9 ||
            c->p.psi_kind != LBM_PSI_EXP)
            return fail(LBM_EINVAL, "context %d: batches take D2Q9, F32 storage and wall kinds NONE or FLAT_SLAB", k);
        for (int32_t j = 0; j < k; ++j)
            if (ctxs[j] == c) return fail(LBM_EINVAL, "context %d listed twice", k);
        w += c->lay.waves;
        t += c->lay.tiles;
    }
    *nwork = w;
    *ntiles = t;
    return LBM_OK;
}

lbm_status lbm_batch_attach_bytes(lbm_ctx *const *ctxs, int32_t n, size_t *bytes) {
    uint32_t nwork = 0, ntiles = 0;
    TRY(attach_check(ctxs, n, &nwork, &ntiles));
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = tables_layout(0, n, nwork, ntiles).total;
    return LBM_OK;
}

lbm_status lbm_batch_attach(lbm_ctx *const *ctxs, int32_t n, void *workspace, size_t workspace_bytes, void *stream,
                            lbm_batch **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    uint32_t nwork = 0, ntiles = 0;
    TRY(attach_check(ctxs, n, &nwork, &ntiles));
    hipStream_t st = (hipStream_t)stream;
    for (int32_t k = 0; k < n; ++k)
        if (ctxs[k]->stream != st) return fail(LBM_EINVAL, "context %d uses another stream than the batch", k);
    if (!workspace || uintptr_t(workspace) % kAlign) return fail(LBM_EINVAL, "workspace NULL or not 256-byte aligned");
    TablesLayout T = tables_layout(0, n, nwork, ntiles);
    if (workspace_bytes < T.total) return fail(LBM_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, T.total);
    lbm_batch *b = new_batch((char *)workspace, T, nwork, ntiles, st, false);
    if (!b) return fail(LBM_ENOMEM, "host allocation failed");
    for (int32_t k = 0; k < n; ++k) {
        lbm_ctx *c = ctxs[k];
        // make every context's current state its buffer fa: batch parity 0
        if (*c->cur) {
            void *t = c->L.fa;
            c->L.fa = c->L.fb;
            c->L.fb = t;
            c->own_cur = 0;
        }
        c->attached = true;
        c->view = true;
        b->lat.push_back(c);
    }
    lbm_status stt = upload_tables(b);
    if (stt != LBM_OK) {
        for (lbm_ctx *c : b->lat) {
            c->cur = &c->own_cur;
            c->attached = false;
            c->view = false;
        }
        delete b;
        return stt;
    }
    *out = b;
    return LBM_OK;
}

static void batch_advance(lbm_batch *b, int64_t n) {
    b->step += n;
    for (lbm_ctx *c : b->lat) *c->step += n;
}

// Two time steps of every lattice of the batch: one launch of the batch's
// two-step variant.
static hipError_t batch_launch_pass2(lbm_batch *b, int parity) {
    return launch_step_pass2_batch(b->d_lats, b->d_twork + b->poff, b->pcnt, b->pass2, parity, b->stream);
}

static lbm_status batch_plain(lbm_batch *b, int64_t n) {
    while (b->pass2 >= 0 && n >= 2) {
        TRY(launch_ok(batch_launch_pass2(b, b->cur), "step_pass2_batch"));
        b->cur ^= 1;
        batch_advance(b, 2);
        n -= 2;
    }
    for (int64_t s = 0; s < n; ++s) {
        TRY(launch_ok(batch_launch(b, b->cur), "step_batch"));
        b->cur ^= 1;
        batch_advance(b, 1);
    }
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps, int32_t chunk) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (nsteps < 0 || chunk < 0 || (chunk % 2)) return fail(LBM_EINVAL, "nsteps >= 0 and an even chunk >= 0 required");
    if (chunk == 0) return batch_plain(b, nsteps);
    if (b->stream == nullptr) return fail(LBM_EINVAL, "graph replay (chunk > 0) needs a non-default stream");
    while (nsteps >= chunk) {
        const int par = b->cur;
        if (b->graph[par] && b->graph_chunk[par] != chunk) {
            (void)hipGraphExecDestroy(b->graph[par]);
            b->graph[par] = nullptr;
        }
        if (!b->graph[par]) {
            hipGraph_t g;
            HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            if (b->pass2 >= 0) {
                for (int s = 0; s < chunk / 2 && e == hipSuccess; ++s) e = batch_launch_pass2(b, par ^ (s & 1));
            } else {
                for (int s = 0; s < chunk && e == hipSuccess; ++s) e = batch_launch(b, par ^ (s & 1));
            }
            hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess) return fail(LBM_EDEVICE, "capture launch: %s", hipGetErrorString(e));
            if (e2 != hipSuccess) return fail(LBM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
            hipError_t e3 = hipGraphInstantiate(&b->graph[par], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) return fail(LBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e3));
            b->graph_chunk[par] = chunk;
        }
        HIPCHK(hipGraphLaunch(b->graph[par], b->stream));
        // chunk is even: one-step launches leave the parity unchanged, chunk / 2
        // two-step launches flip it when chunk / 2 is odd
        if (b->pass2 >= 0) b->cur ^= (chunk / 2) & 1;
        batch_advance(b, chunk);
        nsteps -= chunk;
    }
    return batch_plain(b, nsteps);
}

lbm_status lbm_batch_diagnostics(lbm_batch *b, double *out) {
    if (!b || !out) return fail(LBM_EINVAL, "NULL argument");
    const int n = int(b->lat.size());
    LatDevAny dummy;
    // every lattice is compared with its own snapshot; a lattice without one
    // (new, or just after lbm_set_state) reports +inf and gets one now
    TRY(launch_ok(launch_diag(STORE_F32, b->d_lats, b->d_work, b->nwork, dummy, 0, b->cur, 0, 1, 1, b->stream),
                  "diag_batch"));
    TRY(launch_ok(launch_reduce(b->d_part, b->d_ranges, n, 8, 6, b->d_res, 8, b->stream), "reduce"));
    std::vector<double> r(8 * size_t(n));
    HIPCHK(hipMemcpyAsync(r.data(), b->d_res, r.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    bool bad = false;
    for (int k = 0; k < n; ++k) {
        lbm_ctx *c = b->lat[k];
        const double *v = &r[8 * size_t(k)];
        double *o = out + 6 * size_t(k);
        o[0] = double(*c->step);
        o[1] = v[0]; o[2] = v[1]; o[3] = v[2];
        o[4] = !c->have_prev ? INFINITY : (v[4] > 0 ? v[3] / v[4] : (v[3] > 0 ? INFINITY : 0.0));
        o[5] = v[5];
        bad = bad || v[5] > 0;
        c->have_prev = true;
        c->last_diag_step = -1;
    }
    if (bad) return fail(LBM_EUNSTABLE, "non-finite values in at least one lattice");
    return LBM_OK;
}

lbm_ctx *lbm_batch_lattice(lbm_batch *b, int32_t k) {
    if (!b || k < 0 || k >= int32_t(b->lat.size())) {
        fail(LBM_EINVAL, "no lattice %d in batch", k);
        return nullptr;
    }
    return b->lat[k];
}

// ------------------------------------------------------- tile shapes, tuner
int32_t lbm_tile_shapes(int32_t *waves, int32_t *rows, int32_t *strips, int32_t cap) {
    for (int s = 0; s < kNumTileShapes && s < cap; ++s) {
        if (waves) waves[s] = kShapeWaves[s];
        if (rows) rows[s] = kShapeRows[s];
        if (strips) strips[s] = kShapeStrips[s];
    }
    return kNumTileShapes;
}

lbm_status lbm_set_tile_shape(lbm_ctx *c, int32_t shape) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    CtxScope scope(c);
    if (c->view) return fail(LBM_ESTATE, "lattice belongs to a batch; use lbm_batch_set_tile_shapes");
    if (c->p.lattice == LBM_D2Q21) {
        if (shape < 0 || shape >= kQ21Variants) return fail(LBM_EINVAL, "D2Q21 step variant %d out of range", shape);
        if (shape == 1 && !q21_march_ok(kernel_storage(c->p.storage), c->L.omega))
            return fail(LBM_EINVAL, "the marching D2Q21 step needs F32 storage");
        c->shape = shape;
        return LBM_OK;
    }
    if (shape < 0 || shape >= kNumTileShapes) return fail(LBM_EINVAL, "tile shape %d out of range", shape);
    c->shape = shape;
    return LBM_OK;
}

int32_t lbm_get_tile_shape(const lbm_ctx *c) { return c ? c->shape : -1; }

int32_t lbm_two_step_variants(int32_t *strips, int32_t *rows, int32_t *waves, int32_t cap) {
    for (int v = 0; v < kPass2Variants && v < cap; ++v) {
        if (strips) strips[v] = kPass2Strips[v];
        if (rows) rows[v] = kPass2Rows[v];
        if (waves) waves[v] = kPass2Strips[v] * kPass2WavesPerStrip[v];
    }
    return kPass2Variants;
}

lbm_status lbm_set_two_step(lbm_ctx *c, int32_t variant) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    CtxScope scope(c);
    if (c->view) return fail(LBM_ESTATE, "lattice belongs to a batch");
    if (variant < -1 || variant >= kPass2Variants) return fail(LBM_EINVAL, "two-step variant %d out of range", variant);
    if (variant >= 0 && (c->p.lattice != LBM_D2Q9 || !pass2_ok(kernel_storage(c->p.storage))))
        return fail(LBM_EINVAL, "two steps per pass need a D2Q9 lattice with F32, F16DEV or F64 storage");
    c->pass2 = variant;
    return LBM_OK;
}

int32_t lbm_get_two_step(const lbm_ctx *c) { return c ? c->pass2 : -2; }

}  // extern "C"

namespace {

// Per-step time (ms): the median over kTuneReps blocks of `steps` consecutive
// steps issued by `one`, each block bracketed by events and waited for.  Steps
// run back to back as in production (a wait after every single step would
// time each step from an idle GPU and favour other shapes).
constexpr int kTuneReps = 3;
template <class Fn> lbm_status time_steps(hipStream_t st, int32_t steps, Fn &&one, double *median_ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LBM_EDEVICE, "hipEventCreate: %s", hipGetErrorString(he));
    }
    std::vector<double> t;
    lbm_status stt = LBM_OK;
    for (int rep = 0; rep < kTuneReps && stt == LBM_OK; ++rep) {
        he = hipEventRecord(e0, st);
        for (int32_t i = 0; i < steps && stt == LBM_OK && he == hipSuccess; ++i) stt = one();
        if (stt == LBM_OK && he == hipSuccess) he = hipEventRecord(e1, st);
        if (stt == LBM_OK && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0;
        if (stt == LBM_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess && stt == LBM_OK) stt = fail(LBM_EDEVICE, "timing events: %s", hipGetErrorString(he));
        t.push_back(ms / steps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stt != LBM_OK) return stt;
    std::sort(t.begin(), t.end());
    *median_ms = t[t.size() / 2];
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_tune(lbm_ctx *c, int32_t steps, int32_t *shape_out, double *ms_out) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    CtxScope scope(c);
    if (c->view) return fail(LBM_ESTATE, "lattice belongs to a batch; use lbm_batch_tune");
    if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
    int best = c->shape;
    double best_ms = INFINITY;
    const bool q21 = c->p.lattice == LBM_D2Q21;
    const int count = q21 ? kQ21Variants : kNumTileShapes;
    for (int s = 0; s < count; ++s) {
        if (q21 && s == 1 && !q21_march_ok(kernel_storage(c->p.storage), c->L.omega)) {
            if (ms_out) ms_out[s] = INFINITY;   // marching step does not apply
            continue;
        }
        c->shape = s;
        TRY(lbm_step(c, 1, nullptr));             // first launch of this shape: not timed
        double ms = 0;
        TRY(time_steps(c->stream, steps, [&]() { return lbm_step(c, 1, nullptr); }, &ms));
        if (ms_out) ms_out[s] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = s;
        }
    }
    c->shape = best;
    if (shape_out) *shape_out = best;
    return LBM_OK;
}

lbm_status lbm_tune_two_step(lbm_ctx *c, int32_t steps, int32_t *variant_out, double *ms_out) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    CtxScope scope(c);
    if (c->view) return fail(LBM_ESTATE, "lattice belongs to a batch");
    if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
    const bool ok = c->p.lattice == LBM_D2Q9 && pass2_ok(kernel_storage(c->p.storage));
    int best = -1;
    double best_ms = INFINITY;
    // candidate -1 (single steps with the context's tile shape), then every variant
    for (int v = -1; v < kPass2Variants; ++v) {
        double *slot = ms_out ? (v < 0 ? ms_out + kPass2Variants : ms_out + v) : nullptr;
        if (v >= 0 && !ok) {
            if (slot) *slot = INFINITY;
            continue;
        }
        c->pass2 = v;
        TRY(lbm_step(c, 2, nullptr));             // first pass of this candidate: not timed
        double ms = 0;
        TRY(time_steps(c->stream, steps, [&]() { return lbm_step(c, 2, nullptr); }, &ms));
        ms *= 0.5;                                // per time step
        if (slot) *slot = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    c->pass2 = best;
    if (variant_out) *variant_out = best;
    return LBM_OK;
}

lbm_status lbm_batch_set_tile_shapes(lbm_batch *b, const int32_t *shapes) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    const size_t n = b->lat.size();
    for (size_t k = 0; k < n; ++k) {
        const int s = shapes ? shapes[k] : 0;
        if (s < 0 || s >= kNumTileShapes) return fail(LBM_EINVAL, "lattice %zu: tile shape %d out of range", k, s);
    }
    for (size_t k = 0; k < n; ++k) {
        b->shapes[k] = shapes ? shapes[k] : 0;
        b->lat[k]->shape = b->shapes[k];
    }
    return upload_twork(b);
}

lbm_status lbm_batch_get_tile_shapes(const lbm_batch *b, int32_t *shapes) {
    if (!b || !shapes) return fail(LBM_EINVAL, "NULL argument");
    for (size_t k = 0; k < b->lat.size(); ++k) shapes[k] = b->shapes[k];
    return LBM_OK;
}

// Autotuner.  Times every shape on the whole batch (median of `steps` single
// steps), derives a per-tile cost for each shape, gives every lattice the shape
// with the smallest predicted cost (tiles x per-tile cost; small lattices
// favour shapes that waste fewer rows at their edge), times that mixed
// assignment too, and keeps the fastest of all candidates.  The tuning steps
// are ordinary time steps of the batch.
lbm_status lbm_batch_tune(lbm_batch *b, int32_t steps, int32_t *shapes_out, double *ms_out) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
    const size_t n = b->lat.size();
    auto one = [&]() -> lbm_status {
        TRY(launch_ok(batch_launch(b, b->cur), "step_batch"));
        b->cur ^= 1;
        batch_advance(b, 1);
        return LBM_OK;
    };
    std::vector<int32_t> cand(n);
    double uni[kNumTileShapes], tile_cost[kNumTileShapes];
    int best = 0;
    for (int s = 0; s < kNumTileShapes; ++s) {
        std::fill(cand.begin(), cand.end(), s);
        TRY(lbm_batch_set_tile_shapes(b, cand.data()));
        TRY(one());
        TRY(time_steps(b->stream, steps, one, &uni[s]));
        tile_cost[s] = uni[s] / double(b->toff[kNumTileShapes]);
        if (ms_out) ms_out[s] = uni[s];
        if (uni[s] < uni[best]) best = s;
    }
    std::vector<int32_t> mix(n);
    bool uniform = true;
    for (size_t k = 0; k < n; ++k) {
        const lbm_ctx *c = b->lat[k];
        int bs = 0;
        double bc = INFINITY;
        for (int s = 0; s < kNumTileShapes; ++s) {
            const double cost = double(step_tiles(uint32_t(c->p.nx), uint32_t(c->p.ny), s)) * tile_cost[s];
            if (cost < bc) {
                bc = cost;
                bs = s;
            }
        }
        mix[k] = bs;
        uniform = uniform && bs == mix[0];
    }
    double mix_ms = NAN;
    if (!uniform) {
        TRY(lbm_batch_set_tile_shapes(b, mix.data()));
        TRY(one());
        TRY(time_steps(b->stream, steps, one, &mix_ms));
    }
    if (ms_out) ms_out[kNumTileShapes] = mix_ms;
    if (!(mix_ms < uni[best])) {
        std::fill(cand.begin(), cand.end(), best);
        TRY(lbm_batch_set_tile_shapes(b, cand.data()));
    }
    if (shapes_out) TRY(lbm_batch_get_tile_shapes(b, shapes_out));
    return LBM_OK;
}

lbm_status lbm_batch_set_two_step(lbm_batch *b, int32_t variant) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (variant < -1 || variant >= kPass2Variants) return fail(LBM_EINVAL, "two-step variant %d out of range", variant);
    b->pass2 = variant;
    return upload_twork(b);
}

int32_t lbm_batch_get_two_step(const lbm_batch *b) { return b ? b->pass2 : -2; }

lbm_status lbm_batch_tune_two_step(lbm_batch *b, int32_t steps, int32_t *variant_out, double *ms_out) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
    int best = -1;
    double best_ms = INFINITY;
    for (int v = -1; v < kPass2Variants; ++v) {
        TRY(lbm_batch_set_two_step(b, v));
        TRY(batch_plain(b, 2));                   // first launch of this candidate: not timed
        double ms = 0;
        TRY(time_steps(b->stream, steps, [&]() { return batch_plain(b, 2); }, &ms));
        ms *= 0.5;                                // per time step
        if (ms_out) ms_out[v < 0 ? kPass2Variants : v] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    TRY(lbm_batch_set_two_step(b, best));
    if (variant_out) *variant_out = best;
    return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch *b) {
    if (!b) return LBM_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (lbm_ctx *c : b->lat) {
        if (b->owned) {
            delete c;
        } else {
            // hand the context back with its state, step index and parity
            c->own_cur = b->cur;
            c->cur = &c->own_cur;
            c->attached = false;
            c->view = false;
        }
    }
    delete b;
    if (e != hipSuccess) return fail(LBM_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return LBM_OK;
}

}  // extern "C"
