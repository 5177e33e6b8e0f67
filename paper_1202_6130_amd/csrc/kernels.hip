// HIP kernels (gfx950) of the wetting-model lattice-Boltzmann library and the
// host launchers the C ABI calls.  See lbm.h for the update they implement.
//
// Hot kernel, k_step_tiles: one workgroup owns a 64-column strip (lane l holds
// column x0 + l) and a band of rows; every wave loads its rows at once (pull
// streaming: nine coalesced row reads shifted by -c_i, plus one gathered load
// for the two columns beside the strip), publishes density and
// pseudo-potential in LDS, and after one barrier forms the forces, collides
// and writes nine aligned rows.  Population planes are SoA [9][ny][nx] with a
// padded plane stride.  The marching walk (march) serves the diagnostic pass.
//
// Two steps per launch, k_step_pass2 (and k_step_pass2_batch): a workgroup
// reads its block grown by four nodes once, computes the first step on the
// block grown by two with the populations kept in LDS, and writes the second
// step of the block: half the memory traffic per update, bitwise the same
// fields as two launches of k_step_tiles.
#include <type_traits>

#include <utility>

#include "launch.hpp"
#include "lbm_device.hpp"

namespace lbmwet {

// ---------------------------------------------------------------- marching
// Walks one (strip, segment) tile and hands every row's node data to `act`.
//
// Lane l owns column x0 + l (x0 = 64 * strip, wrapped mod nx), so every
// population row is read and written as whole 64-lane rows.  The
// pseudo-potential of the two columns just outside the strip comes from a
// tenth, gathered load per row (lanes 0..8 and 32..40 fetch the nine
// populations of those two nodes) summed within 16-lane rows.
//
// Software pipeline: the loads of row y+1+D are issued before row y+1 is
// consumed (D = LBM_PF_DEPTH).  Raw and decoded row buffers rotate through
// the unrolled iterations instead of being copied: a copy of a register whose
// load is in flight would wait for that load.
template <class S, class C, int WALL, class Act>
__device__ inline void march(const LatDev<C> &L, const void *src, uint32_t strip, uint32_t seg, Act &act) {
    using Raw = typename Codec<S>::Raw;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nx = L.nx, ny = L.ny;
    const uint32_t x0 = strip * kStripCols;
    const uint32_t x = wrap_fast(x0 + uint32_t(lane), nx);
    const bool active = x0 + uint32_t(lane) < nx;

    RowLoader<S> ld;
    ld.buf.init(src, 9u * L.pstride * uint32_t(sizeof(S)));
    ld.plane = L.pstride;
    ld.x = x;
    ld.xm = wrap_dec(x, nx);
    ld.xp = wrap_inc(x, nx);
    // halo gather lanes: slot k = lane (left) or lane - 32 (right) fetches
    // population gather_pop(k)
    const bool g_left = lane < Q, g_right = lane >= 32 && lane < 32 + Q;
    const bool g_on = g_left || g_right;
    const int g_q = gather_pop(g_left ? lane : (g_right ? lane - 32 : 8));
    {
        const uint32_t h = g_left ? wrap_fast(x0 + nx - 1, nx) : wrap_fast(x0 + kStripCols, nx);
        const uint32_t hc = wrap_fast(uint32_t(int(h) + int(nx) - cx_dyn(g_q)), nx);   // h - c_x, wrapped
        ld.g_col = g_on ? uint32_t(g_q) * L.pstride + hc : 0u;
        ld.g_cy = g_on ? cy_dyn(g_q) : 0;
    }
    const uint32_t y0 = seg * L.seg_rows;
    const uint32_t y1 = min(y0 + L.seg_rows, ny);

    // loads of row r (its pulled populations come from rows r-1, r, r+1)
    auto load_row = [&](uint32_t r, Raw(&dst)[Q], Raw &g) {
        ld.load(wrap_dec(r, ny) * nx, r * nx, wrap_inc(r, ny) * nx, dst, g);
    };
    // psi of the two halo nodes of a row, from its gathered populations
    // (summed in the tree of density(): equal to the owner's density)
    auto halo_psi = [&](Raw g, C &pl, C &pr) {
        const C v = g_on ? Codec<S>::template decode<C>(g, g_q, L.rho_ref) : C(0);
        const C s = row_sum9<C>(v);
        pl = psi_of<C>(Lanes<C>::lane(s, 15));
        pr = psi_of<C>(Lanes<C>::lane(s, 47));
    };

    C fA[Q], fB[Q];
    Raw rA[Q], rB[Q], gA, gB;
#if LBM_PF_DEPTH >= 2
    Raw rC[Q], gC;
#endif
    // prologue: psi of row y0-1, populations of row y0, prefetches
    load_row(wrap_dec(y0, ny), rA, gA);
    load_row(y0, rB, gB);
    decode_row<S, C>(rA, fB, L.rho_ref);
    C psi_m = psi_of<C>(density<C>(fB));
    C hl_m, hr_m, hl_c, hr_c;
    halo_psi(gA, hl_m, hr_m);
    decode_row<S, C>(rB, fA, L.rho_ref);
    C rho_c = density<C>(fA);
    C psi_c = psi_of<C>(rho_c);
    halo_psi(gB, hl_c, hr_c);
    RowWall<C> wall_c = row_wall<C, WALL>(L, y0);
    load_row(wrap_inc(y0, ny), rA, gA);                           // row y0+1 (always <= y1)
#if LBM_PF_DEPTH >= 2
    if (y0 + 2 <= y1) load_row(wrap_inc(wrap_inc(y0, ny), ny), rB, gB);   // row y0+2
#endif

    // Row y: raw row y+1 in `cur`, optionally prefetch row y+1+D into `nxt`;
    // decoded row y in `fc`, row y+1 is decoded into `fn`.
    auto row = [&](uint32_t y, bool prefetch, Raw(&cur)[Q], Raw &gcur, Raw(&nxt)[Q], Raw &gnxt, C(&fc)[Q],
                   C(&fn)[Q]) {
        const uint32_t yn = wrap_inc(y, ny);
        if (prefetch) {
            uint32_t yp = wrap_inc(yn, ny);
#if LBM_PF_DEPTH >= 2
            yp = wrap_inc(yp, ny);
#endif
            load_row(yp, nxt, gnxt);
        }
        const RowWall<C> wall_n = row_wall<C, WALL>(L, yn);      // scalar loads, one row ahead
        decode_row<S, C>(cur, fn, L.rho_ref);
        const C rho_n = density<C>(fn);
        const C psi_p = psi_of<C>(rho_n);
        C hl_p, hr_p;
        halo_psi(gcur, hl_p, hr_p);
        // sum_i w_i psi(x + c_i) c_i from the neighbours across lanes
        C sx, sy;
        psi_sums<C>(psi_p, psi_m, Lanes<C>::left(psi_c, hl_c), Lanes<C>::left(psi_p, hl_p),
                    Lanes<C>::left(psi_m, hl_m), Lanes<C>::right(psi_c, hr_c), Lanes<C>::right(psi_p, hr_p),
                    Lanes<C>::right(psi_m, hr_m), sx, sy);
        act.row(L, wall_c, y, x, active, fc, rho_c, psi_c, sx, sy);
        psi_m = psi_c;
        psi_c = psi_p;
        rho_c = rho_n;
        hl_m = hl_c;
        hl_c = hl_p;
        hr_m = hr_c;
        hr_c = hr_p;
        wall_c = wall_n;
    };

    uint32_t y = y0;
#if LBM_PF_DEPTH >= 2
    // rA = row y0+1, rB = row y0+2 (if any); ring rA -> rB -> rC.  A row
    // prefetches when row y+3 <= y1.  Decoded rows alternate, with a copy.
    auto row3 = [&](uint32_t yy, Raw(&cur)[Q], Raw &gc, Raw(&nxt)[Q], Raw &gn) {
        row(yy, yy + 3 <= y1, cur, gc, nxt, gn, fA, fB);
#pragma unroll
        for (int i = 0; i < Q; ++i) fA[i] = fB[i];
    };
    for (; y + 5 <= y1; y += 3) {
        row(y, true, rA, gA, rC, gC, fA, fB);
        row(y + 1, true, rB, gB, rA, gA, fB, fA);
        row(y + 2, true, rC, gC, rB, gB, fA, fB);
#pragma unroll
        for (int i = 0; i < Q; ++i) fA[i] = fB[i];
    }
    if (y < y1) row3(y, rA, gA, rC, gC);
    if (y + 1 < y1) row3(y + 1, rB, gB, rA, gA);
    if (y + 2 < y1) row3(y + 2, rC, gC, rB, gB);
    if (y + 3 < y1) row3(y + 3, rA, gA, rC, gC);
    if (y + 4 < y1) row3(y + 4, rB, gB, rA, gA);
#else
    // rA = row y0+1.  Rows come in pairs (rA -> rB, then rB -> rA); every
    // row but the last prefetches (the last of all needs nothing more, the
    // one before it loads the halo row y1 below the segment).
    for (; y + 2 < y1; y += 2) {
        row(y, true, rA, gA, rB, gB, fA, fB);
        row(y + 1, true, rB, gB, rA, gA, fB, fA);
    }
    if (y + 1 < y1) {
        row(y, true, rA, gA, rB, gB, fA, fB);
        row(y + 1, false, rB, gB, rA, gA, fB, fA);
    } else {
        row(y, false, rA, gA, rB, gB, fA, fB);
    }
#endif
}

// Collide and store (the time step).
// ONE = 1: the collision compiled for tau = 1 only (see collide).
template <class S, class C, int WALL, int ONE = 0> struct StepAct {
    PopBuf<S> dst;
    __device__ inline void row(const LatDev<C> &L, const RowWall<C> &rw, uint32_t y, uint32_t x, bool active,
                               C f[Q], C rho, C psi_c, C sx, C sy) {
        const uint32_t n = y * L.nx + x;
        C phie, Sx, Sy;
        wall_terms<C, WALL>(L, rw, n, phie, Sx, Sy);
        NodeState<C> s = node_forces<C>(f, rho, psi_c, sx, sy, phie, Sx, Sy, L.G, L.Ux, L.Uy, L.Fx, L.Fy);
        collide<C, ONE>(f, s, L.omega, L.collision);
        if (active) {
            const uint32_t row = y * L.nx;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                dst.store(Codec<S>::template encode<C>(f[i], i, L.rho_ref), x, i * L.pstride + row);
        }
    }
};

// Diagnostics: reported fields, FP64 totals, residual against the snapshot.
template <class S, class C, int WALL> struct DiagAct {
    int write_mom, compare, update;
    double s_rho = 0, s_jx = 0, s_jy = 0, s_du = 0, s_u = 0, s_bad = 0;
    __device__ inline void row(const LatDev<C> &L, const RowWall<C> &rw, uint32_t y, uint32_t x, bool active,
                               C f[Q], C rho, C psi_c, C sx, C sy) {
        const uint32_t n = y * L.nx + x;
        C phie, Sx, Sy;
        wall_terms<C, WALL>(L, rw, n, phie, Sx, Sy);
        NodeState<C> s = node_forces<C>(f, rho, psi_c, sx, sy, phie, Sx, Sy, L.G, L.Ux, L.Uy, L.Fx, L.Fy);
        // reported velocity (j + F/2) / rho; in binary32 arithmetic from the
        // binary64 momenta (the binary32 reciprocal enters once)
        C vx, vy;
        if constexpr (sizeof(C) == 4) {
            vx = C(0.5 * (s.jxd + s.jsxd) * double(s.inv_rho));
            vy = C(0.5 * (s.jyd + s.jsyd) * double(s.inv_rho));
        } else {
            vx = s.ux + C(0.5) * s.Fx * s.inv_rho;
            vy = s.uy + C(0.5) * s.Fy * s.inv_rho;
        }
        // totals: the node's populations summed in binary64 (exact for binary32)
        double d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = double(f[i]);
        const double m = (((d[1] + d[3]) + (d[2] + d[4])) + ((d[5] + d[6]) + (d[7] + d[8]))) + d[0];
        const double mjx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
        const double mjy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
        if (!active) return;
        if (write_mom) {
            L.mom[n] = rho;
            L.mom[L.plane + n] = vx;
            L.mom[2 * L.plane + n] = vy;
        }
        bool ok = isfinite(double(rho)) && isfinite(double(vx)) && isfinite(double(vy));
#pragma unroll
        for (int i = 0; i < Q; ++i) ok = ok && !Codec<S>::template saturated<C>(f[i], i, L.rho_ref);
        s_bad += ok ? 0.0 : 1.0;
        s_rho += m;
        s_jx += mjx;
        s_jy += mjy;
        if (compare) s_du += fabs(double(vx) - double(L.uprev[n])) + fabs(double(vy) - double(L.uprev[L.plane + n]));
        s_u += fabs(double(vx)) + fabs(double(vy));
        if (update) {
            L.uprev[n] = vx;
            L.uprev[L.plane + n] = vy;
        }
    }
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Global wave index of the calling wave, uniform across the wave.
__device__ inline uint32_t logical_wave() {
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    return lb * kBlockWaves + w;
}

// ---------------------------------------------------------------- tiles
// The time step proper.  One workgroup of TW waves owns TS adjacent 64-column
// strips and TW / TS * TR consecutive rows, of which the first and last are
// halo rows: wave w works in strip w / (TW / TS) and loads its rows
// y0 - 1 + (w mod TW / TS) TR + j (j < TR), all at once.  Each wave computes
// density and pseudo-potential of its rows, the outermost waves also of the
// column beside the block (from one gathered load per row), and publishes
// them in LDS; after one barrier every row between the halo rows reads its
// neighbours above, below and across strip boundaries, forms the forces,
// collides and stores.  No wave walks through rows one after another: every
// population row of the tile is in flight at the same time.
template <class C, int ROWS, int COLS> struct TileLds {
    C psi[ROWS][COLS];
    C hal[ROWS][2];
};

template <class S, class C, int WALL, int TW, int TR, int TS, int ONE>
__device__ inline void tile_step(const LatDev<C> &L, const void *src, void *dst, uint32_t group, uint32_t trow,
                                 TileLds<C, TW / TS * TR, TS * kWave> &sm) {
    using Raw = typename Codec<S>::Raw;
    constexpr int R = TR, WS = TW / TS;
    constexpr uint32_t kOut = uint32_t(WS * TR - 2);
    static_assert(TW % TS == 0, "waves must split evenly over the strips");
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    const int sj = w / WS, wr = w - sj * WS;          // strip within the block, wave within the strip
    const uint32_t nx = L.nx, ny = L.ny;
    const uint32_t X0 = group * uint32_t(TS * kStripCols);   // first column of the block
    const uint32_t pos = uint32_t(sj * kStripCols + lane);    // column offset within the block
    const uint32_t x = wrap_fast(X0 + pos, nx);
    const bool active = X0 + pos < nx;
    const uint32_t y0 = trow * kOut;
    const uint32_t out_rows = min(kOut, ny - y0);

    RowLoader<S> ld;
    ld.buf.init(src, 9u * L.pstride * uint32_t(sizeof(S)));
    ld.plane = L.pstride;
    ld.x = x;
    ld.xm = wrap_dec(x, nx);
    ld.xp = wrap_inc(x, nx);
    // gathered halo columns: lanes 0..8 of the waves of the first strip fetch
    // the nine pulled populations of column X0 - 1, lanes 32..40 of the waves
    // of the last strip those of column X0 + 64 TS (both wrapped)
    const bool g_left = lane < Q && sj == 0, g_right = lane >= 32 && lane < 32 + Q && sj == TS - 1;
    const bool g_on = g_left || g_right;
    const int g_q = gather_pop(g_left ? lane : (g_right ? lane - 32 : 8));
    {
        const uint32_t h = g_left ? wrap_fast(X0 + nx - 1, nx) : wrap_fast(X0 + uint32_t(TS * kStripCols), nx);
        const uint32_t hc = wrap_fast(uint32_t(int(h) + int(nx) - cx_dyn(g_q)), nx);   // h - c_x, wrapped
        ld.g_col = g_on ? uint32_t(g_q) * L.pstride + hc : 0u;
        ld.g_cy = g_on ? cy_dyn(g_q) : 0;
    }

    // rows of this wave: tile row index k = wr R + j, lattice row y0 - 1 + k
    C f[R][Q], rho[R], psi[R];
    Raw raw[R][Q], g[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t k = uint32_t(wr * R + j);
        const uint32_t r = wrap_fast(y0 + ny - 1 + k, ny);
        if (k <= out_rows + 1) ld.load(wrap_dec(r, ny) * nx, r * nx, wrap_inc(r, ny) * nx, raw[j], g[j]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t k = uint32_t(wr * R + j);
        rho[j] = C(0);
        psi[j] = C(0);
        if (k <= out_rows + 1) {
            decode_row<S, C>(raw[j], f[j], L.rho_ref);
            rho[j] = density<C>(f[j]);
            psi[j] = psi_of<C>(rho[j]);
            // the halo nodes' density is read out of lanes 15 and 47 by every
            // lane, outside divergent control flow
            const C v = g_on ? Codec<S>::template decode<C>(g[j], g_q, L.rho_ref) : C(0);
            const C sum = row_sum9<C>(v);
            const C hl = psi_of<C>(Lanes<C>::lane(sum, 15));
            const C hr = psi_of<C>(Lanes<C>::lane(sum, 47));
            sm.psi[k][pos] = psi[j];
            if (lane == 0 && sj == 0) sm.hal[k][0] = hl;
            if (lane == 0 && sj == TS - 1) sm.hal[k][1] = hr;
        }
    }
    __syncthreads();
    // pseudo-potential just left of lane 0 / right of lane 63 of this strip
    const int cl = sj * kStripCols - 1, cr = (sj + 1) * kStripCols;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t k = uint32_t(wr * R + j);
        if (k < 1 || k > out_rows) continue;
        const uint32_t r = wrap_fast(y0 - 1 + k, ny);
        const C psi_m = sm.psi[k - 1][pos], psi_p = sm.psi[k + 1][pos];
        C hl_m, hl_c, hl_p, hr_m, hr_c, hr_p;
        if (sj == 0) {
            hl_m = sm.hal[k - 1][0]; hl_c = sm.hal[k][0]; hl_p = sm.hal[k + 1][0];
        } else {
            hl_m = sm.psi[k - 1][cl]; hl_c = sm.psi[k][cl]; hl_p = sm.psi[k + 1][cl];
        }
        if (sj == TS - 1) {
            hr_m = sm.hal[k - 1][1]; hr_c = sm.hal[k][1]; hr_p = sm.hal[k + 1][1];
        } else {
            hr_m = sm.psi[k - 1][cr]; hr_c = sm.psi[k][cr]; hr_p = sm.psi[k + 1][cr];
        }
        // sum_i w_i psi(x + c_i) c_i from the neighbours across lanes (see march)
        C sx, sy;
        psi_sums<C>(psi_p, psi_m, Lanes<C>::left(psi[j], hl_c), Lanes<C>::left(psi_p, hl_p),
                    Lanes<C>::left(psi_m, hl_m), Lanes<C>::right(psi[j], hr_c), Lanes<C>::right(psi_p, hr_p),
                    Lanes<C>::right(psi_m, hr_m), sx, sy);
        StepAct<S, C, WALL, ONE> act;
        act.dst.init(dst, 9u * L.pstride * uint32_t(sizeof(S)));
        act.row(L, row_wall<C, WALL>(L, r), r, x, active, f[j], rho[j], psi[j], sx, sy);
    }
}

// ---------------------------------------------------------------- kernels
template <class S, class C, int WALL, int SHAPE, int ONE>
__global__ __launch_bounds__(kShapeWaves[SHAPE] * kWave) void k_step_tiles(LatDev<C> L, const void *__restrict__ src,
                                                                          void *__restrict__ dst) {
    constexpr int TW = kShapeWaves[SHAPE], TR = kShapeRows[SHAPE], TS = kShapeStrips[SHAPE];
    __shared__ TileLds<C, TW / TS * TR, TS * kWave> sm;
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint32_t groups = (L.strips + TS - 1) / TS;
    const uint32_t trow = lb / groups, group = lb - trow * groups;
    tile_step<S, C, WALL, TW, TR, TS, ONE>(L, src, dst, group, trow, sm);
}

// Batched step over tiles of one shape: twork[b] = (lattice, strip group, tile
// row) of logical workgroup b.
template <class S, class C, int WALL, int SHAPE>
__global__ __launch_bounds__(kShapeWaves[SHAPE] * kWave) void k_step_tiles_batch(const LatDev<C> *__restrict__ lats,
                                                                                const uint4 *__restrict__ twork,
                                                                                int parity) {
    constexpr int TW = kShapeWaves[SHAPE], TR = kShapeRows[SHAPE], TS = kShapeStrips[SHAPE];
    __shared__ TileLds<C, TW / TS * TR, TS * kWave> sm;
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint4 wk = twork[lb];
    const LatDev<C> L = lats[wk.x];
    tile_step<S, C, WALL, TW, TR, TS, 0>(L, parity ? L.fb : L.fa, parity ? L.fa : L.fb, wk.y, wk.z, sm);
}

// ---------------------------------------------------------------- two steps per pass
// Temporal blocking: one workgroup advances an output block of OW = 64 TS
// columns x OH rows by two time steps with one read and one write of the
// populations.  The first step is computed on the block grown by two nodes on
// every side (region R2), which needs the pseudo-potential on the block grown
// by three (R1) and populations pulled from one node further out; its
// populations stay in LDS.  The second step pulls from LDS, forms the
// pseudo-potential on the block grown by one (R3), and writes the block with
// the aligned row stores of k_step_tiles.  Every node of either step goes
// through the device functions of the single step (density, psi, the
// neighbour sums grouped by column, wall terms, node_forces, collide, the
// storage round trip), so a pass equals two single steps bit for bit.
template <int TS, int OH, int WPS> struct Pass2Geo {
    static constexpr int OW = TS * kStripCols;
    static constexpr int NT = TS * WPS * kWave;                    // threads
    static constexpr int W1 = OW + 6, H1 = OH + 6, N1 = W1 * H1;   // psi, step one
    static constexpr int W2 = OW + 4, H2 = OH + 4, N2 = W2 * H2;   // populations after step one
    static constexpr int W3 = OW + 2, H3 = OH + 2, N3 = W3 * H3;   // psi, step two
    static constexpr int K1 = (N1 + NT - 1) / NT, K2 = (N2 + NT - 1) / NT, K3 = (N3 + NT - 1) / NT;
    static constexpr size_t lds_words = size_t(Q) * N2 + N1 + 2 * H2;   // in elements of the arithmetic type
    static constexpr size_t lds_bytes = sizeof(float) * lds_words;
    static_assert(OH % WPS == 0, "output rows must split evenly over the waves of a strip");
};

// One block (column group `group`, row band `trow`) of lattice L; lds holds
// Pass2Geo::lds_bytes of dynamic LDS.
template <class S, class C, int WALL, int TS, int OH, int WPS, int ONE>
__device__ inline void pass2_block(const LatDev<C> &L, const void *src, void *dst, uint32_t group, uint32_t trow,
                                   unsigned char *lds) {
    using G = Pass2Geo<TS, OH, WPS>;
    using Raw = typename Codec<S>::Raw;
    constexpr int NT = G::NT, W1 = G::W1, W2 = G::W2, W3 = G::W3, N2 = G::N2;
    C *sf = reinterpret_cast<C *>(lds);          // [Q][N2] populations of step one
    C *sp = sf + Q * N2;                         // [N1] psi of step one, then [N3] psi of step two
    C *sw = sp + G::N1;                          // [H2][2] row wall terms of step one (WALL_ROW)
    const uint32_t nx = L.nx, ny = L.ny, P = L.pstride;
    const uint32_t X0 = group * uint32_t(G::OW), Y0 = trow * uint32_t(OH);
    // multiples of nx and ny of at least 3, so that X0 - 3 + c never goes negative
    const uint32_t kx = nx >= 3 ? nx : (nx == 2 ? 4u : 3u), ky = ny >= 3 ? ny : (ny == 2 ? 4u : 3u);
    const int tid = int(threadIdx.x);
    const C rref = L.rho_ref;
    // On lattices at least one grown block wide and high every coordinate
    // formed below is < 3 nx (3 ny): two conditional subtractions wrap it.
    const bool big = nx >= uint32_t(W1) && ny >= uint32_t(G::H1);
    auto wrap = [big](uint32_t v, uint32_t n) {
        if (big) {
            v = v >= n ? v - n : v;
            return v >= n ? v - n : v;
        }
        return wrap_fast(v, n);
    };
    if (WALL == WALL_ROW && tid < G::H2) {
        const RowWall<C> rw = row_wall<C, WALL>(L, wrap(Y0 + ky - 2u + uint32_t(tid), ny));
        sw[2 * tid] = rw.phie;
        sw[2 * tid + 1] = rw.Sy;
    }

    // R1: pulled populations, density and psi of step one; populations of R2 to LDS
    {
        PopBuf<S> in;
        in.init(src, 9u * P * uint32_t(sizeof(S)));
        Raw raw[G::K1][Q];
#pragma unroll
        for (int k = 0; k < G::K1; ++k) {
            const int i = tid + k * NT;
            if ((k + 1) * NT <= G::N1 || i < G::N1) {
                const int r = i / W1, c = i - r * W1;
                const uint32_t x = wrap(X0 + kx - 3u + uint32_t(c), nx);
                const uint32_t y = wrap(Y0 + ky - 3u + uint32_t(r), ny);
                const uint32_t xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
                const uint32_t r0 = y * nx, rm = wrap_dec(y, ny) * nx, rp = wrap_inc(y, ny) * nx;
                raw[k][0] = in.load(r0 + x, 0);
                raw[k][1] = in.load(r0 + xm, P);
                raw[k][2] = in.load(rm + x, 2 * P);
                raw[k][3] = in.load(r0 + xp, 3 * P);
                raw[k][4] = in.load(rp + x, 4 * P);
                raw[k][5] = in.load(rm + xm, 5 * P);
                raw[k][6] = in.load(rm + xp, 6 * P);
                raw[k][7] = in.load(rp + xp, 7 * P);
                raw[k][8] = in.load(rp + xm, 8 * P);
            }
        }
#pragma unroll
        for (int k = 0; k < G::K1; ++k) {
            const int i = tid + k * NT;
            if ((k + 1) * NT <= G::N1 || i < G::N1) {
                C f[Q];
                decode_row<S, C>(raw[k], f, rref);
                sp[i] = psi_of<C>(density<C>(f));
                const int r = i / W1, c = i - r * W1;
                if (r >= 1 && r < G::H1 - 1 && c >= 1 && c < W1 - 1) {
                    const int j = (r - 1) * W2 + (c - 1);
#pragma unroll
                    for (int q = 0; q < Q; ++q) sf[q * N2 + j] = f[q];
                }
            }
        }
    }
    __syncthreads();

    // R2: forces and collision of step one, in place in LDS (each node reads only its own populations)
#pragma unroll
    for (int k = 0; k < G::K2; ++k) {
        const int i = tid + k * NT;
        if (!((k + 1) * NT <= N2 || i < N2)) continue;
        const int r2 = i / W2, c2 = i - r2 * W2;
        const C *p = sp + (r2 + 1) * W1 + (c2 + 1);
        C sx, sy;
        psi_sums<C>(p[W1], p[-W1], p[-1], p[W1 - 1], p[-W1 - 1], p[1], p[W1 + 1], p[-W1 + 1], sx, sy);
        C f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sf[q * N2 + i];
        const C rho = density<C>(f);
        C phie, Sx, Sy;
        if (WALL == WALL_ROW) {
            phie = sw[2 * r2];
            Sx = C(0);
            Sy = sw[2 * r2 + 1];
        } else {
            const uint32_t x = wrap(X0 + kx - 2u + uint32_t(c2), nx);
            const uint32_t y = wrap(Y0 + ky - 2u + uint32_t(r2), ny);
            wall_terms<C, WALL>(L, RowWall<C>{C(0), C(0)}, y * nx + x, phie, Sx, Sy);
        }
        NodeState<C> s = node_forces<C>(f, rho, p[0], sx, sy, phie, Sx, Sy, L.G, L.Ux, L.Uy, L.Fx, L.Fy);
        collide<C, ONE>(f, s, L.omega, L.collision);
#pragma unroll
        for (int q = 0; q < Q; ++q)
            sf[q * N2 + i] = Codec<S>::template decode<C>(Codec<S>::template encode<C>(f[q], q, rref), q, rref);
    }
    __syncthreads();

    // R3: pulled populations, density and psi of step two
#pragma unroll
    for (int k = 0; k < G::K3; ++k) {
        const int i = tid + k * NT;
        if (!((k + 1) * NT <= G::N3 || i < G::N3)) continue;
        const int r3 = i / W3, c3 = i - r3 * W3;
        const int j = (r3 + 1) * W2 + (c3 + 1);
        C f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sf[q * N2 + j - kCy[q] * W2 - kCx[q]];
        sp[i] = psi_of<C>(density<C>(f));
    }
    __syncthreads();

    // output block: lane = column, WPS waves per 64-column strip, OH / WPS rows each
    const int lane = tid & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int sj = w / WPS, wr = w - sj * WPS;
    const int c4 = sj * kStripCols + lane;
    const uint32_t gx = X0 + uint32_t(c4);
    const bool active = gx < nx;
    const uint32_t x = wrap_fast(gx, nx);
    StepAct<S, C, WALL, ONE> act;
    act.dst.init(dst, 9u * P * uint32_t(sizeof(S)));
#pragma unroll
    for (int jr = 0; jr < OH / WPS; ++jr) {
        const int r4 = wr * (OH / WPS) + jr;
        const uint32_t y = Y0 + uint32_t(r4);
        if (y >= ny) break;
        const int j = (r4 + 2) * W2 + (c4 + 2);
        C f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = sf[q * N2 + j - kCy[q] * W2 - kCx[q]];
        const C rho = density<C>(f);
        const C *p = sp + (r4 + 1) * W3 + (c4 + 1);
        C sx, sy;
        psi_sums<C>(p[W3], p[-W3], p[-1], p[W3 - 1], p[-W3 - 1], p[1], p[W3 + 1], p[-W3 + 1], sx, sy);
        act.row(L, row_wall<C, WALL>(L, y), y, x, active, f, rho, p[0], sx, sy);
    }
}

template <class S, class C, int WALL, int TS, int OH, int WPS, int ONE>
__global__ __launch_bounds__(TS * WPS * kWave) void k_step_pass2(LatDev<C> L, const void *__restrict__ src,
                                                                 void *__restrict__ dst) {
    extern __shared__ __align__(16) unsigned char pass2_lds[];
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint32_t groups = (L.nx + uint32_t(TS * kStripCols) - 1) / uint32_t(TS * kStripCols);
    const uint32_t trow = lb / groups, group = lb - trow * groups;
    pass2_block<S, C, WALL, TS, OH, WPS, ONE>(L, src, dst, group, trow, pass2_lds);
}

// Two-step passes over the blocks of many lattices: pwork[b] = (lattice,
// column group, row band) of logical workgroup b.
template <int TS, int OH, int WPS>
__global__ __launch_bounds__(TS * WPS * kWave) void k_step_pass2_batch(const LatDev<float> *__restrict__ lats,
                                                                       const uint4 *__restrict__ pwork, int parity) {
    extern __shared__ __align__(16) unsigned char pass2_lds[];
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint4 wk = pwork[lb];
    const LatDev<float> L = lats[wk.x];
    pass2_block<float, float, WALL_ROW, TS, OH, WPS, 0>(L, parity ? L.fb : L.fa, parity ? L.fa : L.fb, wk.y, wk.z,
                                                     pass2_lds);
}

template <class S, class C, int WALL>
__global__ __launch_bounds__(kBlockThreads) void k_diag(const LatDev<C> *__restrict__ lats, const uint4 *__restrict__ work,
                                              uint32_t nwork, LatDev<C> single, int parity, int write_mom,
                                              int compare, int update) {
    const uint32_t gw = logical_wave();
    uint32_t nw = lats ? nwork : single.strips * single.segs;
    if (gw >= nw) return;
    LatDev<C> L;
    uint32_t strip, seg;
    if (lats) {
        const uint4 wk = work[gw];
        L = lats[wk.x];
        strip = wk.y;
        seg = wk.z;
    } else {
        L = single;
        seg = gw / L.strips;
        strip = gw - seg * L.strips;
    }
    const void *src = parity ? L.fb : L.fa;
    DiagAct<S, C, WALL> act;
    act.write_mom = write_mom;
    act.compare = compare;
    act.update = update;
    march<S, C, WALL>(L, src, strip, seg, act);
    const double v[6] = {act.s_rho, act.s_jx, act.s_jy, act.s_du, act.s_u, act.s_bad};
    double *out = L.partials + 8 * size_t(gw - L.wave0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double t = wave_sum(v[k]);
        if ((threadIdx.x & (kWave - 1)) == 0) out[k] = t;
    }
}

// Deterministic reduction of partial rows: out[b*out_stride + j] = sum over
// rows r in [ranges[2b], ranges[2b+1]) of part[r*stride + j], j < width, in a
// fixed order.  One block per output row.
constexpr uint32_t kReduceMaxWidth = 10;

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, const uint32_t *__restrict__ ranges,
                                                uint32_t stride, uint32_t width, double *__restrict__ out,
                                                uint32_t out_stride) {
    // one pass over the rows, every column at once; then a fixed-order tree
    __shared__ double sm[kReduceMaxWidth][256];
    const uint32_t b = blockIdx.x, t = threadIdx.x;
    const uint32_t beg = ranges[2 * b], end = ranges[2 * b + 1];
    double acc[kReduceMaxWidth];
#pragma unroll
    for (uint32_t j = 0; j < kReduceMaxWidth; ++j) acc[j] = 0.0;
    for (uint32_t r = beg + t; r < end; r += blockDim.x) {
        const double *row = part + size_t(r) * stride;
#pragma unroll
        for (uint32_t j = 0; j < kReduceMaxWidth; ++j)
            if (j < width) acc[j] += row[j];
    }
#pragma unroll
    for (uint32_t j = 0; j < kReduceMaxWidth; ++j) sm[j][t] = acc[j];
    __syncthreads();
    for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s)
            for (uint32_t j = 0; j < width; ++j) sm[j][t] += sm[j][t + s];
        __syncthreads();
    }
    if (t < width) out[size_t(b) * out_stride + t] = sm[t][0];
}

// ------------------------------------------------ contact-angle isoline pass
// mode 0: (n, sum x, sum y)
// mode 1: algebraic circle sums about (mx, my):
//         (n, Sx, Sy, Sxx, Sxy, Syy, Sxq, Syq, Sq), q = x^2 + y^2
// mode 2: Gauss-Newton normal equations of r = |p - c| - R about (mx, my):
//         (n, J00, J01, J02, J11, J12, J22, g0, g1, g2), g = -J^T r
struct IsoArgs {
    uint32_t nx, ny;
    int per_node;          // phi indexed per node (else per row)
    int mode;
    double iso, phi_max, mx, my, xc, yc, R;
    int side;              // 0: every point; -1: x <= xs; +1: x >= xs
    int unwrap;            // x taken in [xmid - nx/2, xmid + nx/2)
    double xs, xmid;
};

__device__ inline void iso_accumulate(const IsoArgs &a, double px, double py, double acc[10]) {
    const double x = px - a.mx, y = py - a.my;
    acc[0] += 1.0;
    if (a.mode == 0) {
        acc[1] += px;
        acc[2] += py;
    } else if (a.mode == 1) {
        const double q = x * x + y * y;
        acc[1] += x; acc[2] += y; acc[3] += x * x; acc[4] += x * y; acc[5] += y * y;
        acc[6] += x * q; acc[7] += y * q; acc[8] += q;
    } else if (a.mode == 2) {
        const double dx = x - a.xc, dy = y - a.yc;
        const double d = sqrt(dx * dx + dy * dy);
        const double j0 = -dx / d, j1 = -dy / d, j2 = -1.0, r = d - a.R;
        acc[1] += j0 * j0; acc[2] += j0 * j1; acc[3] += j0 * j2;
        acc[4] += j1 * j1; acc[5] += j1 * j2; acc[6] += j2 * j2;
        acc[7] -= j0 * r; acc[8] -= j1 * r; acc[9] -= j2 * r;
    } else if (a.mode == 5) {
        // circular mean of x over the periodic direction
        const double t = 6.283185307179586 * px / double(a.nx);
        acc[1] += sin(t);
        acc[2] += cos(t);
    }
}

// x of a crossing in the window [xmid - nx/2, xmid + nx/2) when unwrapping.
__device__ inline double iso_unwrap(const IsoArgs &a, double px) {
    if (!a.unwrap) return px;
    const double n = double(a.nx);
    return px - n * floor((px - a.xmid) / n + 0.5);
}

// Calls emit(x, y) for every rho = iso crossing on the edges from node n to
// its right (periodic) and upper neighbours, both ends in region phi < phi_max.
template <class C, class Emit>
__device__ inline void iso_crossings(const IsoArgs &a, const C *__restrict__ rho, const double *__restrict__ phi,
                                     uint32_t n, Emit &&emit) {
    const uint32_t y = n / a.nx, x = n - y * a.nx;
    const double pa = a.per_node ? phi[n] : phi[y];
    if (!(pa < a.phi_max)) return;
    const double ra = double(rho[n]);
    const bool ia = ra >= a.iso;
    const uint32_t xr = x + 1 == a.nx ? 0 : x + 1;
    const uint32_t nr = y * a.nx + xr;
    const double pr = a.per_node ? phi[nr] : phi[y];
    const double rr = double(rho[nr]);
    if (pr < a.phi_max && ia != (rr >= a.iso)) {
        const double t = (a.iso - ra) / (rr - ra);
        emit(double(x) + t, double(y));
    }
    if (y + 1 < a.ny) {
        const uint32_t nu = n + a.nx;
        const double pu = a.per_node ? phi[nu] : phi[y + 1];
        const double ru = double(rho[nu]);
        if (pu < a.phi_max && ia != (ru >= a.iso)) {
            const double t = (a.iso - ra) / (ru - ra);
            emit(double(x), double(y) + t);
        }
    }
}

template <class C>
__global__ __launch_bounds__(256) void k_isoline(IsoArgs a, const C *__restrict__ rho,
                                                 const double *__restrict__ phi, double *__restrict__ part) {
    constexpr int kIsoWaves = 256 / kWave;   // launched with 256 threads
    __shared__ double sm[kIsoWaves][10];
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const uint32_t N = a.nx * a.ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) {
        if (a.mode == 4) {
            // liquid nodes of region III: (count, sum rho, sum rho u_x, sum rho u_y);
            // rho points at the moment planes (rho | u_x | u_y)
            const uint32_t y = n / a.nx;
            const double pa = a.per_node ? phi[n] : phi[y];
            const double r = double(rho[n]);
            if (pa < a.phi_max && r >= a.iso) {
                acc[0] += 1.0;
                acc[1] += r;
                acc[2] += r * double(rho[N + n]);
                acc[3] += r * double(rho[2 * size_t(N) + n]);
            }
        } else {
            iso_crossings(a, rho, phi, n, [&](double px, double py) {
                px = iso_unwrap(a, px);
                if ((a.side < 0 && px > a.xs) || (a.side > 0 && px < a.xs)) return;
                iso_accumulate(a, px, py, acc);
            });
        }
    }
    const uint32_t w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const double t = wave_sum(acc[k]);
        if ((threadIdx.x & (kWave - 1)) == 0) sm[w][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        double s = 0.0;
        for (int i = 0; i < kIsoWaves; ++i) s += sm[i][threadIdx.x];
        part[size_t(blockIdx.x) * 10 + threadIdx.x] = s;
    }
}

// Highest crossing (largest y, then smallest unwrapped x) of each block:
// part[10 b] = found (0/1), part[10 b + 1] = x, part[10 b + 2] = y.
template <class C>
__global__ __launch_bounds__(256) void k_isoline_top(IsoArgs a, const C *__restrict__ rho,
                                                     const double *__restrict__ phi, double *__restrict__ part) {
    constexpr int kIsoWaves = 256 / kWave;
    __shared__ double sm[kIsoWaves][3];
    double found = 0.0, bx = 0.0, by = -1.0;
    const uint32_t N = a.nx * a.ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    auto better = [](double x1, double y1, double x2, double y2) { return y1 > y2 || (y1 == y2 && x1 < x2); };
    if (n < N)
        iso_crossings(a, rho, phi, n, [&](double px, double py) {
            px = iso_unwrap(a, px);
            if (found == 0.0 || better(px, py, bx, by)) {
                found = 1.0;
                bx = px;
                by = py;
            }
        });
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double f2 = __shfl_xor(found, o, kWave), x2 = __shfl_xor(bx, o, kWave), y2 = __shfl_xor(by, o, kWave);
        if (f2 != 0.0 && (found == 0.0 || better(x2, y2, bx, by))) {
            found = 1.0;
            bx = x2;
            by = y2;
        }
    }
    const uint32_t w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sm[w][0] = found;
        sm[w][1] = bx;
        sm[w][2] = by;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double f = 0.0, x = 0.0, y = -1.0;
        for (int i = 0; i < kIsoWaves; ++i)
            if (sm[i][0] != 0.0 && (f == 0.0 || better(sm[i][1], sm[i][2], x, y))) {
                f = 1.0;
                x = sm[i][1];
                y = sm[i][2];
            }
        part[size_t(blockIdx.x) * 10] = f;
        part[size_t(blockIdx.x) * 10 + 1] = x;
        part[size_t(blockIdx.x) * 10 + 2] = y;
    }
}

// x-sums of the reported u_x per row (slip profile); one block per row.
template <class C>
__global__ __launch_bounds__(256) void k_profile(uint32_t nx, const C *__restrict__ ux, double *__restrict__ out) {
    __shared__ double sm[256];
    const uint32_t y = blockIdx.x;
    double acc = 0.0;
    for (uint32_t x = threadIdx.x; x < nx; x += blockDim.x) acc += double(ux[size_t(y) * nx + x]);
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[y] = sm[0];
}

// ------------------------------------------------------------ state copies
// Eq. f2 at equilibrium in FP64: w rho (1 + c.u/theta + ((c.u)^2 - theta u^2) / (2 theta^2)).
template <int LQ> __device__ inline double feq_component(int q, double rho, double ux, double uy) {
    using V = VelSet<LQ>;
    const double cu = V::cx(q) * ux + V::cy(q) * uy;
    if constexpr (LQ == 9)
        return kW[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
    const double th = V::theta;
    return V::w(q) * rho * (1.0 + cu / th + (cu * cu - th * (ux * ux + uy * uy)) / (2.0 * th * th));
}

// Stored (pre-stream) populations such that pulling yields feq(rho0, u0):
// stored_q(x) = feq_q at node x + c_q.
template <class S, class C, int LQ>
__global__ __launch_bounds__(256) void k_init(uint32_t nx, uint32_t ny, uint32_t P, const double *__restrict__ rho0,
                                              const double *__restrict__ ux0, const double *__restrict__ uy0,
                                              typename Codec<S>::Raw *__restrict__ dst, C rho_ref) {
    using V = VelSet<LQ>;
    const uint32_t N = nx * ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t y = n / nx, x = n - y * nx;
    for (int q = 0; q < V::Q; ++q) {
        const uint32_t xs = (x + 3 * nx + V::cx(q)) % nx, ys = (y + 3 * ny + V::cy(q)) % ny;
        const uint32_t m = ys * nx + xs;
        const double v = feq_component<LQ>(q, rho0[m], ux0 ? ux0[m] : 0.0, uy0 ? uy0[m] : 0.0);
        dst[q * P + n] = Codec<S>::template encode<C>(C(v), q, rho_ref);
    }
}

// Post-streaming plane q as float64: out(x) = stored_q(x - c_q), decoded
// exactly as the step kernel decodes it.
template <class S, class C, int LQ>
__global__ __launch_bounds__(256) void k_get_plane(uint32_t nx, uint32_t ny, uint32_t P, int q,
                                                   const typename Codec<S>::Raw *__restrict__ src,
                                                   double *__restrict__ out, C rho_ref) {
    using V = VelSet<LQ>;
    const uint32_t N = nx * ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t y = n / nx, x = n - y * nx;
    const uint32_t xs = (x + 3 * nx - V::cx(q)) % nx, ys = (y + 3 * ny - V::cy(q)) % ny;
    out[n] = double(Codec<S>::template decode<C>(src[q * P + ys * nx + xs], q, rho_ref));
}

// Inverse of k_get_plane: stored_q(x) = in(x + c_q).
template <class S, class C, int LQ>
__global__ __launch_bounds__(256) void k_set_plane(uint32_t nx, uint32_t ny, uint32_t P, int q,
                                                   const double *__restrict__ in,
                                                   typename Codec<S>::Raw *__restrict__ dst, C rho_ref) {
    using V = VelSet<LQ>;
    const uint32_t N = nx * ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t y = n / nx, x = n - y * nx;
    const uint32_t xs = (x + 3 * nx + V::cx(q)) % nx, ys = (y + 3 * ny + V::cy(q)) % ny;
    dst[q * P + n] = Codec<S>::template encode<C>(C(in[ys * nx + xs]), q, rho_ref);
}

// ------------------------------------------------------------- wall tables
__device__ inline double step_profile(double s, double w) { return 0.5 * (1.0 - tanh(s / w)); }

// Signed distance of row y to the nearest face of the solid band
// [ny - P, ny) (faces on rows 0 and ny - P), negative inside the band.
__device__ inline double slab_distance(int y, int ny, int P) {
    if (y <= ny - P) {
        const int a = y, b = ny - P - y;
        return double(a < b ? a : b);
    }
    const int a = y - (ny - P), b = ny - y;
    return -double(a < b ? a : b);
}

// Per-row tables for a flat slab (or all zeros when P == 0):
//   tab[2y] = phi(y)^eps,  tab[2y+1] = S_y(y) = sum_i w_i psi_FS(y + c_iy) c_iy,
//   psi_FS = G_A psiA - G_R psiR;  phi_raw[y] = phi(y) in float64.
template <class C, int LQ>
__global__ __launch_bounds__(256) void k_walls_row(int ny, int P, double width, double core, double tail,
                                                   double eps, double GR, double GA, C *__restrict__ tab,
                                                   double *__restrict__ phi_raw) {
    using V = VelSet<LQ>;
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= ny) return;
    if (P <= 0) {
        tab[2 * y] = C(0);
        tab[2 * y + 1] = C(0);
        phi_raw[y] = 0.0;
        return;
    }
    auto psi_fs = [&](int yy) {
        const double s = slab_distance(((yy % ny) + ny) % ny, ny, P);
        const double r = step_profile(s, core);
        const double a = step_profile(s, tail) - r;
        return GA * a - GR * r;
    };
    double sy = 0.0;
    for (int q = 0; q < V::Q; ++q) sy += V::w(q) * psi_fs(y + V::cy(q)) * V::cy(q);
    const double phi = step_profile(slab_distance(y, ny, P), width);
    tab[2 * y] = C(pow(phi, eps));
    tab[2 * y + 1] = C(sy);
    phi_raw[y] = phi;
}

// Per-node tables from caller fields (phi, psiR, psiA), each [ny][nx]:
//   tab = [phi^eps | S_x | S_y], phi_raw = phi.
template <class C, int LQ>
__global__ __launch_bounds__(256) void k_walls_node(uint32_t nx, uint32_t ny, const double *__restrict__ fields,
                                                    double eps, double GR, double GA, C *__restrict__ tab,
                                                    double *__restrict__ phi_raw) {
    using V = VelSet<LQ>;
    const uint32_t N = nx * ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t y = n / nx, x = n - y * nx;
    double sx = 0.0, sy = 0.0;
    for (int q = 0; q < V::Q; ++q) {
        const uint32_t m = ((y + 3 * ny + V::cy(q)) % ny) * nx + (x + 3 * nx + V::cx(q)) % nx;
        const double fs = GA * fields[2 * size_t(N) + m] - GR * fields[size_t(N) + m];
        sx += V::w(q) * fs * V::cx(q);
        sy += V::w(q) * fs * V::cy(q);
    }
    const double phi = fields[n];
    tab[n] = C(pow(phi, eps));
    tab[N + n] = C(sx);
    tab[2 * size_t(N) + n] = C(sy);
    phi_raw[n] = phi;
}

// Wall functions of arbitrary geometry (Appendix A, eq. iteration): one pass
// of the recursive filter, out = sum_i w_i in(x + r_i) over the lattice's
// velocity set (periodic), held at 1 where bnd != 0.  Set-up only.
template <int LQ>
__global__ __launch_bounds__(256) void k_filter_pass(uint32_t nx, uint32_t ny, const double *__restrict__ in,
                                                     const double *__restrict__ bnd, double *__restrict__ out) {
    using V = VelSet<LQ>;
    const uint32_t N = nx * ny;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t y = n / nx, x = n - y * nx;
    double acc = 0.0;
    for (int q = 0; q < V::Q; ++q) {
        const uint32_t m = ((y + 3 * ny + V::cy(q)) % ny) * nx + (x + 3 * nx + V::cx(q)) % nx;
        acc += V::w(q) * in[m];
    }
    out[n] = bnd[n] != 0.0 ? 1.0 : acc;
}

// psiA = phi - psiR, fields laid out [phi | psiR | psiA].
__global__ __launch_bounds__(256) void k_filter_finish(uint32_t N, double *__restrict__ fields) {
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) fields[2 * size_t(N) + n] = fields[n] - fields[size_t(N) + n];
}

// ================================================================ launchers
static inline uint32_t blocks_for(uint32_t waves) { return (waves + kBlockWaves - 1) / kBlockWaves; }
static inline uint32_t blocks_nodes(uint32_t n) { return (n + 255) / 256; }

// Calls fn(S{}, C{}) with the storage/arithmetic pair of a storage code.
template <class Fn> static hipError_t dispatch(int storage, Fn &&fn) {
    switch (storage) {
    case STORE_F32: return fn(float{}, float{});
    case STORE_F16: return fn(Dev16{}, float{});
    case STORE_F64: return fn(double{}, double{});
    case STORE_F32X: return fn(float{}, double{});
    default: return hipErrorInvalidValue;
    }
}

// Calls fn(integral_constant<int, s>) for a tile shape index.
template <class Fn> static hipError_t with_shape(int shape, Fn &&fn) {
    switch (shape) {
    case 0: return fn(std::integral_constant<int, 0>{});
    case 1: return fn(std::integral_constant<int, 1>{});
    case 2: return fn(std::integral_constant<int, 2>{});
    case 3: return fn(std::integral_constant<int, 3>{});
    case 4: return fn(std::integral_constant<int, 4>{});
    case 5: return fn(std::integral_constant<int, 5>{});
    case 6: return fn(std::integral_constant<int, 6>{});
    case 7: return fn(std::integral_constant<int, 7>{});
    case 8: return fn(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}
static_assert(kNumTileShapes == 9, "with_shape lists every tile shape");

uint32_t step_tiles(uint32_t nx, uint32_t ny, int shape) {
    return tile_groups(nx, shape) * tile_rows(ny, shape);
}

hipError_t launch_step(int storage, const LatDevAny &L, int wall, int shape, int parity, hipStream_t st) {
    return dispatch(storage, [&](auto s, auto c) {
        using S = decltype(s);
        using C = decltype(c);
        LatDev<C> d = L.get<C>();
        const void *src = parity ? d.fb : d.fa;
        void *dst = parity ? d.fa : d.fb;
        // tau = 1 runs the instantiation compiled for it (fewer registers)
        const bool one = L.omega == 1.0;
        return with_shape(shape, [&](auto sh) {
            constexpr int SH = decltype(sh)::value;
            const uint32_t nb = step_tiles(d.nx, d.ny, SH);
            const dim3 block(kShapeWaves[SH] * kWave);
            if (wall == WALL_ROW && one)
                hipLaunchKernelGGL((k_step_tiles<S, C, WALL_ROW, SH, 1>), dim3(nb), block, 0, st, d, src, dst);
            else if (wall == WALL_ROW)
                hipLaunchKernelGGL((k_step_tiles<S, C, WALL_ROW, SH, 0>), dim3(nb), block, 0, st, d, src, dst);
            else if (one)
                hipLaunchKernelGGL((k_step_tiles<S, C, WALL_NODE, SH, 1>), dim3(nb), block, 0, st, d, src, dst);
            else
                hipLaunchKernelGGL((k_step_tiles<S, C, WALL_NODE, SH, 0>), dim3(nb), block, 0, st, d, src, dst);
            return hipGetLastError();
        });
    });
}

template <int V> struct Pass2Var {
    static constexpr int TS = kPass2Strips[V], OH = kPass2Rows[V], WPS = kPass2WavesPerStrip[V];
    using G = Pass2Geo<TS, OH, WPS>;
};

hipError_t launch_step_pass2(int storage, const LatDevAny &L, int wall, int variant, int parity, hipStream_t st) {
    if (!pass2_ok(storage) || L.lattice != 9) return hipErrorInvalidValue;
    auto go = [&](auto s, auto vc) -> hipError_t {
        using S = decltype(s);
        using C = std::conditional_t<std::is_same_v<S, double>, double, float>;
        constexpr int V = decltype(vc)::value;
        using PV = Pass2Var<V>;
        using G = typename PV::G;
        LatDev<C> d = L.get<C>();
        const void *src = parity ? d.fb : d.fa;
        void *dst = parity ? d.fa : d.fb;
        const uint32_t nb = pass2_blocks(d.nx, d.ny, V);
        const size_t lds = G::lds_words * sizeof(C);
        const bool one = L.omega == 1.0;   // tau = 1: the instantiation compiled for it
        if (wall == WALL_ROW && one)
            hipLaunchKernelGGL((k_step_pass2<S, C, WALL_ROW, PV::TS, PV::OH, PV::WPS, 1>), dim3(nb), dim3(G::NT),
                               lds, st, d, src, dst);
        else if (wall == WALL_ROW)
            hipLaunchKernelGGL((k_step_pass2<S, C, WALL_ROW, PV::TS, PV::OH, PV::WPS, 0>), dim3(nb), dim3(G::NT),
                               lds, st, d, src, dst);
        else if (one)
            hipLaunchKernelGGL((k_step_pass2<S, C, WALL_NODE, PV::TS, PV::OH, PV::WPS, 1>), dim3(nb), dim3(G::NT),
                               lds, st, d, src, dst);
        else
            hipLaunchKernelGGL((k_step_pass2<S, C, WALL_NODE, PV::TS, PV::OH, PV::WPS, 0>), dim3(nb), dim3(G::NT),
                               lds, st, d, src, dst);
        return hipGetLastError();
    };
    auto with_var = [&](auto s) -> hipError_t {
        switch (variant) {
        case 0: return go(s, std::integral_constant<int, 0>{});
        case 1: return go(s, std::integral_constant<int, 1>{});
        case 2: return go(s, std::integral_constant<int, 2>{});
        case 3: return go(s, std::integral_constant<int, 3>{});
        case 4: return go(s, std::integral_constant<int, 4>{});
        case 5: return go(s, std::integral_constant<int, 5>{});
        case 6: return go(s, std::integral_constant<int, 6>{});
        case 7: return go(s, std::integral_constant<int, 7>{});
        case 8: return go(s, std::integral_constant<int, 8>{});
        default: return hipErrorInvalidValue;
        }
    };
    static_assert(kPass2Variants == 9, "launch_step_pass2 lists every variant");
    if (storage == STORE_F32) return with_var(float{});
    if (storage == STORE_F64) return with_var(double{});
    return with_var(Dev16{});
}

hipError_t launch_step_pass2_batch(const void *lats, const uint4 *pwork, uint32_t nblocks, int variant, int parity,
                                   hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    auto go = [&](auto vc) -> hipError_t {
        constexpr int V = decltype(vc)::value;
        using PV = Pass2Var<V>;
        hipLaunchKernelGGL((k_step_pass2_batch<PV::TS, PV::OH, PV::WPS>), dim3(nblocks), dim3(PV::G::NT),
                           PV::G::lds_bytes, st, (const LatDev<float> *)lats, pwork, parity);
        return hipGetLastError();
    };
    switch (variant) {
    case 0: return go(std::integral_constant<int, 0>{});
    case 1: return go(std::integral_constant<int, 1>{});
    case 2: return go(std::integral_constant<int, 2>{});
    case 3: return go(std::integral_constant<int, 3>{});
    case 4: return go(std::integral_constant<int, 4>{});
    case 5: return go(std::integral_constant<int, 5>{});
    case 6: return go(std::integral_constant<int, 6>{});
    case 7: return go(std::integral_constant<int, 7>{});
    case 8: return go(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_batch(const void *lats, const uint4 *twork, uint32_t ntiles, int shape, int parity,
                             hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    return with_shape(shape, [&](auto sh) {
        constexpr int SH = decltype(sh)::value;
        hipLaunchKernelGGL((k_step_tiles_batch<float, float, WALL_ROW, SH>), dim3(ntiles),
                           dim3(kShapeWaves[SH] * kWave), 0, st, (const LatDev<float> *)lats, twork, parity);
        return hipGetLastError();
    });
}

hipError_t launch_diag(int storage, const void *lats, const uint4 *work, uint32_t nwork, const LatDevAny &single,
                       int wall, int parity, int write_mom, int compare, int update, hipStream_t st) {
    return dispatch(storage, [&](auto s, auto c) {
        using S = decltype(s);
        using C = decltype(c);
        LatDev<C> d = single.get<C>();
        const uint32_t waves = lats ? nwork : d.strips * d.segs;
        if (wall == WALL_ROW)
            hipLaunchKernelGGL((k_diag<S, C, WALL_ROW>), dim3(blocks_for(waves)), dim3(kBlockThreads), 0, st,
                               (const LatDev<C> *)lats, work, nwork, d, parity, write_mom, compare, update);
        else
            hipLaunchKernelGGL((k_diag<S, C, WALL_NODE>), dim3(blocks_for(waves)), dim3(kBlockThreads), 0, st,
                               (const LatDev<C> *)lats, work, nwork, d, parity, write_mom, compare, update);
        return hipGetLastError();
    });
}

hipError_t launch_reduce(const double *part, const uint32_t *ranges, uint32_t nout, uint32_t stride,
                         uint32_t width, double *out, uint32_t out_stride, hipStream_t st) {
    if (width > kReduceMaxWidth || width > stride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3(nout), dim3(256), 0, st, part, ranges, stride, width, out, out_stride);
    return hipGetLastError();
}

hipError_t launch_isoline(int f64, const IsoParams &p, const void *rho, const double *phi, double *part,
                          hipStream_t st) {
    IsoArgs a{p.nx, p.ny, p.per_node, p.mode, p.iso, p.phi_max, p.mx, p.my, p.xc, p.yc, p.R,
              p.side, p.unwrap, p.xs, p.xmid};
    const uint32_t nb = blocks_nodes(p.nx * p.ny);
    if (p.mode == 3) {
        if (f64)
            hipLaunchKernelGGL(k_isoline_top<double>, dim3(nb), dim3(256), 0, st, a, (const double *)rho, phi, part);
        else
            hipLaunchKernelGGL(k_isoline_top<float>, dim3(nb), dim3(256), 0, st, a, (const float *)rho, phi, part);
        return hipGetLastError();
    }
    if (f64)
        hipLaunchKernelGGL(k_isoline<double>, dim3(nb), dim3(256), 0, st, a, (const double *)rho, phi, part);
    else
        hipLaunchKernelGGL(k_isoline<float>, dim3(nb), dim3(256), 0, st, a, (const float *)rho, phi, part);
    return hipGetLastError();
}

uint32_t isoline_blocks(uint32_t nodes) { return blocks_nodes(nodes); }

hipError_t launch_profile(int f64, uint32_t nx, uint32_t ny, const void *ux, double *out, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_profile<double>, dim3(ny), dim3(256), 0, st, nx, (const double *)ux, out);
    else
        hipLaunchKernelGGL(k_profile<float>, dim3(ny), dim3(256), 0, st, nx, (const float *)ux, out);
    return hipGetLastError();
}

// Calls fn(integral_constant<int, LQ>) for a population count (9 or 21).
template <class Fn> static hipError_t with_lattice(int lattice, Fn &&fn) {
    if (lattice == 21) return fn(std::integral_constant<int, 21>{});
    return fn(std::integral_constant<int, 9>{});
}

hipError_t launch_init(int storage, int lattice, uint32_t nx, uint32_t ny, uint32_t pstride, const double *rho0,
                       const double *ux0, const double *uy0, void *dst, double rho_ref, hipStream_t st) {
    const uint32_t nb = blocks_nodes(nx * ny);
    return dispatch(storage, [&](auto s, auto c) {
        using S = decltype(s);
        using C = decltype(c);
        return with_lattice(lattice, [&](auto lq) {
            constexpr int LQ = decltype(lq)::value;
            hipLaunchKernelGGL((k_init<S, C, LQ>), dim3(nb), dim3(256), 0, st, nx, ny, pstride, rho0, ux0, uy0,
                               (typename Codec<S>::Raw *)dst, C(rho_ref));
            return hipGetLastError();
        });
    });
}

hipError_t launch_plane(int storage, int lattice, int set, uint32_t nx, uint32_t ny, uint32_t pstride, int q,
                        void *pop, double *buf, double rho_ref, hipStream_t st) {
    const uint32_t nb = blocks_nodes(nx * ny);
    return dispatch(storage, [&](auto s, auto c) {
        using S = decltype(s);
        using C = decltype(c);
        using Raw = typename Codec<S>::Raw;
        return with_lattice(lattice, [&](auto lq) {
            constexpr int LQ = decltype(lq)::value;
            if (set)
                hipLaunchKernelGGL((k_set_plane<S, C, LQ>), dim3(nb), dim3(256), 0, st, nx, ny, pstride, q, buf,
                                   (Raw *)pop, C(rho_ref));
            else
                hipLaunchKernelGGL((k_get_plane<S, C, LQ>), dim3(nb), dim3(256), 0, st, nx, ny, pstride, q,
                                   (const Raw *)pop, buf, C(rho_ref));
            return hipGetLastError();
        });
    });
}

hipError_t launch_walls_row(int f64, int lattice, int ny, int P, double width, double core, double tail, double eps,
                            double GR, double GA, void *tab, double *phi_raw, hipStream_t st) {
    const uint32_t nb = blocks_nodes(uint32_t(ny));
    return with_lattice(lattice, [&](auto lq) {
        constexpr int LQ = decltype(lq)::value;
        if (f64)
            hipLaunchKernelGGL((k_walls_row<double, LQ>), dim3(nb), dim3(256), 0, st, ny, P, width, core, tail, eps,
                               GR, GA, (double *)tab, phi_raw);
        else
            hipLaunchKernelGGL((k_walls_row<float, LQ>), dim3(nb), dim3(256), 0, st, ny, P, width, core, tail, eps,
                               GR, GA, (float *)tab, phi_raw);
        return hipGetLastError();
    });
}

hipError_t launch_walls_node(int f64, int lattice, uint32_t nx, uint32_t ny, const double *fields, double eps,
                             double GR, double GA, void *tab, double *phi_raw, hipStream_t st) {
    const uint32_t nb = blocks_nodes(nx * ny);
    return with_lattice(lattice, [&](auto lq) {
        constexpr int LQ = decltype(lq)::value;
        if (f64)
            hipLaunchKernelGGL((k_walls_node<double, LQ>), dim3(nb), dim3(256), 0, st, nx, ny, fields, eps, GR, GA,
                               (double *)tab, phi_raw);
        else
            hipLaunchKernelGGL((k_walls_node<float, LQ>), dim3(nb), dim3(256), 0, st, nx, ny, fields, eps, GR, GA,
                               (float *)tab, phi_raw);
        return hipGetLastError();
    });
}

hipError_t launch_filter_walls(int lattice, uint32_t nx, uint32_t ny, double *fields, const double *bnd,
                               int n_core, int n_wall, hipStream_t st) {
    const size_t N = size_t(nx) * ny;
    double *slot[3] = {fields, fields + N, fields + 2 * N};   // phi, psiR, psiA
    const uint32_t nb = blocks_nodes(uint32_t(N));
    double *cur = slot[0], *nxt = slot[2];
    if (n_core == 0) {
        const hipError_t e = hipMemcpyAsync(slot[1], cur, N * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    for (int pass = 1; pass <= n_wall; ++pass) {
        if (lattice == 21)
            hipLaunchKernelGGL(k_filter_pass<21>, dim3(nb), dim3(256), 0, st, nx, ny, cur, bnd, nxt);
        else
            hipLaunchKernelGGL(k_filter_pass<9>, dim3(nb), dim3(256), 0, st, nx, ny, cur, bnd, nxt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(cur, nxt);
        if (pass == n_core) {
            e = hipMemcpyAsync(slot[1], cur, N * sizeof(double), hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
    }
    if (cur != slot[0]) {
        const hipError_t e = hipMemcpyAsync(slot[0], cur, N * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_filter_finish, dim3(nb), dim3(256), 0, st, uint32_t(N), fields);
    return hipGetLastError();
}

}  // namespace lbmwet
