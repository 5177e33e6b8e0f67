// D2Q21 kernels (gfx950): the paper's own lattice (Sec. II.A, Tab. I), each
// node reaching three sites per step, with the exponential or the
// equation-of-state pseudo-potential (eq. EOS).
//
// k_tile_q21: one workgroup of kQ21Waves waves owns a strip of 64 columns of
// which the 3 on each side are halo columns (58 output columns) and
// kQ21Waves * R consecutive rows (R = 2, or 1 on lattices too small to fill
// the chip with two-row tiles) of which the 3 on each side are halo rows.  Every wave loads its rows at once (21 pulled loads per row, shifts up
// to +-3 in both directions), computes density, momentum and pseudo-potential
// of all 64 columns, including the halo ones from their own loads, and
// publishes the pseudo-potential in LDS; after one barrier every output node
// sums w_i psi(x + c_i) c_i over the 20 moving directions from LDS, forms the
// forces of eqs. force_SC, force_SC_FS and wall_shift, and either collides and
// stores (step) or accumulates the diagnostic sums (diagnostic pass).  At
// tau = 1 the collision needs only the moments, so the populations are not
// kept across the barrier.
//
// k_march_q21 (further down): the binary32 step on large lattices, marching
// workgroups of 256 aligned columns down 128-row segments; it reloads only 6
// rows per segment and stores whole 256-byte rows.  Both kernels build every
// node's update from the same functions in the same order, so they produce
// bitwise the same populations.
#include <type_traits>

#include "launch.hpp"
#include "lbm_device.hpp"

namespace lbmwet {

namespace {

constexpr int kH = 3;   // halo width: the largest |c_i| of D2Q21
constexpr size_t kQ21LdsReserve = 96 * 1024;   // > half of the CU's 160 KB LDS

// Pseudo-potential of the fluid-fluid force.  PSI 0: 1 - exp(-rho); PSI 1:
// eq. EOS, psi^2 = 2 (rho theta - p_EOS) / theta (the 1/theta factor makes
// the bulk pressure equal p_EOS for the force of eq. force_SC with G = -1),
// linear in rho on each branch: k_b (rho - rho_b) + a_b.
template <class C, int PSI> __device__ inline C psi21(const LatDev<C> &L, C rho) {
    if constexpr (PSI == 0) {
        return psi_of<C>(rho);
    } else {
        C a;
        if (rho <= L.eos_r1) a = L.eos_kV * rho;
        else if (rho <= L.eos_r2) a = L.eos_kU * (rho - L.eos_r1) + L.eos_aU;
        else a = L.eos_kL * (rho - L.eos_r2) + L.eos_aL;
        return sqrt(a > C(0) ? a : C(0));
    }
}

// Eq. M0 in a fixed order (every tile computes a halo node's density with
// the same additions as the tile that owns the node).
template <class C> __device__ inline C density21(const C f[Q21]) {
    C a = (f[1] + f[3]) + (f[2] + f[4]);
    C b = (f[5] + f[7]) + (f[6] + f[8]);
    C c = (f[9] + f[11]) + (f[10] + f[12]);
    C d = (f[13] + f[15]) + (f[14] + f[16]);
    C e = (f[17] + f[19]) + (f[18] + f[20]);
    return f[0] + (((a + b) + (c + d)) + e);
}

// Momentum coefficient of each velocity class, B = 1.5 w |c|_inf: the
// equilibrium's momentum term of population i is B_i (s_ix m_x + s_iy m_y),
// s_i = sign(c_i).  Its first moment is (2 B_1 + 4 B_2 + 4 B_3 + 8 B_4 +
// 6 B_5) m, and 1.5 sum_i w_i c_ix^2 = 1 makes the bracket 1.  In binary32 the
// five constants are chosen (within 6e-7 relative of the exact values) so
// that the bracket is exactly 1: the equilibrium then carries exactly the
// momentum it is given, with no per-step gain or loss that would add up.
template <class C> struct Mom21;
template <> struct Mom21<float> {
    static constexpr float b1 = 0x1.000000p-3f;      // 1.5 / 12
    static constexpr float b2 = 0x1.c71c78p-4f;      // 1.5 * 2/27
    static constexpr float b3 = 0x1.ddddd4p-5f;      // 2 * 1.5 * 7/360
    static constexpr float b4 = 0x1.c71c62p-8f;      // 2 * 1.5 / 432
    static constexpr float b5 = 0x1.6c16d0p-9f;      // 3 * 1.5 / 1620
};
template <> struct Mom21<double> {
    static constexpr double b1 = 1.5 / 12.0, b2 = 1.5 * 2.0 / 27.0, b3 = 3.0 * 7.0 / 360.0;
    static constexpr double b4 = 3.0 / 432.0, b5 = 4.5 / 1620.0;
};
template <class C> __device__ constexpr C mom21(int q) {
    using M = Mom21<C>;
    return q == 0 ? C(0) : q <= 4 ? M::b1 : q <= 8 ? M::b2 : q <= 12 ? M::b3 : q <= 16 ? M::b4 : M::b5;
}
constexpr int sgn(int v) { return (v > 0) - (v < 0); }

// Eq. f2 at equilibrium on D2Q21 (theta = 2/3) from density and momentum
// m = rho u: feq_i = w_i rho + w_i rho (1.125 (c_i.u)^2 - 0.75 u^2) + B_i s_i.m,
// the velocity terms added to w_i rho last.  Opposite populations get the
// same first two terms and momentum terms of opposite sign.
template <class C> __device__ inline void equilibrium21(C rho, C inv_rho, C mx, C my, C feq[Q21]) {
    const C ux = mx * inv_rho, uy = my * inv_rho;
    const C u2 = C(0.75) * (ux * ux + uy * uy);
#pragma unroll
    for (int q = 0; q < Q21; ++q) {
        const C r = C(kW21[q]) * rho;
        const C cu = C(kCx21[q]) * ux + C(kCy21[q]) * uy;
        const C a = r * (C(1.125) * cu * cu - u2);
        const C b = mom21<C>(q) * (C(sgn(kCx21[q])) * mx + C(sgn(kCy21[q])) * my);
        feq[q] = r + (a + b);
    }
}

// The rest population closes the mass balance (the collision conserves mass
// exactly in real arithmetic).
template <class C> __device__ inline void close_mass21(C f[Q21], C rho) {
    f[0] = C(0);
    f[0] = rho - (density21<C>(f));
}

template <class C> using Node21 = NodeState<C>;

// Eq. M1 from differences of opposite populations (exact near rest).
template <class C> __device__ inline void momentum21(const C f[Q21], C &jx, C &jy) {
    const C d1 = f[1] - f[3], d2 = f[2] - f[4], d57 = f[5] - f[7], d68 = f[6] - f[8];
    const C d9 = f[9] - f[11], d10 = f[10] - f[12], d13 = f[13] - f[15], d14 = f[14] - f[16];
    const C d17 = f[17] - f[19], d18 = f[18] - f[20];
    jx = ((d1 + (d57 - d68)) + C(2) * (d9 + (d13 - d14))) + C(3) * d17;
    jy = ((d2 + (d57 + d68)) + C(2) * (d10 + (d13 + d14))) + C(3) * d18;
}

// Forces of one node (eqs. force_SC, force_SC_FS, wall_shift) given its
// moments and the neighbour sums sx, sy = sum_i w_i psi(x + c_i) c_i.
template <class C>
__device__ inline Node21<C> node21(C rho, C jx, C jy, C psi_c, C sx, C sy, C phie, C Sx, C Sy,
                                   const LatDev<C> &L) {
    Node21<C> s;
    s.rho = rho;
    s.inv_rho = recip<C>(rho);
    s.jx = jx;
    s.jy = jy;
    s.ux = jx * s.inv_rho;
    s.uy = jy * s.inv_rho;
    s.jxd = double(jx);
    s.jyd = double(jy);
    momentum_after_force<C>(s, psi_c, sx, sy, phie, Sx, Sy, L.G, L.Ux, L.Uy, L.Fx, L.Fy);
    return s;
}

// EDM-BGK collision (Sec. II.B): f' = (1 - 1/tau)(f - feq(u)) + feq(u*).
// ONE: tau = 1, where f' = feq(u*) needs only the node's moments.
template <class C, int ONE> __device__ inline void collide21(C f[Q21], const Node21<C> &s, C omega, int projected) {
    C fs[Q21];
    equilibrium21<C>(s.rho, s.inv_rho, s.jsx, s.jsy, fs);
    if constexpr (ONE) {
#pragma unroll
        for (int i = 0; i < Q21; ++i) f[i] = fs[i];
    } else {
        C fu[Q21];
        equilibrium21<C>(s.rho, s.inv_rho, s.jx, s.jy, fu);
        const C keep = C(1) - omega;
#pragma unroll
        for (int i = 0; i < Q21; ++i) fu[i] = f[i] - fu[i];
        if (projected) project_neq<C, VelSet<21>>(fu);
#pragma unroll
        for (int i = 0; i < Q21; ++i) f[i] = keep * fu[i] + fs[i];
    }
    close_mass21<C>(f, s.rho);
}

// sum_i w_i psi(x + c_i) c_i over the 20 moving directions, from differences
// across the node, which vanish exactly where psi is uniform; ps(c_x, c_y)
// returns psi(x + c).  Both step kernels take this one order of operations.
template <class C, class Ps> __device__ inline void psi_sum21(const Ps &ps, C &sx, C &sy) {
    const C x1 = ps(1, 0) - ps(-1, 0), y1 = ps(0, 1) - ps(0, -1);
    const C a1 = ps(1, 1) - ps(-1, -1), b1 = ps(1, -1) - ps(-1, 1);
    const C x2 = ps(2, 0) - ps(-2, 0), y2 = ps(0, 2) - ps(0, -2);
    const C a2 = ps(2, 2) - ps(-2, -2), b2 = ps(2, -2) - ps(-2, 2);
    const C x3 = ps(3, 0) - ps(-3, 0), y3 = ps(0, 3) - ps(0, -3);
    sx = (((C(kW21[1]) * x1 + C(kW21[5]) * (a1 + b1)) + C(2 * kW21[9]) * x2) + C(2 * kW21[13]) * (a2 + b2)) +
         C(3 * kW21[17]) * x3;
    sy = (((C(kW21[2]) * y1 + C(kW21[5]) * (a1 - b1)) + C(2 * kW21[10]) * y2) + C(2 * kW21[13]) * (a2 - b2)) +
         C(3 * kW21[18]) * y3;
}

template <class S, class C, int WALL, int PSI, int DIAG, int ONE, int R>
__global__ __launch_bounds__(kQ21Waves * kWave) void k_tile_q21(LatDev<C> L, const void *__restrict__ src,
                                                                void *__restrict__ dst, int write_mom, int compare,
                                                                int update) {
    // the diagnostic partials are sized for the default tiling
    static_assert(!DIAG || R == kQ21Rows, "diagnostic pass uses kQ21Rows rows per wave");
    using Raw = typename Codec<S>::Raw;
    constexpr int ROWS = kQ21Waves * R;
    constexpr uint32_t OUT = uint32_t(ROWS - 2 * kH);
    __shared__ C psi_s[ROWS][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    const uint32_t nx = L.nx, ny = L.ny, P = L.pstride;
    const uint32_t strips = (nx + kQ21OutCols - 1) / kQ21OutCols;
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint32_t trow = lb / strips, strip = lb - trow * strips;
    const uint32_t x0 = strip * kQ21OutCols;                     // first output column (lane 3)
    const uint32_t x = wrap_fast(x0 + uint32_t(lane) + 3 * nx - kH, nx);
    const bool active = lane >= kH && lane < kWave - kH && x0 + uint32_t(lane) - kH < nx;
    const uint32_t y0 = trow * OUT;
    const uint32_t out_rows = min(OUT, ny - y0);

    PopBuf<S> buf;
    buf.init(src, 21u * P * uint32_t(sizeof(S)));
    // column of the pulled population with c_x = c: x - c (wrapped)
    uint32_t xs[2 * kH + 1];
#pragma unroll
    for (int c = -kH; c <= kH; ++c) xs[c + kH] = wrap_fast(x + 3 * nx - uint32_t(c + kH) + kH, nx);

    // Populations stay in registers across the barrier only where the
    // collision needs them (tau != 1); otherwise each row keeps its moments.
    constexpr bool KEEP = !DIAG && !ONE;
    C fk[KEEP ? R : 1][Q21], rho[R], jx[R], jy[R], psi[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t k = uint32_t(w * R + j);
        C *g = fk[KEEP ? j : 0];
        rho[j] = C(0);
        jx[j] = C(0);
        jy[j] = C(0);
        psi[j] = C(0);
        if (k < out_rows + 2 * kH) {
            const uint32_t r = wrap_fast(y0 + 3 * ny - kH + k, ny);
            uint32_t ro[2 * kH + 1];       // element offset of row r - c_y, c_y = -3..3
#pragma unroll
            for (int c = -kH; c <= kH; ++c) ro[c + kH] = wrap_fast(r + 3 * ny - uint32_t(c + kH) + kH, ny) * nx;
            Raw raw[Q21];
#pragma unroll
            for (int q = 0; q < Q21; ++q) raw[q] = buf.load(xs[kCx21[q] + kH], uint32_t(q) * P + ro[kCy21[q] + kH]);
#pragma unroll
            for (int q = 0; q < Q21; ++q) g[q] = Codec<S>::template decode<C>(raw[q], q, L.rho_ref);
            rho[j] = density21<C>(g);
            momentum21<C>(g, jx[j], jy[j]);
            psi[j] = psi21<C, PSI>(L, rho[j]);
            psi_s[k][lane] = psi[j];
        }
    }
    __syncthreads();

    // neighbour reads of the halo lanes stay inside the tile (their results
    // are not used)
    const int lc = lane < kH ? kH : (lane >= kWave - kH ? kWave - kH - 1 : lane);
    PopBuf<S> out;
    out.init(dst, 21u * P * uint32_t(sizeof(S)));
    double s_rho = 0, s_jx = 0, s_jy = 0, s_du = 0, s_u = 0, s_bad = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t k = uint32_t(w * R + j);
        if (k < uint32_t(kH) || k >= out_rows + kH) continue;
        const uint32_t r = wrap_fast(y0 + 3 * ny - kH + k, ny);
        C sx, sy;
        psi_sum21<C>([&](int cx, int cy) { return psi_s[int(k) + cy][lc + cx]; }, sx, sy);
        const uint32_t n = r * nx + x;
        C phie, Sx, Sy;
        wall_terms<C, WALL>(L, row_wall<C, WALL>(L, r), n, phie, Sx, Sy);
        const Node21<C> s = node21<C>(rho[j], jx[j], jy[j], psi[j], sx, sy, phie, Sx, Sy, L);
        if constexpr (DIAG) {
            const C vx = s.ux + C(0.5) * s.Fx * s.inv_rho;
            const C vy = s.uy + C(0.5) * s.Fy * s.inv_rho;
            if (active) {
                if (write_mom) {
                    L.mom[n] = rho[j];
                    L.mom[L.plane + n] = vx;
                    L.mom[2 * L.plane + n] = vy;
                }
                const bool ok = isfinite(double(rho[j])) && isfinite(double(vx)) && isfinite(double(vy));
                s_bad += ok ? 0.0 : 1.0;
                s_rho += double(rho[j]);
                s_jx += double(s.jx);
                s_jy += double(s.jy);
                if (compare)
                    s_du += fabs(double(vx) - double(L.uprev[n])) + fabs(double(vy) - double(L.uprev[L.plane + n]));
                s_u += fabs(double(vx)) + fabs(double(vy));
                if (update) {
                    L.uprev[n] = vx;
                    L.uprev[L.plane + n] = vy;
                }
            }
        } else {
            C *g = fk[KEEP ? j : 0];
            collide21<C, !KEEP>(g, s, L.omega, L.collision);
            if (active) {
                const uint32_t row = r * nx;
#pragma unroll
                for (int q = 0; q < Q21; ++q)
                    out.store(Codec<S>::template encode<C>(g[q], q, L.rho_ref), x, uint32_t(q) * P + row);
            }
        }
    }
    if constexpr (DIAG) {
        // wave sums, then the workgroup's sum over its waves in a fixed order:
        // one row of 8 partials per workgroup
        __shared__ double red[kQ21Waves][6];
        const double v[6] = {s_rho, s_jx, s_jy, s_du, s_u, s_bad};
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            double t = v[i];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, kWave);
            if (lane == 0) red[w][i] = t;
        }
        __syncthreads();
        if (threadIdx.x < 6) {
            double t = 0.0;
            for (int v2 = 0; v2 < kQ21Waves; ++v2) t += red[v2][threadIdx.x];
            L.partials[8 * size_t(lb) + threadIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// k_march_q21: the binary32 step on large lattices.  A workgroup of
// kMarchCols threads owns kMarchCols aligned columns (every lane an output, so
// every population row is stored as whole 256-byte rows) and marches down a
// segment of rows, one row per iteration: it loads the row 3 below the next
// output row (issuing the following row's loads first), forms density,
// momentum and pseudo-potential, keeps the pseudo-potential in an LDS ring of
// kRing rows and the moments in an LDS ring of 4 rows, and once the row 3 below
// an output row is in the ring forms that row's forces, collision and stores.
// At tau != 1 the collision also needs the output row's populations: they
// are loaded again (three iterations after their first load, from L2).
// The 3 columns left and right of the workgroup: threads 0..125 load one
// population of one of those 6 nodes each; the 6 densities are summed from LDS
// in the order of density21, so they equal the owning workgroup's bit for bit.
// Each segment reloads 6 rows; the tile kernel reloads 6 of every 32.
constexpr int kMarchCols = kQ21MarchCols, kRing = 8, kHaloNodes = 2 * kH;

// c_x + 3, c_y + 3 of D2Q21 velocity q packed 3 bits per q (lane-dependent q
// without a memory table)
constexpr uint64_t pack21(const int *c) {
    uint64_t v = 0;
    for (int q = 0; q < Q21; ++q) v |= uint64_t(c[q] + 3) << (3 * q);
    return v;
}
constexpr uint64_t kCx21Code = pack21(kCx21), kCy21Code = pack21(kCy21);
__device__ inline int cx21_dyn(int q) { return int((kCx21Code >> (3 * q)) & 7u) - 3; }
__device__ inline int cy21_dyn(int q) { return int((kCy21Code >> (3 * q)) & 7u) - 3; }

template <int WALL, int PSI, int ONE>
__global__ __launch_bounds__(kMarchCols) void k_march_q21(LatDev<float> L, const float *__restrict__ src,
                                                          float *__restrict__ dst, uint32_t seg_rows) {
    using C = float;
    __shared__ C psi_r[kRing][kMarchCols + 2 * kH];   // column offset c at index c + 3
    __shared__ C mom_r[4][3][kMarchCols];              // rho, j_x, j_y of rows waiting for output
    __shared__ C halo_raw[kHaloNodes][Q21];
    const uint32_t t = threadIdx.x;
    const uint32_t nx = L.nx, ny = L.ny, P = L.pstride;
    const uint32_t bxs = (nx + kMarchCols - 1) / kMarchCols;
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint32_t by = lb / bxs, bx = lb - by * bxs;
    const uint32_t x0 = bx * kMarchCols, y0 = by * seg_rows;
    const uint32_t out_rows = min(seg_rows, ny - y0);
    const uint32_t x = wrap_fast(x0 + t, nx);
    const bool active = x0 + t < nx;
    uint32_t xs[2 * kH + 1];                           // column of the pull with c_x = c: x - c
#pragma unroll
    for (int c = -kH; c <= kH; ++c) xs[c + kH] = wrap_fast(x + 3 * nx - uint32_t(c + kH) + kH, nx);
    // halo loader: node e (0..2 left of x0, 3..5 right of x0 + kMarchCols - 1), population hq
    const bool hl = t < uint32_t(kHaloNodes * Q21);
    const uint32_t he = hl ? t / Q21 : 0, hq = hl ? t - he * Q21 : 0;
    const uint32_t hcol = he < uint32_t(kH) ? wrap_fast(x0 + 3 * nx - kH + he, nx)
                                            : wrap_fast(x0 + kMarchCols + (he - kH), nx);
    const int hcx = cx21_dyn(int(hq)), hcy = cy21_dyn(int(hq));
    const uint32_t hx = wrap_fast(hcol + 3 * nx - uint32_t(hcx), nx);

    const uint32_t total = out_rows + 2 * kH;          // rows loaded: y0 - 3 .. y0 + out_rows + 2
    auto row_of = [&](uint32_t i) { return wrap_fast(y0 + 3 * ny - kH + i, ny); };
    auto load_row = [&](uint32_t r, C v[Q21]) {
        uint32_t ro[2 * kH + 1];
#pragma unroll
        for (int c = -kH; c <= kH; ++c) ro[c + kH] = wrap_fast(r + 3 * ny - uint32_t(c + kH) + kH, ny) * nx;
#pragma unroll
        for (int q = 0; q < Q21; ++q) v[q] = src[size_t(q) * P + ro[kCy21[q] + kH] + xs[kCx21[q] + kH]];
    };
    auto load_halo = [&](uint32_t r) -> C {
        if (!hl) return C(0);
        const uint32_t rr = wrap_fast(r + 3 * ny - uint32_t(hcy), ny);
        return src[size_t(hq) * P + rr * nx + hx];
    };
    C nxt[Q21];
    load_row(row_of(0), nxt);
    C hnxt = load_halo(row_of(0));
    for (uint32_t i = 0; i < total; ++i) {
        C g[Q21];
#pragma unroll
        for (int q = 0; q < Q21; ++q) g[q] = nxt[q];
        const C hcur = hnxt;
        if (i + 1 < total) {
            load_row(row_of(i + 1), nxt);
            hnxt = load_halo(row_of(i + 1));
        }
        const C rho = density21<C>(g);
        C jx, jy;
        momentum21<C>(g, jx, jy);
        const uint32_t slot = i % kRing;
        psi_r[slot][t + kH] = psi21<C, PSI>(L, rho);
        mom_r[i % 4][0][t] = rho;
        mom_r[i % 4][1][t] = jx;
        mom_r[i % 4][2][t] = jy;
        if (hl) halo_raw[he][hq] = hcur;
        __syncthreads();
        if (t < uint32_t(kHaloNodes)) {
            C h[Q21];
#pragma unroll
            for (int q = 0; q < Q21; ++q) h[q] = halo_raw[t][q];
            const C hp = psi21<C, PSI>(L, density21<C>(h));
            psi_r[slot][t < uint32_t(kH) ? t : kMarchCols + t] = hp;
        }
        __syncthreads();
        if (i >= uint32_t(2 * kH)) {
            const uint32_t o = i - 2 * kH, ci = i - kH;    // output row y0 + o, loaded as row ci
            const uint32_t y = y0 + o;
            auto ps = [&](int cx, int cy) { return psi_r[(ci + kRing + uint32_t(cy)) % kRing][int(t) + kH + cx]; };
            C sx, sy;
            psi_sum21<C>(ps, sx, sy);
            const uint32_t ms = ci % 4;
            const C r0 = mom_r[ms][0][t], jx0 = mom_r[ms][1][t], jy0 = mom_r[ms][2][t];
            const uint32_t n = y * nx + x;
            C phie, Sx, Sy;
            wall_terms<C, WALL>(L, row_wall<C, WALL>(L, y), n, phie, Sx, Sy);
            const Node21<C> st = node21<C>(r0, jx0, jy0, ps(0, 0), sx, sy, phie, Sx, Sy, L);
            C f[Q21];
            if constexpr (!ONE) load_row(row_of(ci), f);
            collide21<C, ONE>(f, st, L.omega, L.collision);
            if (active) {
#pragma unroll
                for (int q = 0; q < Q21; ++q) __builtin_nontemporal_store(f[q], dst + size_t(q) * P + n);
            }
        }
    }
}

// Calls fn(S{}, C{}) for the storage modes of D2Q21 (binary32, binary64).
template <class Fn> hipError_t dispatch21(int storage, Fn &&fn) {
    switch (storage) {
    case STORE_F32: return fn(float{}, float{});
    case STORE_F64: return fn(double{}, double{});
    default: return hipErrorInvalidValue;
    }
}

template <int DIAG, int R>
hipError_t launch_tile_q21(int storage, const LatDevAny &La, int wall, int parity, int write_mom, int compare,
                           int update, int psi_kind, hipStream_t st) {
    return dispatch21(storage, [&](auto s, auto c) {
        using S = decltype(s);
        using C = decltype(c);
        LatDev<C> d = La.get<C>();
        const void *src = parity ? d.fb : d.fa;
        void *dst = parity ? d.fa : d.fb;
        const dim3 grid(q21_tiles(d.nx, d.ny, R)), block(kQ21Waves * kWave);
        const bool one = DIAG || La.omega == 1.0;
        // One workgroup per CU: its loads in flight (16 waves x 2 rows x 21
        // planes x 256 B = 172 KB) from the 32 CUs of an XCD already exceed
        // that XCD's 4 MB L2; a second resident workgroup evicts the halo lines
        // neighbouring tiles share before they are read again (measured on the
        // 4096^2 binary32 step: 0.94 ms with two workgroups per CU, 0.77 ms with
        // one).  The unused dynamic LDS reservation is what caps residency.
        // One-row tiles (half the loads in flight) are left two per CU.
        const size_t lds_reserve = R == kQ21Rows ? kQ21LdsReserve : 0;
        auto go = [&](auto wallc, auto psic) {
            constexpr int WL = decltype(wallc)::value, PS = decltype(psic)::value;
            if (one)
                hipLaunchKernelGGL((k_tile_q21<S, C, WL, PS, DIAG, 1, R>), grid, block, lds_reserve, st, d, src, dst, write_mom,
                                   compare, update);
            else if constexpr (!DIAG)
                hipLaunchKernelGGL((k_tile_q21<S, C, WL, PS, 0, 0, R>), grid, block, lds_reserve, st, d, src, dst, write_mom,
                                   compare, update);
        };
        using RowW = std::integral_constant<int, WALL_ROW>;
        using NodeW = std::integral_constant<int, WALL_NODE>;
        using PsiExp = std::integral_constant<int, 0>;
        using PsiEos = std::integral_constant<int, 1>;
        if (wall == WALL_ROW) {
            if (psi_kind == 1) go(RowW{}, PsiEos{}); else go(RowW{}, PsiExp{});
        } else {
            if (psi_kind == 1) go(NodeW{}, PsiEos{}); else go(NodeW{}, PsiExp{});
        }
        return hipGetLastError();
    });
}

}  // namespace

hipError_t launch_step_q21(int storage, const LatDevAny &L, int wall, int parity, int variant, hipStream_t st) {
    if (variant == 0) return launch_tile_q21<0, kQ21Rows>(storage, L, wall, parity, 0, 0, 0, L.psi_kind, st);
    if (variant == 2) return launch_tile_q21<0, 1>(storage, L, wall, parity, 0, 0, 0, L.psi_kind, st);
    if (variant != 1) return hipErrorInvalidValue;
    if (!q21_march_ok(storage, L.omega)) return hipErrorInvalidValue;
    const LatDev<float> d = L.get<float>();
    const float *src = (const float *)(parity ? d.fb : d.fa);
    float *dst = (float *)(parity ? d.fa : d.fb);
    const dim3 grid(q21_march_blocks(d.nx, d.ny)), block(kMarchCols);
    auto go = [&](auto wallc, auto psic, auto onec) {
        constexpr int WL = decltype(wallc)::value, PS = decltype(psic)::value, ON = decltype(onec)::value;
        hipLaunchKernelGGL((k_march_q21<WL, PS, ON>), grid, block, 0, st, d, src, dst, kQ21MarchRows);
    };
    auto with_one = [&](auto wallc, auto psic) {
        if (L.omega == 1.0) go(wallc, psic, std::integral_constant<int, 1>{});
        else go(wallc, psic, std::integral_constant<int, 0>{});
    };
    auto with_psi = [&](auto wallc) {
        if (L.psi_kind == 1) with_one(wallc, std::integral_constant<int, 1>{});
        else with_one(wallc, std::integral_constant<int, 0>{});
    };
    if (wall == WALL_ROW) with_psi(std::integral_constant<int, WALL_ROW>{});
    else with_psi(std::integral_constant<int, WALL_NODE>{});
    return hipGetLastError();
}

hipError_t launch_diag_q21(int storage, const LatDevAny &L, int wall, int parity, int write_mom, int compare,
                           int update, hipStream_t st) {
    return launch_tile_q21<1, kQ21Rows>(storage, L, wall, parity, write_mom, compare, update, L.psi_kind, st);
}

}  // namespace lbmwet
