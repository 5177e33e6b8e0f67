// Device-side building blocks of the wetting-model lattice-Boltzmann step
// (arXiv:1202.6130, Sec. II) for gfx950.  Shared by every kernel of the
// library; nothing here is used by anything outside the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

// Build-time switches (defaults are the production choice).
#ifndef LBM_USE_BUFFER
#define LBM_USE_BUFFER 1   // buffer loads/stores: scalar row offsets, 32-bit lane offsets
#endif
#ifndef LBM_PREFETCH
#define LBM_PREFETCH 1     // issue the loads of row y+2 while row y is processed
#endif
#ifndef LBM_USE_DPP
#define LBM_USE_DPP 1      // x-neighbours through DPP wave shifts (else ds_bpermute)
#endif
#ifndef LBM_PSI_EXPM1
#define LBM_PSI_EXPM1 0    // psi = -expm1(-rho) instead of 1 - exp(-rho)
#endif
#ifndef LBM_PF_DEPTH
#define LBM_PF_DEPTH 1     // rows of loads in flight ahead of the row being consumed (1 or 2)
#endif
#ifndef LBM_STORE_AUX
#define LBM_STORE_AUX 2    // cache-policy bits of population stores (gfx950: 1 sc0, 2 nt, 16 sc1);
                           // non-temporal stores measured 3-4% faster for the tiled step
#endif
#ifndef LBM_LOAD_AUX
#define LBM_LOAD_AUX 0     // cache-policy bits of population loads
#endif

namespace lbmwet {

// D2Q9, velocity order (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
constexpr int Q = 9;
constexpr int kCx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double kW[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// D2Q21 (Tab. I), indices 0..8 as D2Q9, then |c| = 2 axes, (+-2,+-2), |c| = 3
// axes; theta = 2/3.
constexpr int Q21 = 21;
constexpr int kCx21[Q21] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2, 3, 0, -3, 0};
constexpr int kCy21[Q21] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2, 0, 3, 0, -3};
constexpr double kW21[Q21] = {91.0 / 324.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0,
                              2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
                              7.0 / 360.0, 7.0 / 360.0, 7.0 / 360.0, 7.0 / 360.0,
                              1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
                              1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0};

// Velocity set by population count (set-up and copy kernels; the hot kernels
// unroll their loops over constant tables).
template <int LQ> struct VelSet;
template <> struct VelSet<9> {
    static constexpr int Q = 9;
    static constexpr double theta = 1.0 / 3.0;
    __device__ static inline int cx(int q) { return kCx[q]; }
    __device__ static inline int cy(int q) { return kCy[q]; }
    __device__ static inline double w(int q) { return kW[q]; }
    __host__ __device__ static constexpr int cxc(int q) { return kCx[q]; }
    __host__ __device__ static constexpr int cyc(int q) { return kCy[q]; }
    __host__ __device__ static constexpr double wc(int q) { return kW[q]; }
};
template <> struct VelSet<21> {
    static constexpr int Q = 21;
    static constexpr double theta = 2.0 / 3.0;
    __device__ static inline int cx(int q) { return kCx21[q]; }
    __device__ static inline int cy(int q) { return kCy21[q]; }
    __device__ static inline double w(int q) { return kW21[q]; }
    __host__ __device__ static constexpr int cxc(int q) { return kCx21[q]; }
    __host__ __device__ static constexpr int cyc(int q) { return kCy21[q]; }
    __host__ __device__ static constexpr double wc(int q) { return kW21[q]; }
};

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kStripCols = 64;     // output columns per wave (one per lane, 64-aligned)
constexpr int kBlockWaves = LBM_BLOCK_WAVES;   // waves per workgroup
constexpr int kBlockThreads = kWave * kBlockWaves;

enum WallMode : int { WALL_ROW = 0, WALL_NODE = 1 };

// ------------------------------------------------------------ storage codecs
// Raw is the register image of one stored population; decode/encode convert
// between it and the arithmetic type C.
template <class S> struct Codec;
// saturated(v, q, rho_ref): the decoded population v is the image of a value
// outside the encodable range (never for the floating-point storages, which
// keep non-finite values as they are).
template <> struct Codec<float> {
    using Raw = uint32_t;
    template <class C> __device__ static inline C decode(Raw r, int, C) { return C(__builtin_bit_cast(float, r)); }
    template <class C> __device__ static inline Raw encode(C v, int, C) { return __builtin_bit_cast(Raw, float(v)); }
    template <class C> __device__ static inline bool saturated(C, int, C) { return false; }
};
template <> struct Codec<double> {
    using Raw = uint64_t;
    template <class C> __device__ static inline C decode(Raw r, int, C) { return C(__builtin_bit_cast(double, r)); }
    template <class C> __device__ static inline Raw encode(C v, int, C) { return __builtin_bit_cast(Raw, double(v)); }
    template <class C> __device__ static inline bool saturated(C, int, C) { return false; }
};
// 16-bit storage of the deviation from the rest equilibrium, scaled by the
// weight: h_i = f_i / w_i - rho_ref  <=>  f_i = w_i (rho_ref + h_i), kept as a
// signed fixed-point number in units of 2^-12 (range [-8, 8): the first steps
// after a sharp initial interface reach |h| ~ 5).  Against IEEE binary16 of
// the same h (spacing 2^-11 for |h| in [0.5, 1), the deviations of both
// phases) it halves the spacing where the interface populations sit; on a
// phase-separating lattice it tracked the binary64 dynamics 2.5 times closer
// (fewer nodes on the wrong side of the iso density).
struct Dev16 {
    uint16_t bits;
};
template <> struct Codec<Dev16> {
    using Raw = uint16_t;
    static constexpr float kUnit = 0x1p-12f, kScale = 0x1p12f;
    __device__ static inline float w(int q) { return q == 0 ? 4.0f / 9.0f : (q < 5 ? 1.0f / 9.0f : 1.0f / 36.0f); }
    __device__ static inline float winv(int q) { return q == 0 ? 2.25f : (q < 5 ? 9.0f : 36.0f); }
    // f = w rho_ref + (w 2^-12) k for the stored integer k, one rounding.  The
    // decoded population is a rounded value: contracted into the sums that
    // consume it (density, momentum), it would round differently where it is
    // consumed from registers than where it went through memory, and the
    // kernels' updates would depend on their data paths.
    template <class C> __device__ static inline C decode(Raw r, int q, C rho_ref) {
#pragma clang fp contract(off)
        const float k = float(int(int16_t(r)));
        return C(__builtin_fmaf(k, w(q) * kUnit, w(q) * float(rho_ref)));
    }
    // k = round(f / w 2^12 - rho_ref 2^12), one rounding in the fma (the scaled
    // weights are exact), saturated to the int16 range (a NaN goes to one of
    // the two bounds, by the maximum/minimum rules for NaN operands), then
    // rounded to the nearest integer (ties to even) by adding 1.5 * 2^23: the
    // sum's mantissa holds 2^22 + k, so its low 16 bits are k in two's
    // complement.
    template <class C> __device__ static inline Raw encode(C v, int q, C rho_ref) {
#pragma clang fp contract(off)
        const float x = __builtin_fmaf(float(v), winv(q) * kScale, -(float(rho_ref) * kScale));
        const float c = __builtin_fminf(__builtin_fmaxf(x, -32768.0f), 32767.0f) + 0x1.8p23f;
        return Raw(__builtin_bit_cast(uint32_t, c) & 0xffffu);
    }
    // A stored code at either bound (-32768, 32767) is a value that did not
    // fit: the diagnostic pass counts such nodes as unstable, as it counts
    // non-finite ones in the floating-point storages.
    template <class C> __device__ static inline bool saturated(C v, int q, C rho_ref) {
        return v == decode<C>(Raw(0x8000u), q, rho_ref) || v == decode<C>(Raw(0x7fffu), q, rho_ref);
    }
};

// ------------------------------------------------------------ memory access
// A population buffer [9][ny][nx] of S.  Element offsets are 32-bit; buffer
// byte sizes are < 4 GiB (checked by the host).
template <class S> struct PopBuf {
    using Raw = typename Codec<S>::Raw;
#if LBM_USE_BUFFER
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ inline void init(const void *p, uint32_t bytes) {
        // gfx9 raw buffer: stride 0, num_records in bytes, dword3 = 0x00020000
        rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
    }
    // lane offset in elements (varies per lane), uniform offset in elements
    __device__ inline Raw load(uint32_t lane_el, uint32_t uni_el) const {
        const int vo = int(lane_el * sizeof(S)), so = int(uni_el * sizeof(S));
        if constexpr (sizeof(S) == 4) return __builtin_amdgcn_raw_buffer_load_b32(rsrc, vo, so, LBM_LOAD_AUX);
        else if constexpr (sizeof(S) == 2) return __builtin_amdgcn_raw_buffer_load_b16(rsrc, vo, so, LBM_LOAD_AUX);
        else return __builtin_bit_cast(Raw, __builtin_amdgcn_raw_buffer_load_b64(rsrc, vo, so, LBM_LOAD_AUX));
    }
    __device__ inline void store(Raw v, uint32_t lane_el, uint32_t uni_el) const {
        const int vo = int(lane_el * sizeof(S)), so = int(uni_el * sizeof(S));
        if constexpr (sizeof(S) == 4) __builtin_amdgcn_raw_buffer_store_b32(v, rsrc, vo, so, LBM_STORE_AUX);
        else if constexpr (sizeof(S) == 2) __builtin_amdgcn_raw_buffer_store_b16(v, rsrc, vo, so, LBM_STORE_AUX);
        else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(rsrc, 0, 0, 0)), v), rsrc, vo, so, LBM_STORE_AUX);
    }
#else
    Raw *base;
    __device__ inline void init(const void *p, uint32_t) { base = (Raw *)p; }
    __device__ inline Raw load(uint32_t lane_el, uint32_t uni_el) const { return base[uni_el + lane_el]; }
    __device__ inline void store(Raw v, uint32_t lane_el, uint32_t uni_el) const { base[uni_el + lane_el] = v; }
#endif
};

// Wrapped neighbour column/row indices.
__device__ inline uint32_t wrap_dec(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }
__device__ inline uint32_t wrap_inc(uint32_t v, uint32_t n) { return v + 1 == n ? 0 : v + 1; }
// v mod n by repeated subtraction: the arguments here exceed n by less than
// one tile width, so this is one or two compares except on lattices narrower
// than a tile (an integer division would cost ~25 instructions before the
// first load of every wave).
__device__ inline uint32_t wrap_fast(uint32_t v, uint32_t n) {
    while (v >= n) v -= n;
    return v;
}

// c_x, c_y of a velocity index that differs between lanes, from packed 2-bit
// codes (c + 1): a lane-indexed constant table would be read from memory, and
// that read would stall every wave before its first population load.
__host__ __device__ constexpr int cx_dyn(int q) { return int((0x20919u >> (2 * q)) & 3u) - 1; }
__host__ __device__ constexpr int cy_dyn(int q) { return int((0x2865u >> (2 * q)) & 3u) - 1; }
constexpr bool velocity_codes_ok() {
    for (int q = 0; q < Q; ++q)
        if (cx_dyn(q) != kCx[q] || cy_dyn(q) != kCy[q]) return false;
    return true;
}
static_assert(velocity_codes_ok(), "packed velocity codes disagree with kCx/kCy");

// Logical workgroup index.  Consecutive hardware workgroups are dealt round
// robin to the 8 XCDs, each with its own L2.
//   LBM_XCD_REMAP 0: plain order: all XCDs work on one narrow band of
//                    logical workgroups at a time;
//   LBM_XCD_REMAP 1: each XCD owns one contiguous range (far-apart bands);
//   LBM_XCD_REMAP 2: plain order in chunks of 8 * LBM_XCD_GROUP, within which
//                    each XCD takes LBM_XCD_GROUP consecutive workgroups
//                    (neighbouring tiles share halo lines in one L2 while the
//                    whole chip still sweeps one band).
// Measured on MI355X (4096^2 step): mapping 2 is 2-3% faster than 0, and 1 is
// slower than both.
__device__ inline uint32_t xcd_logical_block(uint32_t b, uint32_t nb) {
    constexpr uint32_t nxcd = 8;
#if LBM_XCD_REMAP == 1
    uint32_t xcd = b % nxcd, local = b / nxcd;
    uint32_t base = xcd * (nb / nxcd) + min(xcd, nb % nxcd);
    return base + local;
#elif LBM_XCD_REMAP == 2
    constexpr uint32_t G = LBM_XCD_GROUP, chunk = nxcd * G;
    const uint32_t full = nb - nb % chunk;      // the ragged last chunk keeps the plain order
    if (b >= full) return b;
    const uint32_t xcd = b % nxcd, i = b / nxcd;
    return (i / G) * chunk + xcd * G + i % G;
#else
    (void)nb;
    return b;
#endif
}

// Fused multiply-add, written out where the update wants one.  The update's
// device functions below switch contraction off and fuse only here, so that
// every kernel that inlines them rounds them the same way (HIP otherwise
// fuses a multiply and an add across statements after inlining, and kernels
// sharing a function then disagreed in the last place where their
// surroundings differed).
__device__ inline float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class C> __device__ inline C cexp(C v);
template <> __device__ inline float cexp<float>(float v) { return __expf(v); }
template <> __device__ inline double cexp<double>(double v) { return exp(v); }

// Cross-lane neighbours along x: from_left(v, e) gives lane l the value of
// lane l-1 and lane 0 the value e (the column left of the strip);
// from_right(v, e) gives lane l the value of lane l+1 and lane 63 the value e.
// DPP wave shifts keep the `old` operand in the lane that has no source.
__device__ inline int dpp_shr1(int old, int v) { return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xF, 0xF, false); }
__device__ inline int dpp_shl1(int old, int v) { return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xF, 0xF, false); }
// row_shr:n within 16-lane rows, zero where the source lane is outside the row
template <int N> __device__ inline int dpp_row_shr(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x110 + N, 0xF, 0xF, true);
}

template <class C> struct Lanes;
template <> struct Lanes<float> {
    static __device__ inline float left(float v, float e) {
        return __builtin_bit_cast(float, dpp_shr1(__builtin_bit_cast(int, e), __builtin_bit_cast(int, v)));
    }
    static __device__ inline float right(float v, float e) {
        return __builtin_bit_cast(float, dpp_shl1(__builtin_bit_cast(int, e), __builtin_bit_cast(int, v)));
    }
    template <int N> static __device__ inline float shr(float v) {
        return __builtin_bit_cast(float, dpp_row_shr<N>(__builtin_bit_cast(int, v)));
    }
    static __device__ inline float lane(float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    }
};
template <> struct Lanes<double> {
    static __device__ inline double left(double v, double e) {
        const int2 p = __builtin_bit_cast(int2, v), q = __builtin_bit_cast(int2, e);
        return __builtin_bit_cast(double, make_int2(dpp_shr1(q.x, p.x), dpp_shr1(q.y, p.y)));
    }
    static __device__ inline double right(double v, double e) {
        const int2 p = __builtin_bit_cast(int2, v), q = __builtin_bit_cast(int2, e);
        return __builtin_bit_cast(double, make_int2(dpp_shl1(q.x, p.x), dpp_shl1(q.y, p.y)));
    }
    template <int N> static __device__ inline double shr(double v) {
        const int2 p = __builtin_bit_cast(int2, v);
        return __builtin_bit_cast(double, make_int2(dpp_row_shr<N>(p.x), dpp_row_shr<N>(p.y)));
    }
    static __device__ inline double lane(double v, int l) {
        const int2 p = __builtin_bit_cast(int2, v);
        return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(p.x, l),
                                                     __builtin_amdgcn_readlane(p.y, l)));
    }
};

// Sum of lanes 16r .. 16r+8 of each 16-lane row r, left in lane 16r+15, when
// lanes 16r+9 .. 16r+15 hold zero.  The tree is ((v0+v1)+(v2+v3)) +
// ((v4+v5)+(v6+v7)) + v8 up to operand order, i.e. exactly density() below.
template <class C> __device__ inline C row_sum9(C v) {
    v = v + Lanes<C>::template shr<1>(v);
    v = v + Lanes<C>::template shr<2>(v);
    v = v + Lanes<C>::template shr<4>(v);
    v = v + Lanes<C>::template shr<8>(v);
    return v;
}

// Raw post-streaming populations of one row (pull: f_i(x) = f'_i(x - c_i)),
// plus the halo gather: lanes 0..8 load population q = lane of the node left
// of the strip, lanes 32..40 population q = lane - 32 of the node right of
// it; the other lanes load a harmless in-bounds word and later use zero.
template <class S> struct RowLoader {
    using Raw = typename Codec<S>::Raw;
    PopBuf<S> buf;
    uint32_t plane;
    uint32_t x, xm, xp;            // this lane's column and its wrapped neighbours
    uint32_t g_col;                // gather: q * plane + source column (elements)
    int g_cy;                      // gather: row shift of population q

    // rm/r0/rp: element offsets (row * nx) of rows r-1, r, r+1
    __device__ inline void load(uint32_t rm, uint32_t r0, uint32_t rp, Raw f[Q], Raw &g) const {
        f[0] = buf.load(x, 0 * plane + r0);
        f[1] = buf.load(xm, 1 * plane + r0);
        f[2] = buf.load(x, 2 * plane + rm);
        f[3] = buf.load(xp, 3 * plane + r0);
        f[4] = buf.load(x, 4 * plane + rp);
        f[5] = buf.load(xm, 5 * plane + rm);
        f[6] = buf.load(xp, 6 * plane + rm);
        f[7] = buf.load(xp, 7 * plane + rp);
        f[8] = buf.load(xm, 8 * plane + rp);
        const uint32_t rs = g_cy > 0 ? rm : (g_cy == 0 ? r0 : rp);
        g = buf.load(g_col + rs, 0);
    }
};

template <class S, class C>
__device__ inline void decode_row(const typename Codec<S>::Raw r[Q], C f[Q], C rho_ref) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = Codec<S>::template decode<C>(r[i], i, rho_ref);
}

// Eq. M0 in a fixed order that is mirror-symmetric in x and in y (the
// populations of each mirror pair are added first), so that a mirror-
// symmetric state keeps mirror-symmetric densities in binary32.  The halo
// gathers of the step kernels sum the same nine values in the same tree
// (gather_pop below).
template <class C> __device__ inline C density(const C f[Q]) {
    return (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]))) + f[0];
}

// Population fetched by gather slot k = 0..8 (lanes 0..8 and 32..40 of a
// halo gather): slots in the order of the tree of density(), so that
// row_sum9 over the slots reproduces density() bit for bit.
__host__ __device__ constexpr int gather_pop(int k) { return int((0x087654231ull >> (4 * k)) & 15u); }
constexpr bool gather_order_ok() {
    const int want[Q] = {1, 3, 2, 4, 5, 6, 7, 8, 0};
    for (int k = 0; k < Q; ++k)
        if (gather_pop(k) != want[k]) return false;
    return true;
}
static_assert(gather_order_ok(), "gather slots must follow the tree of density()");

// Neighbour sums of psi (eq. force_SC) at one node, from the 3 x 3 block of
// pseudo-potentials around it (p = this column, l = left, r = right; c = this
// row, n = the row above, s = the row below):
//   sx = sum_i w_i psi(x + c_i) c_ix = w1 (r_c - l_c) + w2 ((r_n - l_n) + (r_s - l_s))
//   sy = sum_i w_i psi(x + c_i) c_iy = w1 (p_n - p_s) + w2 ((r_n - r_s) + (l_n - l_s))
// Differences across the node come first: they are exact for nearby values
// and exactly zero where psi is uniform, and the sums carry no cancellation.
// (Grouped by column instead, w1 psi + w2 (psi_n + psi_s) on either side and
// their difference, binary32 rounding of the column sums acted as a force that
// repeated at a quasi-steady node in every step.)
template <class C>
__device__ inline void psi_sums(C pn, C ps, C lc, C ln, C ls, C rc, C rn, C rs, C &sx, C &sy) {
#pragma clang fp contract(off)
    const C w1 = C(1.0 / 9.0), w2 = C(1.0 / 36.0);
    sx = fmac(w1, rc - lc, w2 * ((rn - ln) + (rs - ls)));
    sy = fmac(w1, pn - ps, w2 * ((rn - rs) + (ln - ls)));
}

// Pseudo-potential of the fluid-fluid force.
template <class C> __device__ inline C psi_of(C rho) {
#if LBM_PSI_EXPM1
    return -expm1(rho * C(-1));
#else
    return C(1) - cexp<C>(-rho);
#endif
}

// Lattice constants in the arithmetic type.  In binary32 the rounded D2Q9
// weights sum to 1 + 2^-27 and the momentum coefficients 6 w1 + 12 w2 to
// 1 + 2^-27, so every collision would create mass and momentum at that rate.
// The binary32 set below keeps w0, w1 and 3 w1 = 1/3 at their nearest values
// and moves w2 and 3 w2 down by one unit in the last place: then
// w0 + 4 w1 + 4 w2 = 1 and 2 (3 w1) + 4 (3 w2) = 1 hold exactly.
template <class C> struct LatConst;
template <> struct LatConst<float> {
    static constexpr float w0 = 0x1.c71c72p-2f;   // 4/9
    static constexpr float w1 = 0x1.c71c72p-4f;   // 1/9
    static constexpr float w2 = 0x1.c71c70p-6f;   // 1/36, one ulp low
    static constexpr float m1 = 0x1.555556p-2f;   // 3 w1 = 1/3
    static constexpr float m2 = 0x1.555554p-4f;   // 3 w2 = 1/12, one ulp low
};
template <> struct LatConst<double> {
    static constexpr double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w2 = 1.0 / 36.0;
    static constexpr double m1 = 1.0 / 3.0, m2 = 1.0 / 12.0;
};

// 1/rho: the hardware reciprocal in binary32 (1 ulp; the momentum of the
// equilibrium does not go through it), a correctly rounded division in FP64.
template <class C> __device__ inline C recip(C v);
template <> __device__ inline float recip<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ inline double recip<double>(double v) { return 1.0 / v; }

// Everything the collision needs at one node.  jxd .. jsyd carry the
// momenta in binary64 (for binary64 arithmetic they equal the members of
// type C).
template <class C> struct NodeState {
    C rho, inv_rho;
    C jx, jy;                      // momentum j = sum_i f_i c_i (pre-force)
    C ux, uy;                      // u = j / rho
    C Fx, Fy;                      // total force density
    C jsx, jsy;                    // rho u* = j + F, rounded once
    double jxd, jyd, jsxd, jsyd;   // j and j + F in binary64
};

// rho u* = j + F with F = F_FF + F_LR + phi^eps [rho (U - u) - F_FF] + F_ext
// (eqs. force_SC, force_SC_FS, wall_shift), rearranged without cancellation
// as (1 - phi^eps)(j + F_FF) + phi^eps rho U + F_LR + F_ext and formed in
// binary64 whatever the storage: near a wall F_FF and F_LR reach 0.1-0.2
// while a driving force is ~1e-6, and binary32 sums of those terms lose the
// driving force to a rounding that repeats every step.  Reads s.rho, s.jxd,
// s.jyd; sets the rest.
template <class C>
__device__ inline void momentum_after_force(NodeState<C> &s, C psi_c, C sx, C sy, C phie, C Sx, C Sy, C G,
                                            C Ux, C Uy, C Fxe, C Fye) {
#pragma clang fp contract(off)
    const double r = double(s.rho), ph = double(phie), om = 1.0 - ph;
    const double gp = -double(G) * double(psi_c);
    const double jx = s.jxd, jy = s.jyd;
    // om (j + F_FF) + ((ph rho U + rho S) + F_ext), with j + F_FF = fma(gp, s, j)
    const double tx = fmac(r, double(Sx), ph * (r * double(Ux))) + double(Fxe);
    const double ty = fmac(r, double(Sy), ph * (r * double(Uy))) + double(Fye);
    const double jsx = fmac(om, fmac(gp, double(sx), jx), tx);
    const double jsy = fmac(om, fmac(gp, double(sy), jy), ty);
    s.jsxd = jsx;
    s.jsyd = jsy;
    s.jsx = C(jsx);
    s.jsy = C(jsy);
    s.Fx = C(jsx - jx);
    s.Fy = C(jsy - jy);
}

// Forces of one node (eqs. force_SC, force_SC_FS, wall_shift) given the
// neighbour sums of psi (psi_sums).  The momentum (eq. M1) is a sum of
// differences of opposite populations (exact near rest).
template <class C>
__device__ inline NodeState<C> node_forces(const C f[Q], C rho, C psi_c, C sx, C sy, C phie,
                                           C Sx, C Sy, C G, C Ux, C Uy, C Fxe, C Fye) {
#pragma clang fp contract(off)
    NodeState<C> s;
    s.rho = rho;
    s.inv_rho = recip<C>(rho);
    s.jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    s.jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    s.jxd = double(s.jx);
    s.jyd = double(s.jy);
    s.ux = s.jx * s.inv_rho;
    s.uy = s.jy * s.inv_rho;
    // long-range wall force rho S (S precomputed from the static psi_FS);
    // short-range exchange phi^eps [rho (U - u) - F_FF]
    momentum_after_force<C>(s, psi_c, sx, sy, phie, Sx, Sy, G, Ux, Uy, Fxe, Fye);
    return s;
}

// Second-order equilibrium (eq. f2 at equilibrium, theta = 1/3) from density
// and momentum m = rho u:
//   feq_i = w_i rho + w_i rho (4.5 (c_i.u)^2 - 1.5 u^2) + 3 w_i c_i.m .
// Opposite velocities share the even part and differ by the odd part, so
// sum_i feq_i c_i = m exactly in real arithmetic with the constants above.
// The small velocity terms are formed on their own and added to w_i rho
// last: folded into (1 - 1.5 u^2) first, they were rounded at the spacing of
// numbers near 1, the same way at a steady node in every step.
template <class C> __device__ inline void equilibrium(C rho, C inv_rho, C mx, C my, C feq[Q]) {
#pragma clang fp contract(off)
    using K = LatConst<C>;
    const C ux = mx * inv_rho, uy = my * inv_rho;
    const C u2 = C(1.5) * (ux * ux + uy * uy);
    const C r0 = K::w0 * rho, r1 = K::w1 * rho, r2 = K::w2 * rho;
    feq[0] = r0 - r0 * u2;
    const C ax = r1 * (C(4.5) * ux * ux - u2), bx = K::m1 * mx;
    feq[1] = r1 + (ax + bx);
    feq[3] = r1 + (ax - bx);
    const C ay = r1 * (C(4.5) * uy * uy - u2), by = K::m1 * my;
    feq[2] = r1 + (ay + by);
    feq[4] = r1 + (ay - by);
    const C s = ux + uy, d = uy - ux;
    const C as = r2 * (C(4.5) * s * s - u2), bs = K::m2 * (mx + my);
    feq[5] = r2 + (as + bs);
    feq[7] = r2 + (as - bs);
    const C ad = r2 * (C(4.5) * d * d - u2), bd = K::m2 * (my - mx);
    feq[6] = r2 + (ad + bd);
    feq[8] = r2 + (ad - bd);
}

// The moving populations of the equilibrium for binary32 arithmetic, in
// binary64 and not yet rounded: the rest part w_i rho and the momentum term
// 3 w_i c_i.m (m = j + F in binary64, never rounded to binary32) in binary64,
// the small second-order term in binary32; feq[0] is left to the mass
// closure.  Each outgoing population is then rounded once.  In binary32 the
// rounding of m and of the rest-plus-second-order part before the momentum
// term is added repeated identically at a quasi-steady node in every step
// and moved the interface of the 1024 x 512 sessile drop by ~1e-4 nodes.
__device__ inline void equilibrium_b32(float rho, float inv_rho, double mx, double my, double feq[Q]) {
#pragma clang fp contract(off)
    using K = LatConst<float>;
    const float ux = float(mx) * inv_rho, uy = float(my) * inv_rho;
    const float u2 = 1.5f * fmac(ux, ux, uy * uy);
    const float r1 = K::w1 * rho, r2 = K::w2 * rho;
    const double R1 = double(rho) * (1.0 / 9.0), R2 = double(rho) * (1.0 / 36.0);
    constexpr double k3 = 1.0 / 3.0, k12 = 1.0 / 12.0;
    // even part, then the momentum term fused in: ex +- m / 3 rounded once
    const double ex = R1 + double(r1 * fmac(4.5f * ux, ux, -u2));
    feq[1] = fmac(mx, k3, ex);
    feq[3] = fmac(-mx, k3, ex);
    const double ey = R1 + double(r1 * fmac(4.5f * uy, uy, -u2));
    feq[2] = fmac(my, k3, ey);
    feq[4] = fmac(-my, k3, ey);
    const float su = ux + uy, du = uy - ux;
    const double ms = mx + my, md = my - mx;
    const double es = R2 + double(r2 * fmac(4.5f * su, su, -u2));
    feq[5] = fmac(ms, k12, es);
    feq[7] = fmac(-ms, k12, es);
    const double ed = R2 + double(r2 * fmac(4.5f * du, du, -u2));
    feq[6] = fmac(md, k12, ed);
    feq[8] = fmac(-md, k12, ed);
    feq[0] = 0.0;
}

// The rest population closes the mass balance (the collision conserves mass
// exactly in real arithmetic).  Binary64: f'_0 = rho - sum_{i>0} f'_i.
// Binary32: f'_0 = f_0 + sum_{i>0} (f_i - f'_i) from the incoming populations
// fin: the eight differences are exact (nearby values) and small, so the
// stored populations of a node sum to its incoming mass up to the rounding
// of f'_0 alone.  A binary32 density in f'_0 = rho - ... rounds at the spacing
// of numbers near rho, the same way at a steady node in every step: such
// nodes created or destroyed mass at a fixed rate (on a 256 x 128 sessile
// drop after 20000 steps, 1.2e-4 of the density against 3e-6 with this
// closure).
template <class C> __device__ inline void close_mass(C f[Q], C rho, const C fin[Q]) {
#pragma clang fp contract(off)
    if constexpr (sizeof(C) == 4) {
        (void)rho;
        const C d = (((fin[1] - f[1]) + (fin[3] - f[3])) + ((fin[2] - f[2]) + (fin[4] - f[4]))) +
                    (((fin[5] - f[5]) + (fin[6] - f[6])) + ((fin[7] - f[7]) + (fin[8] - f[8])));
        f[0] = fin[0] + d;
    } else {
        (void)fin;
        f[0] = rho - (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8])));
    }
}

// EDM-BGK collision: f' = f - (f - feq(u))/tau + feq(u*) - feq(u)
//                       = (1 - 1/tau) (f - feq(u)) + feq(u*),
// with rho u* = j + F.
// The non-equilibrium part g = f - feq(u) reduced to its component in the
// truncated Hermite form of eq. f2 (the projection step of Sec. II.A applied
// to f; the equilibrium is already of that form): with Pi = sum_i g_i c_i c_i,
// g_i <- w_i (c_i c_i - theta I) : Pi / (2 theta^2).  Used by both lattices.
template <class C, class VS> __device__ inline void project_neq(C g[VS::Q]) {
#pragma clang fp contract(off)
    constexpr double th = VS::theta;
    C pxx = C(0), pxy = C(0), pyy = C(0);
#pragma unroll
    for (int i = 1; i < VS::Q; ++i) {
        const int cx = VS::cxc(i), cy = VS::cyc(i);
        if (cx != 0) pxx += C(cx * cx) * g[i];
        if (cx * cy != 0) pxy += C(cx * cy) * g[i];
        if (cy != 0) pyy += C(cy * cy) * g[i];
    }
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        const int cx = VS::cxc(i), cy = VS::cyc(i);
        const C k = C(VS::wc(i) / (2.0 * th * th));
        g[i] = k * ((C(cx * cx - th) * pxx + C(2 * cx * cy) * pxy) + C(cy * cy - th) * pyy);
    }
}

// ONE = 1: compiled for tau = 1 only (the caller guarantees omega == 1);
// ONE = 0: tau taken at run time, the same arithmetic at tau = 1.
template <class C, int ONE = 0>
__device__ inline void collide(C f[Q], const NodeState<C> &s, C omega, int projected) {
#pragma clang fp contract(off)
    if constexpr (sizeof(C) == 4) {
        C fin[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) fin[i] = f[i];
        double fs[Q];
        equilibrium_b32(s.rho, s.inv_rho, s.jsxd, s.jsyd, fs);
        if (ONE || omega == C(1)) {
            // tau = 1: the factor (1 - 1/tau) is exactly zero, f' = feq(u*)
#pragma unroll
            for (int i = 1; i < Q; ++i) f[i] = C(fs[i]);
        } else {
            // the non-equilibrium part in binary64 (the rest population's
            // is not needed: the projection's second moment has no c_0 term,
            // and f'_0 comes from the mass closure)
            double fu[Q];
            equilibrium_b32(s.rho, s.inv_rho, s.jxd, s.jyd, fu);
            const double keep = 1.0 - double(omega);
#pragma unroll
            for (int i = 1; i < Q; ++i) fu[i] = double(f[i]) - fu[i];
            if (projected) project_neq<double, VelSet<9>>(fu);
#pragma unroll
            for (int i = 1; i < Q; ++i) f[i] = C(fmac(keep, fu[i], fs[i]));
        }
        close_mass<C>(f, s.rho, fin);
    } else {
        C fs[Q];
        equilibrium<C>(s.rho, s.inv_rho, s.jsx, s.jsy, fs);
        if (ONE || omega == C(1)) {
#pragma unroll
            for (int i = 0; i < Q; ++i) f[i] = fs[i];
            close_mass<C>(f, s.rho, f);
            return;
        }
        C fu[Q];
        equilibrium<C>(s.rho, s.inv_rho, s.jx, s.jy, fu);
        const C keep = C(1) - omega;
#pragma unroll
        for (int i = 0; i < Q; ++i) fu[i] = f[i] - fu[i];
        if (projected) project_neq<C, VelSet<9>>(fu);
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = fmac(keep, fu[i], fs[i]);
        close_mass<C>(f, s.rho, f);
    }
}

// Wall terms of one row (WALL_ROW: per-row scalars) or node (WALL_NODE).
template <class C> struct RowWall {
    C phie, Sy;
};

template <class C, int WALL>
__device__ inline RowWall<C> row_wall(const LatDev<C> &L, uint32_t y) {
    RowWall<C> w{C(0), C(0)};
    if (WALL == WALL_ROW) {
        w.phie = L.row_tab[2 * y];
        w.Sy = L.row_tab[2 * y + 1];
    }
    return w;
}

template <class C, int WALL>
__device__ inline void wall_terms(const LatDev<C> &L, const RowWall<C> &rw, uint32_t n, C &phie, C &Sx, C &Sy) {
    if (WALL == WALL_ROW) {
        phie = rw.phie;
        Sx = C(0);
        Sy = rw.Sy;
    } else {
        phie = L.node_tab[n];
        Sx = L.node_tab[L.plane + n];
        Sy = L.node_tab[2 * L.plane + n];
    }
}

}  // namespace lbmwet
