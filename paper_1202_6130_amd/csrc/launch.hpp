// Host-visible launchers of the library's kernels (kernels.hip) and the plain
// descriptors they take.  Included by the C-ABI implementation (abi.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmwet {

// storage code -> (stored type, arithmetic type):
//   F32 (float, float), F16 (binary16 deviation, float), F64 (double, double),
//   F32X (float, double)
enum Storage : int { STORE_F32 = 0, STORE_F16 = 1, STORE_F64 = 2, STORE_F32X = 3 };

template <class C> struct LatDev;

// Type-erased lattice descriptor: float parameters kept in double and narrowed
// to the arithmetic type when a launcher builds the kernel argument.
struct LatDevAny {
    uint32_t nx = 0, ny = 0, plane = 0;
    uint32_t pstride = 0;          // population plane stride (elements), >= plane
    int lattice = 9;               // populations per node (9 or 21)
    int psi_kind = 0;              // 0: 1 - exp(-rho), 1: eq. EOS
    uint32_t strips = 0, segs = 0, seg_rows = 0;
    uint32_t wave0 = 0;
    void *fa = nullptr, *fb = nullptr;
    const void *row_tab = nullptr, *node_tab = nullptr;
    void *mom = nullptr;
    void *uprev = nullptr;
    double *partials = nullptr;
    double G = 0, omega = 1, Ux = 0, Uy = 0, Fx = 0, Fy = 0, rho_ref = 1;
    // equation-of-state pseudo-potential (eq. EOS) per branch b (vapour,
    // unstable, liquid): psi^2 = k_b (rho - rho_b) + a_b with rho_b = 0, r1, r2
    double eos_kV = 0, eos_kU = 0, eos_kL = 0, eos_aU = 0, eos_aL = 0, eos_r1 = 0, eos_r2 = 0;
    int collision = 0;             // 1: non-equilibrium part projected onto eq. f2

    template <class C> LatDev<C> get() const;
};

template <class C> struct LatDev {
    uint32_t nx, ny, plane;
    uint32_t strips, segs, seg_rows;
    uint32_t wave0;
    uint32_t pstride;              // population plane stride (elements)
    void *fa, *fb;
    const C *row_tab;
    const C *node_tab;
    C *mom;
    C *uprev;
    double *partials;
    C G, omega, Ux, Uy, Fx, Fy, rho_ref;
    C eos_kV, eos_kU, eos_kL, eos_aU, eos_aL, eos_r1, eos_r2;
    int collision;
};

template <class C> inline LatDev<C> LatDevAny::get() const {
    LatDev<C> d;
    d.nx = nx; d.ny = ny; d.plane = plane;
    d.strips = strips; d.segs = segs; d.seg_rows = seg_rows;
    d.wave0 = wave0; d.pstride = pstride;
    d.fa = fa; d.fb = fb;
    d.row_tab = (const C *)row_tab;
    d.node_tab = (const C *)node_tab;
    d.mom = (C *)mom;
    d.uprev = (C *)uprev;
    d.partials = partials;
    d.G = C(G); d.omega = C(omega); d.Ux = C(Ux); d.Uy = C(Uy);
    d.Fx = C(Fx); d.Fy = C(Fy); d.rho_ref = C(rho_ref);
    d.eos_kV = C(eos_kV); d.eos_kU = C(eos_kU); d.eos_kL = C(eos_kL);
    d.eos_aU = C(eos_aU); d.eos_aL = C(eos_aL); d.eos_r1 = C(eos_r1); d.eos_r2 = C(eos_r2);
    d.collision = collision;
    return d;
}

// Isoline passes over region III (phi < phi_max).  mode 0: (n, sum x,
// sum y); 1: algebraic circle sums about (mx, my); 2: Gauss-Newton normal
// equations of the geometric circle fit; 3: highest crossing per block;
// 4: liquid nodes (rho >= iso): (n, sum rho, sum rho u_x, sum rho u_y) with
// rho pointing at the moment planes; 5: (n, sum sin, sum cos) of 2 pi x / nx.
// side/xs keep one side of x = xs; unwrap/xmid take x periodic about xmid.
struct IsoParams {
    uint32_t nx, ny;
    int per_node, mode;
    double iso, phi_max, mx, my, xc, yc, R;
    int side = 0, unwrap = 0;
    double xs = 0, xmid = 0;
};

constexpr uint32_t kStripColsHost = 64;

#ifndef LBM_BLOCK_WAVES
#define LBM_BLOCK_WAVES 4   // waves per workgroup of the marching kernels
#endif
constexpr uint32_t kBlockWavesHost = LBM_BLOCK_WAVES;

#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 2     // workgroup-to-XCD mapping (see xcd_logical_block)
#endif
#ifndef LBM_XCD_GROUP
#define LBM_XCD_GROUP 8     // consecutive workgroups per XCD in mapping 2
#endif

// Step tile shapes.  A tile is a workgroup of kShapeWaves[s] wavefronts over
// kShapeStrips[s] adjacent 64-column strips; each wave loads kShapeRows[s]
// rows of one strip, and the tile updates all of them but the first and last
// (halo) rows: waves / strips * rows - 2 rows of 64 * strips columns.  Every
// shape computes bitwise the same update; they differ in halo overhead, edge
// waste on small lattices and occupancy, which is what the autotuner measures.
constexpr int kNumTileShapes = 9;
constexpr int kShapeWaves[kNumTileShapes] = {16, 8, 8, 16, 16, 8, 16, 16, 16};
constexpr int kShapeRows[kNumTileShapes] = {2, 2, 4, 3, 2, 4, 4, 4, 3};
constexpr int kShapeStrips[kNumTileShapes] = {1, 1, 1, 1, 2, 2, 2, 4, 2};
constexpr uint32_t shape_out_rows(int s) { return uint32_t(kShapeWaves[s] / kShapeStrips[s] * kShapeRows[s] - 2); }
constexpr uint32_t tile_groups(uint32_t nx, int s) {
    return ((nx + 63) / 64 + uint32_t(kShapeStrips[s]) - 1) / uint32_t(kShapeStrips[s]);
}
constexpr uint32_t tile_rows(uint32_t ny, int s) { return (ny + shape_out_rows(s) - 1) / shape_out_rows(s); }

uint32_t step_tiles(uint32_t nx, uint32_t ny, int shape);
hipError_t launch_step(int storage, const LatDevAny &L, int wall, int shape, int parity, hipStream_t st);
// Two time steps per pass (k_step_pass2, D2Q9, F32 and F16 storage): variant
// v updates blocks of 64 * kPass2Strips[v] columns x kPass2Rows[v] rows, one
// workgroup of kPass2Strips[v] * kPass2WavesPerStrip[v] waves each, with the
// populations between the two steps in LDS.  Bitwise two single steps.
constexpr int kPass2Variants = 9;
constexpr int kPass2Strips[kPass2Variants] = {1, 1, 2, 1, 1, 1, 1, 1, 1};
constexpr int kPass2Rows[kPass2Variants] = {8, 8, 8, 12, 12, 16, 16, 24, 24};
constexpr int kPass2WavesPerStrip[kPass2Variants] = {4, 8, 4, 6, 12, 8, 16, 8, 12};
inline bool pass2_ok(int storage) { return storage == STORE_F32 || storage == STORE_F16 || storage == STORE_F64; }
constexpr uint32_t pass2_blocks(uint32_t nx, uint32_t ny, int v) {
    return ((nx + 64u * uint32_t(kPass2Strips[v]) - 1) / (64u * uint32_t(kPass2Strips[v]))) *
           ((ny + uint32_t(kPass2Rows[v]) - 1) / uint32_t(kPass2Rows[v]));
}
hipError_t launch_step_pass2(int storage, const LatDevAny &L, int wall, int variant, int parity, hipStream_t st);
// The same over the blocks of many F32 flat-wall lattices: pwork[b] = (lattice,
// column group, row band) for variant `variant`.
hipError_t launch_step_pass2_batch(const void *lats, const uint4 *pwork, uint32_t nblocks, int variant, int parity,
                                   hipStream_t st);
hipError_t launch_step_batch(const void *lats, const uint4 *twork, uint32_t ntiles, int shape, int parity,
                             hipStream_t st);
hipError_t launch_diag(int storage, const void *lats, const uint4 *work, uint32_t nwork, const LatDevAny &single,
                       int wall, int parity, int write_mom, int compare, int update, hipStream_t st);
// Recursive-filter wall functions (Appendix A): fields[0..N) holds the solid
// indicator on entry; on return [phi | psiR | psiA] (3N doubles).  bnd: N
// doubles, nonzero on the nodes held at 1.
hipError_t launch_filter_walls(int lattice, uint32_t nx, uint32_t ny, double *fields, const double *bnd,
                               int n_core, int n_wall, hipStream_t st);
hipError_t launch_reduce(const double *part, const uint32_t *ranges, uint32_t nout, uint32_t stride,
                         uint32_t width, double *out, uint32_t out_stride, hipStream_t st);
hipError_t launch_isoline(int f64, const IsoParams &p, const void *rho, const double *phi, double *part,
                          hipStream_t st);
uint32_t isoline_blocks(uint32_t nodes);
hipError_t launch_profile(int f64, uint32_t nx, uint32_t ny, const void *ux, double *out, hipStream_t st);
hipError_t launch_init(int storage, int lattice, uint32_t nx, uint32_t ny, uint32_t pstride, const double *rho0,
                       const double *ux0, const double *uy0, void *dst, double rho_ref, hipStream_t st);
hipError_t launch_plane(int storage, int lattice, int set, uint32_t nx, uint32_t ny, uint32_t pstride, int q,
                        void *pop, double *buf, double rho_ref, hipStream_t st);
hipError_t launch_walls_row(int f64, int lattice, int ny, int P, double width, double core, double tail, double eps,
                            double GR, double GA, void *tab, double *phi_raw, hipStream_t st);
hipError_t launch_walls_node(int f64, int lattice, uint32_t nx, uint32_t ny, const double *fields, double eps,
                             double GR, double GA, void *tab, double *phi_raw, hipStream_t st);

// D2Q21 step (Tab. I): workgroups of kQ21Waves waves over strips of
// kQ21OutCols output columns (64 lanes with 3 halo columns on each side) and
// kQ21Waves * rows_per_wave loaded rows (3 halo rows above and below);
// kQ21Rows rows per wave unless stated.
constexpr int kQ21Waves = 16;
constexpr int kQ21Rows = 2;
constexpr uint32_t kQ21OutCols = 58;
inline uint32_t q21_strips(uint32_t nx) { return (nx + kQ21OutCols - 1) / kQ21OutCols; }
inline uint32_t q21_tiles(uint32_t nx, uint32_t ny, int rows_per_wave = kQ21Rows) {
    const uint32_t out_rows = uint32_t(kQ21Waves * rows_per_wave - 6);
    return q21_strips(nx) * ((ny + out_rows - 1) / out_rows);
}
// D2Q21 step variants: 0 tiles of kQ21Rows rows per wave (any storage), 1
// marching workgroups of kQ21MarchCols aligned columns over segments of
// kQ21MarchRows rows (binary32 storage only), 2 tiles of one row per wave (any
// storage; twice the workgroups of variant 0 on small lattices).
constexpr int kQ21Variants = 3;
constexpr uint32_t kQ21MarchCols = 256, kQ21MarchRows = 128;
constexpr uint32_t kQ21FillBlocks = 256;   // one workgroup per CU of the chip
inline bool q21_march_ok(int storage, double omega) { return storage == STORE_F32 && omega > 0.0; }
inline uint32_t q21_march_blocks(uint32_t nx, uint32_t ny) {
    return ((nx + kQ21MarchCols - 1) / kQ21MarchCols) * ((ny + kQ21MarchRows - 1) / kQ21MarchRows);
}
hipError_t launch_step_q21(int storage, const LatDevAny &L, int wall, int parity, int variant, hipStream_t st);
// The diagnostic pass of a D2Q21 lattice: one row of 8 partials per workgroup
// of the kQ21Rows tiling (q21_tiles rows).
hipError_t launch_diag_q21(int storage, const LatDevAny &L, int wall, int parity, int write_mom, int compare,
                           int update, hipStream_t st);

}  // namespace lbmwet
