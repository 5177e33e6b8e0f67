/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the wetting-model
 * lattice-Boltzmann update of Colosqui, Kavousanakis, Papathanasiou &
 * Kevrekidis, "A mesoscopic model for microscale hydrodynamics and interfacial
 * phenomena: slip, films, and contact angle hysteresis" (arXiv:1202.6130).
 *
 * One time step (Sec. II) at every node x of a periodic nx*ny D2Q9 lattice:
 *   rho = sum_i f_i,  j = sum_i f_i c_i,  u = j/rho           (eqs. M0, M1)
 *   psi = 1 - exp(-rho)                                       (pseudo-potential)
 *   F_FF = -G psi(x) sum_i w_i psi(x + c_i) c_i               (eq. force_SC)
 *   F_LR = rho(x) sum_i w_i [G_A psiA - G_R psiR](x + c_i) c_i (eq. force_SC_FS,
 *          eq. pseudopotential; repulsive core, attractive tail)
 *   dF_S = phi^eps [rho (U_wall - u) - F_FF]                  (eq. wall_shift)
 *   F = F_FF + F_LR + dF_S + F_ext,  u* = u + F/rho
 *   f'_i = f_i - (f_i - feq_i(rho,u))/tau + feq_i(rho,u*) - feq_i(rho,u)
 *          (eq. BE-BGK with the exact-difference force term of Sec. II.B;
 *           feq from eq. f2 at equilibrium, theta = 1/3)
 *   f_i(x + c_i, t+1) = f'_i(x, t)                            (streaming)
 * Velocity order i = 0..8: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 * (-1,-1) (1,-1); weights 4/9, 1/9 x4, 1/36 x4.
 *
 * Conventions for every entry point
 *  - Status: 0 = LBM_OK, negative = error.  The library never aborts and never
 *    throws across the ABI; lbm_last_error(ctx) returns the message of the
 *    last failed call on that context, lbm_last_error(NULL) the calling
 *    thread's last message (any call, with or without a context).
 *  - Host arrays are float64, row-major [ny][nx] (index y*nx + x), read or
 *    written during the call only and never retained.
 *  - Device memory: the caller owns one workspace (lbm_workspace_bytes) and
 *    lends it to the context; the library allocates no device memory of its
 *    own.  The workspace must stay valid until lbm_destroy.
 *  - Stream: every kernel and copy goes on the caller's hipStream_t (passed as
 *    void*; NULL = the default stream).  Calls marked "synchronises" block
 *    until the stream is idle; the others only enqueue work.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int lbm_status;
#define LBM_OK         0
#define LBM_EINVAL    (-1)  /* invalid argument or parameter                  */
#define LBM_ENOMEM    (-2)  /* workspace too small, or host allocation failed  */
#define LBM_EDEVICE   (-3)  /* a HIP runtime call or kernel launch failed     */
#define LBM_EUNSTABLE (-4)  /* non-finite density or velocity detected        */
#define LBM_ENOFIT    (-5)  /* contact angle: < 16 points or degenerate fit   */
#define LBM_ESTATE    (-6)  /* call not valid in the context's current state  */

/* Population storage in HBM and arithmetic type:
 *  F32     binary32 storage, FP32 arithmetic (72 B per lattice update)
 *  F16DEV  h_i = f_i / w_i - rho_ref in IEEE binary16, FP32 arithmetic (36 B)
 *  F64     binary64 storage, FP64 arithmetic (144 B)
 *  F32X    binary32 storage, FP64 arithmetic (72 B; rounding of the stored
 *          populations is the only FP32 error) */
#define LBM_STORE_F32    0
#define LBM_STORE_F16DEV 1
#define LBM_STORE_F64    2
#define LBM_STORE_F32X   3

/* Wall functions (Appendix A).
 *  NONE      : no solid anywhere (phi = psiR = psiA = 0).
 *  FLAT_SLAB : a solid band of slab_rows rows [ny - slab_rows, ny), faces on
 *              rows 0 and ny - slab_rows; with s the signed distance (nodes)
 *              to the nearest face (negative inside the band) and
 *              T(s; w) = (1 - tanh(s / w)) / 2:
 *              phi = T(s; wall_width), psiR = T(s; core_range),
 *              psiA = T(s; tail_range) - T(s; core_range).
 *  FIELDS    : per-node (phi, psiR, psiA) given by the caller at creation.
 *  MASK      : arbitrary geometry (Appendix A, eq. iteration): the caller
 *              gives two per-node indicators (0 or 1), the solid region H and
 *              the outer-boundary nodes B held at 1; at creation the library
 *              filters G^0 = H recursively, G^n = sum_i w_i G^(n-1)(x + c_i)
 *              with the lattice's own weights and B reset to 1 after each
 *              pass, and takes psiR = G^filter_core, phi = G^filter_wall,
 *              psiA = phi - psiR (the paper: 5 and 22). */
#define LBM_WALL_NONE      0
#define LBM_WALL_FLAT_SLAB 1
#define LBM_WALL_FIELDS    2
#define LBM_WALL_MASK      3

/* Velocity sets (Sec. II.A): D2Q9, and D2Q21 of Tab. I (theta = 2/3, each
 * node reaching three sites per step; storage F32 or F64, no batches). */
#define LBM_D2Q9  9
#define LBM_D2Q21 21

/* Pseudo-potential of the fluid-fluid force (eq. force_SC):
 *  EXP : psi = 1 - exp(-rho)                              (D2Q9 or D2Q21)
 *  EOS : psi = sqrt(2 (rho theta - p_EOS(rho)) / theta), p_EOS the
 *        piecewise-linear equation of state of eq. EOS with slopes
 *        eos[0..2] * theta (vapour, unstable, liquid) joined at rho_1 =
 *        eos[3] and rho_2 = eos[4]; the paper uses it with G = -1 (D2Q21
 *        only).  The 1/theta makes the bulk pressure equal p_EOS. */
#define LBM_PSI_EXP 0
#define LBM_PSI_EOS 1

/* Collision (Sec. II.A-B):
 *  BGK       : f' = (1 - 1/tau)(f - feq(u)) + feq(u*)   (EDM forcing)
 *  PROJECTED : the projection step the paper adds after eq. f2: f is first
 *              replaced by the truncated Hermite form of eq. f2 with its own
 *              M0, M1, M2, then BGK as above; equivalently the non-equilibrium
 *              part f - feq(u) is reduced to w_i (c_i c_i - theta I):Pi / (2
 *              theta^2), Pi its second moment.  Identical to BGK at tau = 1. */
#define LBM_COLL_BGK       0
#define LBM_COLL_PROJECTED 1

typedef struct {
    int32_t nx, ny;          /* lattice size, both >= 1; Q*nx*ny*(bytes per
                                stored population) < 2^32                    */
    int32_t storage;         /* LBM_STORE_*                                   */
    int32_t wall_kind;       /* LBM_WALL_*                                    */
    double tau;              /* relaxation time, > 0.5                        */
    double G;                /* fluid-fluid coupling (G < 0: cohesion)        */
    double G_R, G_A;         /* repulsive / attractive wall amplitudes        */
    double eps;              /* wall-probability exponent, >= 1               */
    double U_wall[2];        /* wall velocity                                 */
    double F_ext[2];         /* uniform external force density                */
    double wall_width;       /* FLAT_SLAB: phi width         (> 0, default 2) */
    double core_range;       /* FLAT_SLAB: psiR width        (> 0, default 1) */
    double tail_range;       /* FLAT_SLAB: psiA outer width  (> 0, default 3) */
    double rho_ref;          /* F16DEV reference density (> 0)                */
    int32_t slab_rows;       /* FLAT_SLAB: rows of solid, 1 <= P < ny         */
    int32_t diag_interval;   /* K: a diagnostic pass after every K-th step;
                                0 = only on request                          */
    int32_t seg_rows;        /* rows per wave segment of the diagnostic pass; 0 = library choice */
    int32_t lattice;         /* LBM_D2Q9 (default) or LBM_D2Q21               */
    int32_t psi_kind;        /* LBM_PSI_EXP (default) or LBM_PSI_EOS          */
    double eos[5];           /* eq. EOS: theta_V/theta, theta_U/theta,
                                theta_L/theta, rho_1, rho_2 (defaults: the
                                paper's 0.25, -0.25, 1, 0.222, 0.869)        */
    int32_t collision;       /* LBM_COLL_BGK (default) or LBM_COLL_PROJECTED  */
    int32_t filter_core;     /* MASK: passes for psiR, 0 <= . <= filter_wall (5) */
    int32_t filter_wall;     /* MASK: passes for phi, 1 <= . <= 1000       (22) */
    int32_t reserved;        /* must be 0                                     */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Fills *p with the defaults: tau = 1, G = -5, G_R = G_A = 0, eps = 1,
 * U_wall = F_ext = 0, wall_width = 2, core_range = 1, tail_range = 3,
 * rho_ref = 1, slab_rows = 8, storage F32, wall NONE, diag_interval 0,
 * lattice D2Q9, psi EXP, eos = the paper's parameters, collision BGK,
 * filter_core 5, filter_wall 22.
 * Paper: the model parameters of Sec. II (tau of eq. BE-BGK; G of
 * eq. force_SC; G_R, G_A, eps of eqs. pseudopotential and wall_shift; the
 * EOS of Sec. II.B; the filter passes 5 and 22 of Appendix A).  The numeric
 * defaults of the D2Q9 fluid are not the paper's (it uses D2Q21 with the
 * EOS pseudo-potential). */
lbm_status lbm_params_default(lbm_params *p);

/* Error message ("" if none; never NULL).  ctx != NULL: the message of the
 * last failed call on that context (kept until the next failure on it, valid
 * until lbm_destroy).  ctx == NULL: the calling thread's last message, for
 * calls that fail before a context exists (lbm_create, batch calls).
 * Paper: none (error reporting of the interface). */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Measurement utility, no lattice involved: copies `bytes` from device
 * memory src to device memory dst on `stream` (a hipStream_t, NULL for the
 * default stream) with 16-byte non-temporal loads and stores, as fast as a
 * plain copy runs on this GPU.  It is the bandwidth reference next to the
 * step kernels' HBM roofline (each of them reads and writes every stored
 * population once per step, as a copy does).  src, dst and bytes must be
 * multiples of 16 and the ranges must not overlap (else LBM_EINVAL); the
 * caller owns both buffers.  Asynchronous: returns after the launch.
 * Paper: none (a bandwidth reference for the measurements). */
lbm_status lbm_device_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Device bytes a context with these parameters needs (written to *bytes).
 * Paper: none (memory layout of this library). */
lbm_status lbm_workspace_bytes(const lbm_params *p, size_t *bytes);

/* Creates a context and sets f = feq(rho0, u0) at every node (post-streaming
 * populations at t = 0).
 *  rho0        host [ny][nx], required, every value > 0 and finite.
 *  u0          host [2][ny][nx] = (u_x, u_y), or NULL (fluid at rest).
 *  wall_fields host [3][ny][nx] = (phi, psiR, psiA) for LBM_WALL_FIELDS, or
 *              [2][ny][nx] = (solid H, held boundary B) for LBM_WALL_MASK;
 *              else must be NULL.  phi in [0, 1]; H, B in {0, 1}.
 *  workspace   device pointer, 256-byte aligned, >= lbm_workspace_bytes.
 *  stream      hipStream_t or NULL.
 * Synchronises.  On error *out is NULL and nothing is retained.
 * Paper: the lattice and parameters of Sec. II; the wall functions of
 * Appendix A (eq. iteration for MASK).  The initial state f = feq(rho0, u0)
 * (eq. f2 at equilibrium) is not in the paper. */
lbm_status lbm_create(const lbm_params *p, const double *rho0, const double *u0,
                      const double *wall_fields, void *workspace,
                      size_t workspace_bytes, void *stream, lbm_ctx **out);

/* Advances nsteps >= 0 time steps (the update above).  With diag_interval K
 * > 0, a diagnostic pass (totals, velocity residual against the previous pass,
 * non-finite count) runs after every step whose index is a multiple of K.
 * residual_out == NULL: enqueues only.
 * residual_out != NULL: synchronises after every diagnostic pass, returns
 * LBM_EUNSTABLE at the first pass that counts a non-finite density or
 * velocity (the steps after it are not taken), and writes the residual of
 * the latest pass (as out[4] of lbm_diagnostics) to *residual_out.  With
 * K = 0 a pass runs after the last step (unless that step already had one);
 * with K > 0 only the scheduled passes run, and *residual_out is +inf when
 * the lattice has had none yet.
 * Paper: Sec. II (streaming, eqs. force_SC, force_SC_FS, wall_shift,
 * BE-BGK with the exact difference method); the residual is not in the
 * paper (a steady-state criterion of this interface). */
lbm_status lbm_step(lbm_ctx *c, int64_t nsteps, double *residual_out);

/* Runs a diagnostic pass now (unless the last step already had one) and
 * returns, synchronising:
 *  out[0] step index t      out[1] sum rho       out[2] sum j_x
 *  out[3] sum j_y (j = pre-force momentum)
 *  out[4] residual r = sum|u(t) - u(t')| / sum|u(t)| over both components,
 *         t' = the previous pass (+inf if there was none), u = reported
 *         velocity (j + F/2)/rho
 *  out[5] number of nodes with non-finite rho or u
 * Returns LBM_EUNSTABLE if out[5] > 0.
 * Paper: eqs. M0 and M1 for the totals; the residual and the non-finite
 * count are not in the paper. */
lbm_status lbm_diagnostics(lbm_ctx *c, double out[6]);

/* lbm_diagnostics for callers that cannot allocate device memory or lend
 * scratch space (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the same pass, results and return codes, but its
 * per-wave partial sums go to one static device array of the library instead
 * of the context's workspace (the reported results still go to the
 * context).  The array holds LBM_NOALLOC_MAX_ROWS rows of 8 doubles (2 MiB);
 * every GPU the library runs on keeps its own copy until the process ends,
 * resolved on the first call on that GPU (the device current at lbm_create).
 * A lattice needing more rows (D2Q9: 64-column strips x segments of
 * seg_rows rows; D2Q21: one row per step tile) gives LBM_EINVAL.  The call
 * allocates nothing on the device or the host and synchronises.  Calls on
 * one GPU share the array: calls that overlap in time on one GPU (other
 * threads, other streams) race and must not be issued.  The array needs no
 * clearing: every pass writes each partial row it reads. */
#define LBM_NOALLOC_MAX_ROWS 32768
lbm_status lbm_diagnostics_noalloc(lbm_ctx *c, double out[6]);

/* Macroscopic fields at the current time (eqs. M0, M1): rho, and the reported
 * velocity u = (j + F/2)/rho (average of the pre- and post-force velocities
 * of the exact difference method).  Any output may be NULL; totals =
 * (sum rho, sum j_x, sum j_y), accumulated in FP64.  Synchronises.
 * Paper: eqs. M0, M1; the half-force velocity of the exact difference
 * method (Sec. II.B). */
lbm_status lbm_moments(lbm_ctx *c, double *rho, double *ux, double *uy,
                       double totals[3]);

/* Static contact angle (Sec. III.B): least-squares circle through the
 * rho = iso crossings on lattice edges (linear interpolation along the edge;
 * an edge counts when exactly one end has rho >= iso and both ends have
 * phi < 0.01, i.e. region III; horizontal edges wrap in x, vertical edges do
 * not wrap in y), algebraic start then Gauss-Newton on the geometric
 * distance; theta = acos(1 - h/R) with h = yc + R - y_ref.
 * out = (theta in degrees, R, xc, yc).  LBM_ENOFIT if fewer than 16 points or
 * the fit is degenerate.  Synchronises.
 * Paper: Sec. III.B (circle fit of the rho isoline, theta = acos(1 - h/R)). */
lbm_status lbm_contact_angle(lbm_ctx *c, double iso, double y_ref, double out[4]);

/* Dynamic contact angles of a moving drop (Sec. III.C): the rho = iso
 * crossings of region III (phi < 0.01, as lbm_contact_angle) are taken along
 * the periodic x about their circular mean (so a drop across x = 0 stays
 * whole); the highest crossing is the apex; one least-squares circle is
 * fitted to the crossings with x <= x_apex (rear) and one to those with
 * x >= x_apex (front), each needing >= 8 points.  U is the mass-weighted mean
 * u_x (reported velocity) of the liquid nodes (rho >= iso) of region III; the
 * advancing side is the one U points to (the front when U = 0).
 *  out[0] theta_A (degrees)   out[1] theta_R        out[2] U
 *  out[3] R of the advancing circle   out[4] R of the receding circle
 *  out[5] x_apex in [0, nx)   out[6] y_apex   out[7] mean rho of those liquid nodes
 * The capillary number of the paper is Ca = U mu_L / gamma with mu_L =
 * out[7] * theta * (tau - 1/2) and the caller's surface tension gamma.
 * Returns LBM_ENOFIT when a fit has too few points or degenerates.
 * Synchronises.
 * Paper: Sec. III.C (advancing and receding angles of a driven drop, two
 * circle fits, capillary number). */
lbm_status lbm_dynamic_angles(lbm_ctx *c, double iso, double y_ref, double out[8]);

/* Slip in a FLAT_SLAB channel (Sec. III.A): the x-averaged reported u_x(y)
 * over region-III rows of the gap [0, ny - slab_rows] is fitted by a parabola
 * and evaluated at the hydrodynamic boundary y_w, phi(y_w) = 0.01, of both
 * walls.  out = (b, u_s, c2): slip length u_s / |du/dy|(y_w), slip velocity
 * and the fit's second derivative.  LBM_EINVAL unless wall_kind is
 * FLAT_SLAB.  Synchronises.
 * Paper: Sec. III.A (slip against the Poiseuille profile, hydrodynamic
 * boundary where phi = 0.01). */
lbm_status lbm_slip_length(lbm_ctx *c, double out[3]);

/* Populations at the current time, post-streaming, as host float64
 * [Q][ny][nx] (Q = 9 or 21, velocity order of the oracle tables: D2Q9 as
 * above; D2Q21 continues with (2,0) (0,2) (-2,0) (0,-2), (2,2) (-2,2)
 * (-2,-2) (2,-2), (3,0) (0,3) (-3,0) (0,-3)).  Synchronises.
 * Paper: the populations f_i of Sec. II.A (velocity sets of Tab. I).  Reading
 * them out (checkpoints, fault injection) is not in the paper. */
lbm_status lbm_get_state(lbm_ctx *c, double *f);

/* Replaces the populations (same layout as lbm_get_state) and the step index;
 * forgets the previous diagnostic pass.  Values are rounded to the storage
 * type.  Synchronises.
 * Paper: the populations f_i of Sec. II.A; restoring them is not in the
 * paper. */
lbm_status lbm_set_state(lbm_ctx *c, const double *f, int64_t step_index);

/* Current step index (-1 for NULL).  Paper: the time t of Sec. II (dt = 1). */
int64_t lbm_step_index(const lbm_ctx *c);

/* Frees the host-side context; the workspace returns to the caller.  Waits
 * for the context's stream first.  NULL is accepted.  LBM_ESTATE while the
 * context is attached to a batch.  Paper: none (resource handling). */
lbm_status lbm_destroy(lbm_ctx *c);

/* ------------------------------------------------------------------------
 * Step tile shapes.  The time step runs as workgroups over blocks of
 * strips[s] adjacent 64-column strips; shape s has waves[s] wavefronts per
 * workgroup, waves[s]/strips[s] per strip, each loading rows[s] rows, and
 * updates waves[s]/strips[s]*rows[s] - 2 rows per workgroup (the first and
 * last loaded rows are halo).  Every shape computes bitwise the same update;
 * the choice only changes speed.  Shape 0 is the default of a new context.
 * ------------------------------------------------------------------------ */

/* Writes up to cap (waves, rows, strips) triples (any array may be NULL) and
 * returns the number of shapes.
 * Paper: none (execution layout of the step of Sec. II; no effect on results). */
int32_t lbm_tile_shapes(int32_t *waves, int32_t *rows, int32_t *strips, int32_t cap);

/* Sets / returns the tile shape of a context (not one inside a batch:
 * LBM_ESTATE).  lbm_get_tile_shape returns -1 for NULL.
 * D2Q21 contexts have three step variants instead, bitwise the same update:
 *  0  tiles of 16 waves x 2 rows (58 x 26 output nodes), any storage and tau;
 *  1  marching workgroups of 256 aligned columns over segments of 128 rows
 *     (F32 storage only, else LBM_EINVAL);
 *  2  tiles of 16 waves x 1 row (58 x 10 output nodes), any storage and tau.
 * A new D2Q21 context starts with 1 where it applies and the lattice holds at
 * least 256 such segments, else with 2.
 * Paper: none (execution layout of the step of Sec. II; no effect on results). */
lbm_status lbm_set_tile_shape(lbm_ctx *c, int32_t shape);
int32_t lbm_get_tile_shape(const lbm_ctx *c);

/* Two time steps per pass (temporal blocking; Sec. II.A streaming and the
 * collision of eq. BE-BGK applied twice).  With a variant v >= 0 set,
 * lbm_step advances D2Q9 lattices with F32, F16DEV or F64 storage two steps per
 * kernel launch: each workgroup reads a block of 64 * strips[v] columns x
 * rows[v] rows plus a halo of four nodes, computes the first step on the
 * block grown by two nodes with the populations kept in on-chip memory, and
 * writes the second step of the block.  The result equals two single steps
 * bit for bit (tile shapes do not matter); only the traffic to memory is
 * halved.  A single step is taken where one step is left, or where a
 * diagnostic pass (diag_interval) falls after the first step of a pair.
 * lbm_two_step_variants writes up to cap (strips, rows, waves per
 * workgroup) triples (any array may be NULL) and returns the number of
 * variants.  lbm_set_two_step(c, -1) returns to single steps (the default);
 * another lattice or storage gives LBM_EINVAL, a batch lattice LBM_ESTATE.
 * lbm_get_two_step returns the variant, -1 when off, -2 for NULL.
 * Paper: Sec. II.A (streaming) and eq. BE-BGK, applied twice per launch;
 * the temporal blocking itself is not in the paper. */
int32_t lbm_two_step_variants(int32_t *strips, int32_t *rows, int32_t *waves, int32_t cap);
lbm_status lbm_set_two_step(lbm_ctx *c, int32_t variant);
int32_t lbm_get_two_step(const lbm_ctx *c);

/* Autotuner for one lattice: for every shape runs one untimed step, then
 * three timed blocks of `steps` consecutive ordinary time steps (events
 * around each block), and keeps the shape of smallest median per-step time.
 * shape_out (nullable) gets the choice, ms_out (nullable, one entry per
 * shape) the medians.  The lattice advances by 3 * steps + 1 steps per
 * candidate.
 * The candidates are the lbm_tile_shapes(...) shapes, for D2Q21 the three
 * step variants above (ms_out gets INFINITY for variant 1 where it does not
 * apply).  Synchronises.
 * Paper: none (autotuning of the execution layout). */
lbm_status lbm_tune(lbm_ctx *c, int32_t steps, int32_t *shape_out, double *ms_out);

/* Autotuner between single steps (with the context's tile shape, so call
 * lbm_tune first) and the two-steps-per-pass variants: for every candidate
 * runs one untimed pair of steps, then three timed blocks of `steps` pairs,
 * and keeps the candidate of smallest median time per step (the variant, or
 * -1 for single steps; variant_out, nullable).  ms_out (nullable) gets
 * lbm_two_step_variants(...) + 1 entries: per-step medians of the variants,
 * then of single steps; INFINITY for variants that do not apply to the
 * lattice (then only single steps are timed).  The lattice advances by
 * 6 * steps + 2 steps per timed candidate.  Synchronises.
 * Paper: none (autotuning of the execution layout). */
lbm_status lbm_tune_two_step(lbm_ctx *c, int32_t steps, int32_t *variant_out, double *ms_out);

/* ------------------------------------------------------------------------
 * Batched ensembles: many independent lattices (each with its own size and
 * parameters, all F32 storage) advanced together, one kernel launch per time
 * step and tile shape in use, covering every lattice; the steps are replayed
 * from a HIP graph.  Each lattice follows exactly the single-lattice update
 * above, so a lattice gives bitwise the same fields alone and inside any
 * batch, whatever the tile shapes.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Device bytes for a batch of n lattices (written to *bytes).
 * Paper: none (memory layout of this library). */
lbm_status lbm_batch_workspace_bytes(const lbm_params *ps, int32_t n, size_t *bytes);

/* Creates a batch.  ps[k], rho0s[k], u0s[k] describe lattice k as in
 * lbm_create (wall kinds NONE or FLAT_SLAB; u0s may be NULL or hold NULL
 * entries, each else [2][ny][nx]).  seg_rows = rows per wave segment for
 * every lattice (0 = the library's choice).  Synchronises.
 * Paper: each lattice as lbm_create; batching is not in the paper. */
lbm_status lbm_batch_create(const lbm_params *ps, int32_t n,
                            const double *const *rho0s, const double *const *u0s,
                            int32_t seg_rows, void *workspace, size_t workspace_bytes,
                            void *stream, lbm_batch **out);

/* Advances every lattice of the batch by nsteps steps.  chunk > 0: the steps
 * are recorded once into a HIP graph of `chunk` steps (even) and replayed;
 * chunk = 0: plain launches.  Enqueues only.
 * Paper: Sec. II for each lattice; batching is not in the paper. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps, int32_t chunk);

/* Per-lattice diagnostics, as lbm_diagnostics, for every lattice: out[6*k ..]
 * (out[0] is that lattice's step index; the residual compares with the
 * lattice's previous diagnostic pass, +inf if it has none).  Synchronises.
 * Paper: eqs. M0, M1 per lattice; the residual is not in the paper. */
lbm_status lbm_batch_diagnostics(lbm_batch *b, double *out);

/* A context view of lattice k (valid until lbm_batch_destroy) for
 * lbm_moments / lbm_contact_angle / lbm_slip_length / lbm_get_state /
 * lbm_diagnostics.  lbm_step and lbm_set_state on a view return LBM_ESTATE;
 * lbm_destroy on a view is a no-op.
 * Paper: none (access to a lattice of a batch). */
lbm_ctx *lbm_batch_lattice(lbm_batch *b, int32_t k);

/* Device bytes of the tables for lbm_batch_attach over these contexts.
 * Paper: none (memory layout of this library). */
lbm_status lbm_batch_attach_bytes(lbm_ctx *const *ctxs, int32_t n, size_t *bytes);

/* Groups n existing contexts (from lbm_create: F32 storage, wall kind NONE or
 * FLAT_SLAB, all on `stream`) into a batch without touching their state:
 * lbm_batch_step then advances all of them by one launch per time step.  The
 * workspace (>= lbm_batch_attach_bytes) holds only the batch's tables; each
 * context keeps its own.  While attached, lbm_step, lbm_set_state and
 * lbm_destroy on a context return LBM_ESTATE; the read-out calls remain
 * valid.  This is the primitive of continuous batching: when membership
 * changes, destroy the batch and attach the new set.
 * Paper: Sec. II for each lattice; continuous batching is not in the paper. */
lbm_status lbm_batch_attach(lbm_ctx *const *ctxs, int32_t n, void *workspace,
                            size_t workspace_bytes, void *stream, lbm_batch **out);

/* Per-lattice tile shapes of a batch (shapes[k] for lattice k; NULL sets
 * shape 0 everywhere).  A batch starts with each context's own shape (0 for
 * lbm_batch_create).  Recorded graphs are dropped.  Synchronises.
 * Paper: none (execution layout; no effect on results). */
lbm_status lbm_batch_set_tile_shapes(lbm_batch *b, const int32_t *shapes);
lbm_status lbm_batch_get_tile_shapes(const lbm_batch *b, int32_t *shapes);

/* Autotuner for a batch.  Times every shape on the whole batch (median over
 * three blocks of `steps` consecutive steps, after one untimed step; each
 * candidate advances the batch by 3 steps + 1), derives a per-tile cost for
 * each shape, gives every lattice the shape of least predicted cost (its tile
 * count times that cost), times that mixed assignment too when it is not
 * uniform, and keeps the fastest candidate.  shapes_out (nullable, n entries)
 * gets the choice; ms_out (nullable, lbm_tile_shapes() + 1 entries) the
 * median step times of the uniform candidates and of the mixed one (NaN when
 * not timed).  The tuning steps are ordinary time steps.  Synchronises.
 * Paper: none (autotuning of the execution layout). */
lbm_status lbm_batch_tune(lbm_batch *b, int32_t steps, int32_t *shapes_out, double *ms_out);

/* Two time steps per launch for a whole batch (the single-lattice
 * lbm_set_two_step, applied to every lattice of the batch with one variant):
 * lbm_batch_step then advances every lattice two steps per launch (per graph
 * replay, chunk / 2 launches), single steps only for an odd remainder.
 * Bitwise the same fields as single steps.  -1 returns to single steps.
 * lbm_batch_get_two_step returns the variant, -1 when off, -2 for NULL.
 * lbm_batch_tune_two_step times single steps (with the batch's tile shapes)
 * and every variant on the whole batch (one untimed pair, then three timed
 * blocks of `steps` pairs each), keeps the fastest (variant_out, nullable)
 * and writes lbm_two_step_variants(...) + 1 per-step medians to ms_out
 * (nullable): the variants, then single steps.  Every lattice advances by
 * 6 * steps + 2 steps per candidate.  Synchronises.
 * Paper: Sec. II applied twice per launch; not in the paper as such. */
lbm_status lbm_batch_set_two_step(lbm_batch *b, int32_t variant);
int32_t lbm_batch_get_two_step(const lbm_batch *b);
lbm_status lbm_batch_tune_two_step(lbm_batch *b, int32_t steps, int32_t *variant_out, double *ms_out);

/* Frees the host-side batch (waits for its stream).  A batch from
 * lbm_batch_create frees its contexts; an attached batch hands its contexts
 * back with their state, step index and tile shape.  NULL is accepted.
 * Paper: none (resource handling). */
lbm_status lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
