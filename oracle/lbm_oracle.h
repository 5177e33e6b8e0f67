/*
 * Plain FP64 CPU oracle for the wetting-model lattice-Boltzmann update of
 * Colosqui, Kavousanakis, Papathanasiou & Kevrekidis, "A mesoscopic model for
 * microscale hydrodynamics and interfacial phenomena" (arXiv:1202.6130).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library.  It is
 * slow on purpose: straight loops, one formula per function, no blocking, no
 * fusion.  Nothing in the product path may link, load or call it; only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg do.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * State convention: f[(y*nx + x)*Q + i] holds the populations at time t after
 * streaming (i.e. just before the collision of step t).  Velocity sets
 * (Sec. II.A):
 *   D2Q9  (Q = 9):
 *     i : 0      1      2      3       4       5      6       7        8
 *     c : (0,0) (1,0)  (0,1)  (-1,0)  (0,-1)  (1,1)  (-1,1)  (-1,-1)  (1,-1)
 *     w : 4/9   1/9 x4                        1/36 x4
 *     theta = sum_i w_i c_ix^2 = 1/3
 *   D2Q21 (Q = 21, Tab. I), indices 0..8 as D2Q9, then
 *     9..12 (2,0) (0,2) (-2,0) (0,-2); 13..16 (2,2) (-2,2) (-2,-2) (2,-2);
 *     17..20 (3,0) (0,3) (-3,0) (0,-3);
 *     w : 91/324 (rest), 1/12 (|c|=1 axes), 2/27 ((+-1,+-1)), 7/360 (|c|=2
 *     axes), 1/432 ((+-2,+-2)), 1/1620 (|c|=3 axes); theta = 2/3
 * Fully periodic nx*ny.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny;
    double tau;        /* BGK relaxation time (Sec. II, eq. BE-BGK), > 0.5   */
    double G;          /* Shan-Chen coupling of the fluid-fluid force        */
    double G_R, G_A;   /* repulsive / attractive amplitudes (eq. pseudopotential) */
    double eps;        /* wall-probability exponent, >= 1 (eq. wall_shift)   */
    double U_wall[2];  /* wall velocity (eq. wall_shift)                     */
    double F_ext[2];   /* uniform external force density (Sec. III.A)        */
    int lattice;       /* 9 (D2Q9) or 21 (D2Q21, Tab. I); 0 reads as 9       */
    int psi_kind;      /* 0: psi = 1 - exp(-rho); 1: EOS, eq. EOS            */
    double eos[5];     /* EOS: theta_V/theta, theta_U/theta, theta_L/theta,
                          rho_1, rho_2 (eq. EOS)                              */
    int collision;     /* 0: BGK; 1: projection onto eq. f2 before BGK       */
} orc_params;

/* D2Q9 tables (the oracle's own copy). */
extern const int    ORC_CX[9];
extern const int    ORC_CY[9];
extern const double ORC_W[9];
extern const double ORC_THETA;

/* D2Q21 tables (Tab. I). */
extern const int    ORC21_CX[21];
extern const int    ORC21_CY[21];
extern const double ORC21_W[21];
extern const double ORC21_THETA;

/* Equilibrium of eq. f2 with M2 = rho u u + rho theta I (D2Q9). */
void orc_equilibrium(double rho, double ux, double uy, double feq[9]);

/* The same for a lattice (9 or 21); feq holds Q values. */
void orc_equilibrium_q(int lattice, double rho, double ux, double uy, double *feq);

/* Pseudo-potential of the fluid-fluid force at density rho:
 *   psi_kind 0: 1 - exp(-rho);
 *   psi_kind 1: sqrt(2 (rho theta - p_EOS(rho)) / theta) with the
 *   piecewise-linear p_EOS of eq. EOS (see the reading of the 1/theta factor
 *   in the source). */
double orc_psi(const orc_params *p, double rho);

/* Piecewise-linear equation of state p_EOS(rho) (eq. EOS). */
double orc_p_eos(const orc_params *p, double rho);

/* Flat-slab wall functions (Appendix A allows analytic profiles for flat
 * walls).  Solid band = rows [ny-P, ny); faces on rows 0 and ny-P.
 * phi = T(s;width), psiR = T(s;core), psiA = T(s;tail) - T(s;core), with
 * T(s;w) = (1 - tanh(s/w))/2 and s the signed distance to the nearest face. */
void orc_flat_slab_walls(int nx, int ny, int P, double width, double core,
                         double tail, double *phi, double *psiR, double *psiA);

/* f = f^eq(rho0, u0) at every node; u0 may be NULL (fluid at rest). */
void orc_init(const orc_params *p, const double *rho0, const double *ux0,
              const double *uy0, double *f);

/* Per-node quantities of one step, for inspection: rho, u (= j/rho), the
 * three force pieces and the shifted velocity.  Any output may be NULL. */
void orc_forces(const orc_params *p, const double *phi, const double *psiR,
                const double *psiA, const double *f, double *rho, double *ux,
                double *uy, double *Fff, double *Flr, double *dFs,
                double *Ftot, double *usx, double *usy);

/* Wall functions of arbitrary geometry by the recursive filter of Appendix A
 * (eq. iteration): solid and bnd are [ny*nx] indicators (0 or 1) of the solid
 * region and of its outer-boundary nodes, reset to 1 after every pass;
 * psiR = G^(n_core), phi = G^(n_wall), psiA = phi - psiR. */
void orc_filter_walls(int lattice, int nx, int ny, const double *solid, const double *bnd,
                      int n_core, int n_wall, double *phi, double *psiR, double *psiA);

/* Projection of one node's Q populations onto the truncated Hermite form of
 * eq. f2 with their own M0, M1, M2 (Sec. II.A). */
void orc_project_q(int lattice, const double *f, double *fp);

/* Collision at every node (no streaming): fpost = f - (f - feq(u))/tau
 * + feq(u*) - feq(u), with f first replaced by its projection when
 * p->collision == 1.  Exposed separately so the tests can check the
 * conservation laws of the collision alone. */
void orc_collide(const orc_params *p, const double *phi, const double *psiR,
                 const double *psiA, const double *f, double *fpost);

/* Streaming: fout_i(x + c_i) = fpost_i(x), periodic (D2Q9). */
void orc_stream(int nx, int ny, const double *fpost, double *fout);

/* The same for a lattice (9 or 21). */
void orc_stream_q(int lattice, int nx, int ny, const double *fpost, double *fout);

/* One full step (collide, then stream). f_in and f_out must differ. */
void orc_step(const orc_params *p, const double *phi, const double *psiR,
              const double *psiA, const double *f_in, double *f_out);

/* nsteps steps in place on f (allocates one scratch lattice). Returns 0, or
 * -1 when the scratch lattice cannot be allocated. */
int orc_run(const orc_params *p, const double *phi, const double *psiR,
            const double *psiA, double *f, long nsteps);

/* Reported macroscopic fields: rho, u_out = (j + F/2)/rho, and totals
 * (sum rho, sum j_x, sum j_y) with j the pre-force momentum. */
void orc_macros(const orc_params *p, const double *phi, const double *psiR,
                const double *psiA, const double *f, double *rho, double *ux,
                double *uy, double totals[3]);

/* Iso-density crossings on lattice edges, restricted to nodes whose phi is
 * below phi_max.  Writes up to cap points (px, py); returns the number found
 * (which may exceed cap: then only cap were written). */
long orc_isoline_points(int nx, int ny, const double *rho, const double *phi,
                        double iso, double phi_max, double *px, double *py,
                        long cap);

/* Least-squares circle through n points: algebraic (Kasa) start, then
 * Gauss-Newton on the geometric distance.  out = (xc, yc, R).  Returns 0 on
 * success, -1 if the fit is degenerate. */
int orc_circle_fit(long n, const double *px, const double *py, double out[3]);

/* Contact angle of a sessile drop (Sec. III.B): circle fit to the rho = iso
 * crossings in region III (phi < 0.01), theta = acos((y_ref - yc)/R).
 * out = (theta_deg, R, xc, yc).  Returns 0, or -1 if no fit (<16 points or
 * degenerate). */
int orc_contact_angle(const orc_params *p, const double *phi,
                      const double *psiR, const double *psiA, const double *f,
                      double iso, double y_ref, double out[4]);

/* Sec. III.C: out = (theta_A, theta_R [deg], U, R_A, R_R, x_apex, y_apex,
 * mean liquid rho); returns 0, or -1 if a fit is impossible. */
int orc_dynamic_angles(const orc_params *p, const double *phi, const double *psiR,
                       const double *psiA, const double *f, double iso, double y_ref,
                       double out[8]);

/* Slip in a flat channel (Sec. III.A): x-averaged u_out,x(y), a parabola
 * fitted over region-III rows of the fluid gap [0, ny-P], evaluated at the
 * hydrodynamic boundary y_w where phi(y_w) = 0.01.  out = (b, u_s, c2) with
 * u_s the fitted velocity at y_w (mean of both walls), b = u_s / |du/dy|(y_w)
 * and c2 the second derivative of the fit.  Returns 0 or -1. */
int orc_slip_length(const orc_params *p, const double *phi, const double *psiR,
                    const double *psiA, const double *f, int P, double width,
                    double out[3]);

/* Velocity residual sum|u_a - u_b| / sum|u_a| over both components. */
double orc_residual(long n, const double *uxa, const double *uya,
                    const double *uxb, const double *uyb);

#ifdef __cplusplus
}
#endif
#endif
