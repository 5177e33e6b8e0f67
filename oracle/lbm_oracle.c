/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).
 *
 * Each function follows one passage of arXiv:1202.6130 and says which.  The
 * model is the paper's wall model on a D2Q9 Shan-Chen fluid:
 *   - fluid-fluid force      : eq. force_SC, written with an explicit coupling
 *                              G:  F_FF = -G psi(x) sum_i w_i psi(x+c_i) c_i,
 *                              psi = 1 - exp(-rho)  (the paper's form is G=-1)
 *   - fluid-solid long range : eq. force_SC_FS with eq. pseudopotential, core
 *                              repulsive and tail attractive:
 *                              F_LR = rho sum_i w_i [G_A psiA - G_R psiR](x+c_i) c_i
 *   - short-range exchange   : eq. wall_shift, with the velocity shift read in
 *                              velocity units:  dF_S = phi^eps [rho(U - u) - F_FF]
 *   - forcing                : exact difference method (Sec. II.B):
 *                              df = feq(rho, u*) - feq(rho, u), u* = u + F/rho
 *   - collision              : BGK (eq. BE-BGK) with feq from eq. f2
 *   - streaming              : f_i(x + c_i, t+1) = f'_i(x, t)  (Sec. II.A)
 *
 * The paper's own model (Sec. II.A-B) uses the D2Q21 lattice of Tab. I and
 * the equation-of-state pseudo-potential of eq. EOS with an attractive
 * fluid-fluid force (G = -1 in the notation above); both are selected by the
 * parameters, every loop runs over the chosen velocity set.
 *
 * The per-node loops carry OpenMP annotations.  The default build ignores
 * them (one thread); a second build with -fopenmp serves long reference runs
 * only.  Each node's arithmetic and every sum keep their order, so both
 * builds give bitwise the same results.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

const int ORC_CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int ORC_CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double ORC_W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                         1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                         1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const double ORC_THETA = 1.0 / 3.0;

/* Tab. I: D2Q21 abscissas and Gauss-Hermite weights (rest state first). */
const int ORC21_CX[21] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2, 3, 0, -3, 0};
const int ORC21_CY[21] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2, 0, 3, 0, -3};
const double ORC21_W[21] = {91.0 / 324.0,
                            1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0,
                            2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
                            7.0 / 360.0, 7.0 / 360.0, 7.0 / 360.0, 7.0 / 360.0,
                            1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
                            1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0};
const double ORC21_THETA = 2.0 / 3.0;

typedef struct {
    int Q;
    const int *cx, *cy;
    const double *w;
    double theta;
} orc_lattice;

static orc_lattice lattice_of(int lattice)
{
    orc_lattice L;
    if (lattice == 21) {
        L.Q = 21; L.cx = ORC21_CX; L.cy = ORC21_CY; L.w = ORC21_W; L.theta = ORC21_THETA;
    } else {
        L.Q = 9; L.cx = ORC_CX; L.cy = ORC_CY; L.w = ORC_W; L.theta = ORC_THETA;
    }
    return L;
}

static long node(int nx, int ny, int x, int y)
{
    /* periodic wrap in both directions */
    x = ((x % nx) + nx) % nx;
    y = ((y % ny) + ny) % ny;
    return (long)y * nx + x;
}

/* Eq. f2 at equilibrium: f_i = w_i [M0 + M1.c/theta + (M2 - M0 theta I):(cc - theta I)/(2 theta^2)]
 * with M0 = rho, M1 = rho u, M2 = rho u u + rho theta I (eqs. M0-M2, feqc). */
void orc_equilibrium_q(int lattice, double rho, double ux, double uy, double *feq)
{
    const orc_lattice L = lattice_of(lattice);
    const double th = L.theta;
    for (int i = 0; i < L.Q; ++i) {
        double cx = L.cx[i], cy = L.cy[i];
        double M1c = rho * (ux * cx + uy * cy);
        /* (M2 - rho theta I) : (c c - theta I) with M2 - rho theta I = rho u u */
        double uucc = rho * (ux * ux * (cx * cx - th) + 2.0 * ux * uy * cx * cy +
                             uy * uy * (cy * cy - th));
        feq[i] = L.w[i] * (rho + M1c / th + uucc / (2.0 * th * th));
    }
}

void orc_equilibrium(double rho, double ux, double uy, double feq[9])
{
    orc_equilibrium_q(9, rho, ux, uy, feq);
}

/* T(s; w) = (1 - tanh(s/w))/2: 1 deep in the solid, 1/2 on the face, 0 in the
 * fluid bulk. */
static double tanh_profile(double s, double w) { return 0.5 * (1.0 - tanh(s / w)); }

void orc_flat_slab_walls(int nx, int ny, int P, double width, double core,
                         double tail, double *phi, double *psiR, double *psiA)
{
    for (int y = 0; y < ny; ++y) {
        double s;
        if (P <= 0) {
            s = INFINITY; /* no solid anywhere */
        } else if (y <= ny - P) {
            /* fluid gap (faces on rows 0 and ny-P included) */
            int a = y, b = ny - P - y;
            s = (double)(a < b ? a : b);
        } else {
            /* inside the solid band */
            int a = y - (ny - P), b = ny - y;
            s = -(double)(a < b ? a : b);
        }
        for (int x = 0; x < nx; ++x) {
            long n = (long)y * nx + x;
            double tp = isinf(s) ? 0.0 : tanh_profile(s, width);
            double tr = isinf(s) ? 0.0 : tanh_profile(s, core);
            double tt = isinf(s) ? 0.0 : tanh_profile(s, tail);
            phi[n] = tp;
            psiR[n] = tr;
            psiA[n] = tt - tr;
        }
    }
}

/* Appendix A, eq. iteration: recursive Gaussian filter of the solid
 * indicator.  G^0 = H (1 on the solid region, 0 elsewhere); each pass
 * replaces G by sum_i w_i G(x + r_i) over the lattice's velocity set
 * (periodic wrap) and then sets G = 1 again on the outer-boundary nodes
 * (bnd != 0), which belong to the solid bulk.  The pass count N_s is read as
 * the number of repeated applications.  The wall functions follow the
 * paper's choice: psiR = G^(n_core), phi = G^(n_wall), psiA = phi - psiR. */
void orc_filter_walls(int lattice, int nx, int ny, const double *solid, const double *bnd,
                      int n_core, int n_wall, double *phi, double *psiR, double *psiA)
{
    const orc_lattice L = lattice_of(lattice);
    const long N = (long)nx * ny;
    double *g = (double *)malloc(sizeof(double) * N);
    double *h = (double *)malloc(sizeof(double) * N);
    memcpy(g, solid, sizeof(double) * N);
    for (long n = 0; n < N; ++n) psiR[n] = g[n];
    for (int pass = 1; pass <= n_wall; ++pass) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int i = 0; i < L.Q; ++i) acc += L.w[i] * g[node(nx, ny, x + L.cx[i], y + L.cy[i])];
                h[(long)y * nx + x] = acc;
            }
        for (long n = 0; n < N; ++n) g[n] = bnd[n] != 0.0 ? 1.0 : h[n];
        if (pass == n_core)
            for (long n = 0; n < N; ++n) psiR[n] = g[n];
    }
    for (long n = 0; n < N; ++n) {
        phi[n] = g[n];
        psiA[n] = g[n] - psiR[n];
    }
    free(g);
    free(h);
}

void orc_init(const orc_params *p, const double *rho0, const double *ux0,
              const double *uy0, double *f)
{
    const int Q = lattice_of(p->lattice).Q;
    long N = (long)p->nx * p->ny;
    for (long n = 0; n < N; ++n) {
        double ux = ux0 ? ux0[n] : 0.0;
        double uy = uy0 ? uy0[n] : 0.0;
        orc_equilibrium_q(p->lattice, rho0[n], ux, uy, &f[n * Q]);
    }
}

/* Eqs. M0 and M1: zeroth and first moments of the populations. */
static void moments(const orc_lattice *L, const double *fn, double *rho, double *jx, double *jy)
{
    double r = 0.0, a = 0.0, b = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        r += fn[i];
        a += fn[i] * L->cx[i];
        b += fn[i] * L->cy[i];
    }
    *rho = r;
    *jx = a;
    *jy = b;
}

/* Eq. EOS: vapour, unstable and liquid branches of slopes theta_V, theta_U,
 * theta_L, joined continuously at rho_1 and rho_2. */
double orc_p_eos(const orc_params *p, double rho)
{
    const double th = lattice_of(p->lattice).theta;
    const double tV = p->eos[0] * th, tU = p->eos[1] * th, tL = p->eos[2] * th;
    const double r1 = p->eos[3], r2 = p->eos[4];
    const double p1 = r1 * tV, p2 = p1 + (r2 - r1) * tU;
    if (rho <= r1) return rho * tV;
    if (rho <= r2) return p1 + (rho - r1) * tU;
    return p2 + (rho - r2) * tL;
}

/* Pseudo-potential of eq. force_SC.  psi_kind 0: 1 - exp(-rho).  psi_kind 1:
 * the EOS pseudo-potential.  A Taylor expansion of eq. force_SC gives
 * sum_i w_i psi(x + r_i) r_i = theta grad psi + ..., so an attractive force
 * (G = -1) adds -theta psi^2 / 2 to the ideal pressure rho theta; the bulk
 * pressure equals p_EOS when psi^2 = 2 (rho theta - p_EOS) / theta.  The
 * printed form lacks the 1/theta; this reading restores the stated
 * coexistence (checked against the mechanical-stability integral). */
double orc_psi(const orc_params *p, double rho)
{
    if (p->psi_kind == 1) {
        const double th = lattice_of(p->lattice).theta;
        double a = 2.0 * (rho * th - orc_p_eos(p, rho)) / th;
        return sqrt(a > 0.0 ? a : 0.0);
    }
    return 1.0 - exp(-rho);
}

void orc_forces(const orc_params *p, const double *phi, const double *psiR,
                const double *psiA, const double *f, double *rho_o, double *ux_o,
                double *uy_o, double *Fff, double *Flr, double *dFs,
                double *Ftot, double *usx, double *usy)
{
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
    const orc_lattice L = lattice_of(p->lattice);
    const int Q = L.Q;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *psi = (double *)malloc(sizeof(double) * N);
    double *psiFS = (double *)malloc(sizeof(double) * N);

    /* moments and pseudo-potentials at every node */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double jx, jy;
        moments(&L, &f[n * Q], &rho[n], &jx, &jy);
        psi[n] = orc_psi(p, rho[n]);
        /* eq. pseudopotential, with the repulsive core entering with the
         * opposite sign of the attractive tail */
        psiFS[n] = p->G_A * psiA[n] - p->G_R * psiR[n];
    }

#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            long n = (long)y * nx + x;
            double r, jx, jy;
            moments(&L, &f[n * Q], &r, &jx, &jy);
            double ux = jx / r, uy = jy / r;

            /* eq. force_SC: fluid-fluid force from neighbour pseudo-potentials */
            double sffx = 0.0, sffy = 0.0;
            /* eq. force_SC_FS, first term: long-range fluid-solid force */
            double sfsx = 0.0, sfsy = 0.0;
            for (int i = 0; i < Q; ++i) {
                long m = node(nx, ny, x + L.cx[i], y + L.cy[i]);
                sffx += L.w[i] * psi[m] * L.cx[i];
                sffy += L.w[i] * psi[m] * L.cy[i];
                sfsx += L.w[i] * psiFS[m] * L.cx[i];
                sfsy += L.w[i] * psiFS[m] * L.cy[i];
            }
            double ffx = -p->G * psi[n] * sffx;
            double ffy = -p->G * psi[n] * sffy;
            double lrx = r * sfsx;
            double lry = r * sfsy;

            /* eq. wall_shift: dF_S = rho phi^eps du_wall, du_wall = U - u - F_FF/rho */
            double pe = pow(phi[n], p->eps);
            double dsx = pe * (r * (p->U_wall[0] - ux) - ffx);
            double dsy = pe * (r * (p->U_wall[1] - uy) - ffy);

            double Fx = ffx + lrx + dsx + p->F_ext[0];
            double Fy = ffy + lry + dsy + p->F_ext[1];

            if (rho_o) rho_o[n] = r;
            if (ux_o) ux_o[n] = ux;
            if (uy_o) uy_o[n] = uy;
            if (Fff) { Fff[2 * n] = ffx; Fff[2 * n + 1] = ffy; }
            if (Flr) { Flr[2 * n] = lrx; Flr[2 * n + 1] = lry; }
            if (dFs) { dFs[2 * n] = dsx; dFs[2 * n + 1] = dsy; }
            if (Ftot) { Ftot[2 * n] = Fx; Ftot[2 * n + 1] = Fy; }
            /* exact difference method: shifted velocity u* = u + g dt, g = F/rho */
            if (usx) usx[n] = ux + Fx / r;
            if (usy) usy[n] = uy + Fy / r;
        }
    }
    free(rho);
    free(psi);
    free(psiFS);
}

/* Projection (Sec. II.A, after eq. f2): the populations are replaced by the
 * truncated Hermite form of eq. f2 built from their own M0, M1 and M2
 * (eqs. M0-M2), which keeps those three moments and drops every component of
 * higher order. */
void orc_project_q(int lattice, const double *f, double *fp)
{
    const orc_lattice L = lattice_of(lattice);
    const double th = L.theta;
    double M0 = 0, M1x = 0, M1y = 0, Mxx = 0, Mxy = 0, Myy = 0;
    for (int i = 0; i < L.Q; ++i) {
        double cx = L.cx[i], cy = L.cy[i];
        M0 += f[i];
        M1x += f[i] * cx;
        M1y += f[i] * cy;
        Mxx += f[i] * cx * cx;
        Mxy += f[i] * cx * cy;
        Myy += f[i] * cy * cy;
    }
    for (int i = 0; i < L.Q; ++i) {
        double cx = L.cx[i], cy = L.cy[i];
        /* (M2 - M0 theta I) : (c c - theta I) */
        double h2 = (Mxx - M0 * th) * (cx * cx - th) + 2.0 * Mxy * cx * cy + (Myy - M0 * th) * (cy * cy - th);
        fp[i] = L.w[i] * (M0 + (M1x * cx + M1y * cy) / th + h2 / (2.0 * th * th));
    }
}

void orc_collide(const orc_params *p, const double *phi, const double *psiR,
                 const double *psiA, const double *f, double *fpost)
{
    const long N = (long)p->nx * p->ny;
    const int Q = lattice_of(p->lattice).Q;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *ux = (double *)malloc(sizeof(double) * N);
    double *uy = (double *)malloc(sizeof(double) * N);
    double *usx = (double *)malloc(sizeof(double) * N);
    double *usy = (double *)malloc(sizeof(double) * N);
    orc_forces(p, phi, psiR, psiA, f, rho, ux, uy, NULL, NULL, NULL, NULL, usx, usy);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double feq_u[21], feq_s[21], fproj[21];
        const double *fn = &f[n * Q];
        orc_equilibrium_q(p->lattice, rho[n], ux[n], uy[n], feq_u);
        orc_equilibrium_q(p->lattice, rho[n], usx[n], usy[n], feq_s);
        if (p->collision == 1) {
            /* the projection step enforces eq. f2 before the collision */
            orc_project_q(p->lattice, fn, fproj);
            fn = fproj;
        }
        for (int i = 0; i < Q; ++i) {
            double fi = fn[i];
            /* BGK relaxation (eq. BE-BGK) plus the EDM force term */
            fpost[n * Q + i] = fi - (fi - feq_u[i]) / p->tau + (feq_s[i] - feq_u[i]);
        }
    }
    free(rho);
    free(ux);
    free(uy);
    free(usx);
    free(usy);
}

void orc_stream_q(int lattice, int nx, int ny, const double *fpost, double *fout)
{
    const orc_lattice L = lattice_of(lattice);
    const int Q = L.Q;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < Q; ++i) {
                long src = (long)y * nx + x;
                long dst = node(nx, ny, x + L.cx[i], y + L.cy[i]);
                fout[dst * Q + i] = fpost[src * Q + i];
            }
}

void orc_stream(int nx, int ny, const double *fpost, double *fout)
{
    orc_stream_q(9, nx, ny, fpost, fout);
}

void orc_step(const orc_params *p, const double *phi, const double *psiR,
              const double *psiA, const double *f_in, double *f_out)
{
    const long N = (long)p->nx * p->ny;
    const int Q = lattice_of(p->lattice).Q;
    double *fpost = (double *)malloc(sizeof(double) * N * Q);
    orc_collide(p, phi, psiR, psiA, f_in, fpost);
    orc_stream_q(p->lattice, p->nx, p->ny, fpost, f_out);
    free(fpost);
}

int orc_run(const orc_params *p, const double *phi, const double *psiR,
            const double *psiA, double *f, long nsteps)
{
    const long N = (long)p->nx * p->ny;
    const int Q = lattice_of(p->lattice).Q;
    double *g = (double *)malloc(sizeof(double) * N * Q);
    if (!g) return -1;
    for (long s = 0; s < nsteps; ++s) {
        orc_step(p, phi, psiR, psiA, f, g);
        memcpy(f, g, sizeof(double) * N * Q);
    }
    free(g);
    return 0;
}

void orc_macros(const orc_params *p, const double *phi, const double *psiR,
                const double *psiA, const double *f, double *rho, double *ux,
                double *uy, double totals[3])
{
    const long N = (long)p->nx * p->ny;
    double *r = (double *)malloc(sizeof(double) * N);
    double *vx = (double *)malloc(sizeof(double) * N);
    double *vy = (double *)malloc(sizeof(double) * N);
    double *F = (double *)malloc(sizeof(double) * N * 2);
    orc_forces(p, phi, psiR, psiA, f, r, vx, vy, NULL, NULL, NULL, F, NULL, NULL);
    double sr = 0.0, sx = 0.0, sy = 0.0;
    for (long n = 0; n < N; ++n) {
        if (rho) rho[n] = r[n];
        /* velocity averaged over the step: (j + F/2)/rho */
        if (ux) ux[n] = vx[n] + 0.5 * F[2 * n] / r[n];
        if (uy) uy[n] = vy[n] + 0.5 * F[2 * n + 1] / r[n];
        sr += r[n];
        sx += r[n] * vx[n];
        sy += r[n] * vy[n];
    }
    if (totals) {
        totals[0] = sr;
        totals[1] = sx;
        totals[2] = sy;
    }
    free(r);
    free(vx);
    free(vy);
    free(F);
}

long orc_isoline_points(int nx, int ny, const double *rho, const double *phi,
                        double iso, double phi_max, double *px, double *py,
                        long cap)
{
    long k = 0;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            long a = (long)y * nx + x;
            if (!(phi[a] < phi_max)) continue;
            /* edge to the right neighbour (periodic in x) */
            long b = (long)y * nx + (x + 1) % nx;
            if (phi[b] < phi_max && ((rho[a] >= iso) != (rho[b] >= iso))) {
                double t = (iso - rho[a]) / (rho[b] - rho[a]);
                if (k < cap) { px[k] = x + t; py[k] = y; }
                ++k;
            }
            /* edge to the upper neighbour (no wrap in y) */
            if (y + 1 < ny) {
                long c = (long)(y + 1) * nx + x;
                if (phi[c] < phi_max && ((rho[a] >= iso) != (rho[c] >= iso))) {
                    double t = (iso - rho[a]) / (rho[c] - rho[a]);
                    if (k < cap) { px[k] = x; py[k] = y + t; }
                    ++k;
                }
            }
        }
    }
    return k;
}

/* Solve the 3x3 system A z = b by Gaussian elimination with partial pivoting.
 * Returns -1 if A is singular to working precision. */
static int solve3(double A[3][3], double b[3], double z[3])
{
    double scale = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) scale = fmax(scale, fabs(A[r][c]));
    if (!(scale > 0.0)) return -1;
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (fabs(A[piv][col]) <= 1e-14 * scale) return -1;
        if (piv != col) {
            for (int c = 0; c < 3; ++c) {
                double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < 3; ++r) {
            double m = A[r][col] / A[col][col];
            for (int c = col; c < 3; ++c) A[r][c] -= m * A[col][c];
            b[r] -= m * b[col];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < 3; ++c) s -= A[r][c] * z[c];
        z[r] = s / A[r][r];
    }
    return 0;
}

int orc_circle_fit(long n, const double *px, const double *py, double out[3])
{
    if (n < 3) return -1;
    /* work about the centroid for conditioning */
    double mx = 0.0, my = 0.0;
    for (long k = 0; k < n; ++k) { mx += px[k]; my += py[k]; }
    mx /= n;
    my /= n;

    /* Kasa: minimise sum (x^2 + y^2 + D x + E y + F)^2 over (D, E, F) */
    double A[3][3] = {{0}}, b[3] = {0}, z[3];
    for (long k = 0; k < n; ++k) {
        double x = px[k] - mx, y = py[k] - my, q = x * x + y * y;
        double v[3] = {x, y, 1.0};
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) A[r][c] += v[r] * v[c];
            b[r] -= v[r] * q;
        }
    }
    if (solve3(A, b, z) != 0) return -1;
    double xc = -0.5 * z[0], yc = -0.5 * z[1];
    double R2 = xc * xc + yc * yc - z[2];
    if (!(R2 > 0.0)) return -1;
    double R = sqrt(R2);

    /* Gauss-Newton on r_k = |p_k - c| - R */
    for (int it = 0; it < 20; ++it) {
        double J[3][3] = {{0}}, g[3] = {0}, d[3];
        for (long k = 0; k < n; ++k) {
            double dx = px[k] - mx - xc, dy = py[k] - my - yc;
            double dist = sqrt(dx * dx + dy * dy);
            if (!(dist > 0.0)) return -1;
            double jr[3] = {-dx / dist, -dy / dist, -1.0};
            double res = dist - R;
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) J[r][c] += jr[r] * jr[c];
                g[r] -= jr[r] * res;
            }
        }
        if (solve3(J, g, d) != 0) return -1;
        xc += d[0];
        yc += d[1];
        R += d[2];
        if (fabs(d[0]) + fabs(d[1]) + fabs(d[2]) < 1e-13 * (1.0 + fabs(R))) break;
    }
    if (!(R > 0.0) || !isfinite(R)) return -1;
    out[0] = xc + mx;
    out[1] = yc + my;
    out[2] = R;
    return 0;
}

int orc_contact_angle(const orc_params *p, const double *phi,
                      const double *psiR, const double *psiA, const double *f,
                      double iso, double y_ref, double out[4])
{
    const long N = (long)p->nx * p->ny;
    double *rho = (double *)malloc(sizeof(double) * N);
    orc_macros(p, phi, psiR, psiA, f, rho, NULL, NULL, NULL);
    long cap = 2 * N;
    double *px = (double *)malloc(sizeof(double) * cap);
    double *py = (double *)malloc(sizeof(double) * cap);
    /* region III: hydrodynamic region, phi < 0.01 (Sec. III.C) */
    long n = orc_isoline_points(p->nx, p->ny, rho, phi, iso, 0.01, px, py, cap);
    int rc = -1;
    double c[3];
    if (n >= 16 && orc_circle_fit(n, px, py, c) == 0) {
        /* theta_Y = acos(1 - h/R) with h = yc + R - y_ref (Sec. III.B) */
        double cs = (y_ref - c[1]) / c[2];
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        out[0] = acos(cs) * 180.0 / M_PI;
        out[1] = c[2];
        out[2] = c[0];
        out[3] = c[1];
        rc = 0;
    }
    free(rho);
    free(px);
    free(py);
    return rc;
}

/* Sec. III.C: advancing and receding angles of a moving drop from two
 * circles fitted to the rear and front parts of its region-III isoline, both
 * ending at the apex, and the drop's mean speed U.  x is taken periodic about
 * the circular mean of the crossings so that a drop across x = 0 stays whole;
 * the apex is the highest crossing (the smaller x on a tie); U is the
 * rho-weighted mean u_x of the region-III nodes with rho >= iso (u the
 * reported velocity); the advancing side is the one U points to. */
int orc_dynamic_angles(const orc_params *p, const double *phi, const double *psiR,
                       const double *psiA, const double *f, double iso, double y_ref,
                       double out[8])
{
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *ux = (double *)malloc(sizeof(double) * N);
    double *uy = (double *)malloc(sizeof(double) * N);
    orc_macros(p, phi, psiR, psiA, f, rho, ux, uy, NULL);
    long cap = 2 * N;
    double *px = (double *)malloc(sizeof(double) * cap);
    double *py = (double *)malloc(sizeof(double) * cap);
    double *sx = (double *)malloc(sizeof(double) * cap);
    double *sy = (double *)malloc(sizeof(double) * cap);
    long n = orc_isoline_points(nx, ny, rho, phi, iso, 0.01, px, py, cap);
    int rc = -1;
    if (n >= 16) {
        double ss = 0, sc = 0;
        for (long k = 0; k < n; ++k) {
            ss += sin(2.0 * M_PI * px[k] / nx);
            sc += cos(2.0 * M_PI * px[k] / nx);
        }
        double xmid = atan2(ss, sc) * nx / (2.0 * M_PI);
        if (xmid < 0) xmid += nx;
        long top = -1;
        for (long k = 0; k < n; ++k) {
            px[k] -= nx * floor((px[k] - xmid) / nx + 0.5);
            if (top < 0 || py[k] > py[top] || (py[k] == py[top] && px[k] < px[top])) top = k;
        }
        double c[2][3];
        int ok = 1;
        for (int side = 0; side < 2 && ok; ++side) {
            long m = 0;
            for (long k = 0; k < n; ++k)
                if (side == 0 ? px[k] <= px[top] : px[k] >= px[top]) {
                    sx[m] = px[k];
                    sy[m] = py[k];
                    ++m;
                }
            ok = m >= 8 && orc_circle_fit(m, sx, sy, c[side]) == 0;
        }
        double mass = 0, mom = 0, cnt = 0;
        for (long a = 0; a < N; ++a)
            if (phi[a] < 0.01 && rho[a] >= iso) {
                mass += rho[a];
                mom += rho[a] * ux[a];
                cnt += 1;
            }
        if (ok && mass > 0) {
            double U = mom / mass;
            int adv = U >= 0 ? 1 : 0;
            for (int k = 0; k < 2; ++k) {
                int sdx = k == 0 ? adv : 1 - adv;
                double cs = (y_ref - c[sdx][1]) / c[sdx][2];
                if (cs > 1.0) cs = 1.0;
                if (cs < -1.0) cs = -1.0;
                out[k] = acos(cs) * 180.0 / M_PI;
                out[3 + k] = c[sdx][2];
            }
            out[2] = U;
            out[5] = px[top] - nx * floor(px[top] / nx);
            out[6] = py[top];
            out[7] = mass / cnt;
            rc = 0;
        }
    }
    free(rho); free(ux); free(uy); free(px); free(py); free(sx); free(sy);
    return rc;
}

int orc_slip_length(const orc_params *p, const double *phi, const double *psiR,
                    const double *psiA, const double *f, int P, double width,
                    double out[3])
{
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
    double *ux = (double *)malloc(sizeof(double) * N);
    orc_macros(p, phi, psiR, psiA, f, NULL, ux, NULL, NULL);
    int top = ny - P;           /* row of the upper face */
    double yc = 0.5 * top;      /* centre of the gap, for conditioning */
    double A[3][3] = {{0}}, b[3] = {0}, z[3];
    int rows = 0;
    for (int y = 0; y <= top; ++y) {
        /* region III rows only; phi is uniform along a row for a flat slab */
        if (!(phi[(long)y * nx] < 0.01)) continue;
        double m = 0.0;
        for (int x = 0; x < nx; ++x) m += ux[(long)y * nx + x];
        m /= nx;
        double t = y - yc;
        double v[3] = {1.0, t, t * t};
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) A[r][c] += v[r] * v[c];
            b[r] += v[r] * m;
        }
        ++rows;
    }
    free(ux);
    if (rows < 3 || solve3(A, b, z) != 0) return -1;
    /* hydrodynamic boundary: T(s; width) = 0.01 -> s = width * atanh(0.98) */
    double sw = width * atanh(0.98);
    double yb = sw - yc, yt = (top - sw) - yc;
    double ub = z[0] + z[1] * yb + z[2] * yb * yb;
    double ut = z[0] + z[1] * yt + z[2] * yt * yt;
    double gb = fabs(z[1] + 2.0 * z[2] * yb);
    double gt = fabs(z[1] + 2.0 * z[2] * yt);
    double us = 0.5 * (ub + ut);
    double g = 0.5 * (gb + gt);
    out[0] = g > 0.0 ? us / g : INFINITY;
    out[1] = us;
    out[2] = 2.0 * z[2];
    return 0;
}

double orc_residual(long n, const double *uxa, const double *uya,
                    const double *uxb, const double *uyb)
{
    double num = 0.0, den = 0.0;
    for (long k = 0; k < n; ++k) {
        num += fabs(uxa[k] - uxb[k]) + fabs(uya[k] - uyb[k]);
        den += fabs(uxa[k]) + fabs(uya[k]);
    }
    return den > 0.0 ? num / den : 0.0;
}
