/*
 * FP64 CPU oracle for the D2Q8 porous MRT-LB scheme (Liu & He, arXiv:1311.7239)
 * and the D2Q5 MRT thermal model of its Appendix B.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product library.
 *
 * The code follows the paper's equations in the paper's order, in plain
 * double precision, with a push-style streaming step:
 *   m = M f (Eq. 8), u from Eqs. (18)-(19), F from Eq. (3), p from Eq. (20),
 *   m^eq from Eqs. (11)-(12), S from Eq. (16), m+ from Eq. (14),
 *   f+ = M^-1 m+ with M^-1 from Gauss-Jordan elimination, then
 *   f_i(x + e_i, t + 1) = f_i+(x, t) (Eq. 15).
 * Boundaries: periodic wrap, or halfway bounce-back on walls half a link
 * outside the edge nodes; a link that crosses the top wall y = ny picks up
 * the moving-wall term of the lid (corners included). Or on-node walls with
 * non-equilibrium extrapolation (the paper's default, Sec. 3, Ref. [40]).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Eq. (10), rows in the moment order of Eq. (9): p, e, jx, qx, jy, qy, pxx, pxy. */
static const double M_PAPER[8][8] = {
    { 1,  1,  1,  1,  1,  1,  1,  1},
    {-1, -1, -1, -1,  1,  1,  1,  1},
    { 1,  0, -1,  0,  1, -1, -1,  1},
    {-2,  0,  2,  0,  1, -1, -1,  1},
    { 0,  1,  0, -1,  1,  1, -1, -1},
    { 0, -2,  0,  2,  1,  1, -1, -1},
    { 1, -1,  1, -1,  0,  0,  0,  0},
    { 0,  0,  0,  0,  1, -1,  1, -1},
};

/* Eq. (B.4). */
static const double N_PAPER[5][5] = {
    { 1,  1,  1,  1,  1},
    { 0,  1,  0, -1,  0},
    { 0,  0,  1,  0, -1},
    {-4,  1,  1,  1,  1},
    { 0,  1, -1,  1, -1},
};

/* Eq. (7) with c = 1: axis links i = 1..4 at angles (i-1) pi/2, diagonal
 * links i = 5..8 at angles (2i-9) pi/4 with length sqrt(2). */
static const int EX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[8] = {0, 1, 0, -1, 1, 1, -1, -1};
/* D2Q5 of Eq. (B.3). */
static const int TX[5] = {0, 1, 0, -1, 0};
static const int TY[5] = {0, 0, 1, 0, -1};

/* Weights omega_i of the text after Eq. (20) (omega_0 belongs to the absent
 * rest particle). */
static const double W0 = 4.0 / 9.0;
static const double W[8] = {1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 */

/* ---------------------------------------------------------------- matrices */

/* Gauss-Jordan elimination with partial pivoting on an n x n row-major
 * matrix (n <= 8). A plain textbook routine; used once per call. */
static void gauss_jordan_inverse(int n, const double *A, double *Ainv)
{
    double a[8][16];
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) {
            a[r][c] = A[r * n + c];
            a[r][n + c] = (r == c) ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t;
            }
        double d = a[col][col];
        for (int c = 0; c < 2 * n; ++c) a[col][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double fac = a[r][col];
            if (fac == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) a[r][c] -= fac * a[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = a[r][n + c];
}

static double MINV[8][8];
static double NINV[5][5];
static int matrices_ready = 0;

static void ensure_matrices(void)
{
    if (matrices_ready) return;
    gauss_jordan_inverse(8, &M_PAPER[0][0], &MINV[0][0]);
    gauss_jordan_inverse(5, &N_PAPER[0][0], &NINV[0][0]);
    matrices_ready = 1;
}

void orc_flow_matrices(double M[64], double Minv[64])
{
    ensure_matrices();
    memcpy(M, M_PAPER, sizeof(M_PAPER));
    memcpy(Minv, MINV, sizeof(MINV));
}

void orc_thermal_matrices(double N[25], double Ninv[25])
{
    ensure_matrices();
    memcpy(N, N_PAPER, sizeof(N_PAPER));
    memcpy(Ninv, NINV, sizeof(NINV));
}

void orc_velocities(int ex[8], int ey[8])
{
    for (int i = 0; i < 8; ++i) { ex[i] = EX[i]; ey[i] = EY[i]; }
}

void orc_default_params(orc_params *p)
{
    memset(p, 0, sizeof(*p));
    p->rho0 = 1.0;
    p->J = 1.0;
    p->s_e = 1.1;             /* Sec. 3: s2 = 1.1 */
    p->s_q = 1.2;             /* Sec. 3: s4 = s6 = 1.2 */
    p->alpha2 = -1.0;         /* Sec. 2.2, after Eq. (12) */
    p->c1 = -2.0;
    p->c2 = -2.0;
    p->gamma1 = 2.0 / 3.0;
    p->gamma2 = 0.0;
    p->gamma3 = 2.0 / 3.0;
    p->sigma = 1.0;
    p->zeta3 = 1.1;           /* Sec. 3.4: zeta3 = zeta4 = 1.1 */
    p->zeta4 = 1.1;
    p->varpi = 0.0;           /* App. B: varpi = 0 */
}

void orc_ergun(long n, const double *phi, double dp, double *K, double *Fphi)
{
    for (long k = 0; k < n; ++k) {
        double ph = phi[k];
        if (Fphi) Fphi[k] = 1.75 / sqrt(150.0 * ph * ph * ph);
        if (K) {
            if (ph >= 1.0) K[k] = INFINITY;  /* no solid matrix: free fluid */
            else K[k] = ph * ph * ph * dp * dp / (150.0 * (1.0 - ph) * (1.0 - ph));
        }
    }
}

/* -------------------------------------------------------- per-node pieces */

/* Relaxation rates of Eq. (13): s1 = s3 = s5 = 1 (Sec. 3), s7 = s8 = 1/tau,
 * with nu_e = J nu = cs^2 (tau - 1/2) (Eq. 21). */
static void relaxation_rates(const orc_params *p, double J, double s[8])
{
    double nu_e = J * p->nu;
    double tau = 0.5 + nu_e / CS2;
    s[0] = 1.0; s[1] = p->s_e; s[2] = 1.0; s[3] = p->s_q;
    s[4] = 1.0; s[5] = p->s_q; s[6] = 1.0 / tau; s[7] = 1.0 / tau;
}

void orc_equilibrium_moments(const orc_params *p, double phi, double pres,
                             double ux, double uy, double meq[8])
{
    /* Eqs. (11)-(12); j = rho0 u (incompressibility approximation). */
    double r = p->rho0;
    double u2 = ux * ux + uy * uy;
    meq[0] = 5.0 / 3.0 * phi * pres + 2.0 / 3.0 * r * u2 / phi;
    meq[1] = p->alpha2 * phi * pres + 0.75 * p->gamma2 * r * u2 / phi;
    meq[2] = r * ux;
    meq[3] = 0.5 * p->c1 * r * ux;
    meq[4] = r * uy;
    meq[5] = 0.5 * p->c2 * r * uy;
    meq[6] = 1.5 * p->gamma1 * r * (ux * ux - uy * uy) / phi;
    meq[7] = 1.5 * p->gamma3 * r * ux * uy / phi;
}

void orc_forcing_moments(const orc_params *p, double phi, double ux, double uy,
                         double Fx, double Fy, double S[8])
{
    /* Eq. (16). */
    double r = p->rho0;
    S[0] = 0.0;
    S[1] = r * 4.0 * (ux * Fx + uy * Fy) / (5.0 * phi);
    S[2] = r * Fx;
    S[3] = -r * Fx;
    S[4] = r * Fy;
    S[5] = -r * Fy;
    S[6] = r * 2.0 * (ux * Fx - uy * Fy) / phi;
    S[7] = r * (ux * Fy + uy * Fx) / phi;
}

void orc_velocity(const orc_params *p, double phi, double K, double Fphi,
                  double ax, double ay, const double f[8], double u[2], double F[2])
{
    const double dt = 1.0;
    double r = p->rho0;
    /* Eq. (19) */
    double jx = 0.0, jy = 0.0;
    for (int i = 0; i < 8; ++i) { jx += EX[i] * f[i]; jy += EY[i] * f[i]; }
    double vx = jx / r + 0.5 * dt * phi * ax;
    double vy = jy / r + 0.5 * dt * phi * ay;
    double l0 = 0.5 * (1.0 + phi * 0.5 * dt * p->nu / K);
    double l1 = phi * 0.5 * dt * Fphi / sqrt(K);
    double vmag = sqrt(vx * vx + vy * vy);
    /* Eq. (18) */
    double den = l0 + sqrt(l0 * l0 + l1 * vmag);
    u[0] = vx / den;
    u[1] = vy / den;
    /* Eq. (3) */
    double umag = sqrt(u[0] * u[0] + u[1] * u[1]);
    F[0] = -phi * p->nu / K * u[0] - phi * Fphi / sqrt(K) * umag * u[0] + phi * ax;
    F[1] = -phi * p->nu / K * u[1] - phi * Fphi / sqrt(K) * umag * u[1] + phi * ay;
}

double orc_pressure(const orc_params *p, double phi, const double f[8], double ux, double uy)
{
    /* Eq. (20) with s0(u) = -2 rho0 |u|^2/(3 phi); rho0 is applied once
     * (the printed form multiplies it in twice, which is moot at rho0 = 1
     * and would break conservation of m1 otherwise). */
    double sum = 0.0;
    for (int i = 0; i < 8; ++i) sum += f[i];
    double s0 = -2.0 * (ux * ux + uy * uy) / (3.0 * phi);
    return CS2 / (phi * (1.0 - W0)) * (sum + p->rho0 * s0);
}

static void collide_node_J(const orc_params *p, double J, double phi, double K, double Fphi,
                           double ax, double ay, const double f[8], double fplus[8],
                           double u[2], double *pres);

void orc_collide_node(const orc_params *p, double phi, double K, double Fphi,
                      double ax, double ay, const double f[8], double fplus[8],
                      double u[2], double *pres)
{
    collide_node_J(p, p->J, phi, K, Fphi, ax, ay, f, fplus, u, pres);
}

/* The collision of one node whose viscosity ratio is J (s_nu = 1/tau with
 * nu_e = J nu = cs^2 (tau - 1/2), Eq. 21). */
static void collide_node_J(const orc_params *p, double J, double phi, double K, double Fphi,
                           double ax, double ay, const double f[8], double fplus[8],
                           double u[2], double *pres)
{
    ensure_matrices();
    const double dt = 1.0;
    double s[8];
    relaxation_rates(p, J, s);

    double m[8];
    for (int a = 0; a < 8; ++a) {
        double acc = 0.0;
        for (int i = 0; i < 8; ++i) acc += M_PAPER[a][i] * f[i];
        m[a] = acc;
    }
    double F[2];
    orc_velocity(p, phi, K, Fphi, ax, ay, f, u, F);
    double pr = orc_pressure(p, phi, f, u[0], u[1]);
    double meq[8], S[8];
    orc_equilibrium_moments(p, phi, pr, u[0], u[1], meq);
    orc_forcing_moments(p, phi, u[0], u[1], F[0], F[1], S);
    double mp[8];
    for (int a = 0; a < 8; ++a)
        mp[a] = m[a] - s[a] * (m[a] - meq[a]) + dt * (1.0 - 0.5 * s[a]) * S[a];
    for (int i = 0; i < 8; ++i) {
        double acc = 0.0;
        for (int a = 0; a < 8; ++a) acc += MINV[i][a] * mp[a];
        fplus[i] = acc;
    }
    if (pres) *pres = pr;
}

/* D2Q5 collision of Eq. (B.2) at one node, using the flow velocity u. */
static void thermal_collide_node(const orc_params *p, const double g[5], double ux,
                                 double uy, double gplus[5])
{
    double n[5];
    for (int a = 0; a < 5; ++a) {
        double acc = 0.0;
        for (int j = 0; j < 5; ++j) acc += N_PAPER[a][j] * g[j];
        n[a] = acc;
    }
    double T = n[0];
    /* Eq. (B.6) */
    double neq[5] = {T, ux * T / p->sigma, uy * T / p->sigma, p->varpi * T, 0.0};
    /* Eq. (B.7), zeta1 = zeta2 = 1/tau_T */
    double th[5] = {1.0, 1.0 / p->tau_T, 1.0 / p->tau_T, p->zeta3, p->zeta4};
    double np_[5];
    for (int a = 0; a < 5; ++a) np_[a] = n[a] - th[a] * (n[a] - neq[a]);
    for (int j = 0; j < 5; ++j) {
        double acc = 0.0;
        for (int a = 0; a < 5; ++a) acc += NINV[j][a] * np_[a];
        gplus[j] = acc;
    }
}

/* ------------------------------------------------------------------ steps */

/* Index of the opposite link. */
static int opposite8(int i) { return (i < 4) ? ((i + 2) & 3) : (4 + ((i - 4 + 2) & 3)); }
static int opposite5(int j) { return (j == 0) ? 0 : 1 + ((j - 1 + 2) & 3); }

static double buoyancy_y(const orc_params *p, double T)
{
    /* Sec. 3.4: a = g beta (T - T0) j */
    return p->gbeta * (T - p->T0);
}

static void nee_walls(const orc_params *p, const double *phi, const double *K, const double *Fphi,
                      double *f, double *g);

void orc_step(const orc_params *p, const double *phi, const double *K, const double *Fphi,
              const double *f, double *fnew, const double *g, double *gnew)
{
    ensure_matrices();
    const int nx = p->nx, ny = p->ny;
    const double r = p->rho0;
    const int thermal = p->thermal && g && gnew;
    /* D2Q5 link weight of the rest-state distribution: (4 + varpi)/20. */
    const double wT = (4.0 + p->varpi) / 20.0;
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            double ax = p->ax, ay = p->ay;
            if (thermal) {
                double T = 0.0;
                for (int j = 0; j < 5; ++j) T += g[k * 5 + j];
                ay += buoyancy_y(p, T);
            }
            double fp[8], u[2], pr;
            collide_node_J(p, p->Jcell ? p->Jcell[k] : p->J, phi[k], K[k], Fphi[k], ax, ay,
                           &f[k * 8], fp, u, &pr);
            for (int i = 0; i < 8; ++i) {
                int xt = x + EX[i], yt = y + EY[i];
                int out_x = (xt < 0 || xt >= nx), out_y = (yt < 0 || yt >= ny);
                if (out_x && p->bc_x == ORC_PERIODIC) { xt = (xt + nx) % nx; out_x = 0; }
                if (out_y && p->bc_y == ORC_PERIODIC) { yt = (yt + ny) % ny; out_y = 0; }
                if (!out_x && !out_y) {
                    fnew[((long)yt * nx + xt) * 8 + i] = fp[i];
                } else if ((out_x && p->bc_x == ORC_NEE) || (out_y && p->bc_y == ORC_NEE)) {
                    /* leaves through an on-node wall: the wall node's own
                     * populations are rebuilt after streaming */
                } else {
                    /* halfway bounce-back; the link returns to this node as
                     * the opposite population, with the moving-wall term
                     * 2 rho0 w (e . u_w)/cs^2 of the wall it crossed. */
                    int o = opposite8(i);
                    double uwx = (p->bc_y == ORC_WALLS && yt >= ny) ? p->lid_ux : 0.0;
                    double eu = EX[o] * uwx;
                    fnew[k * 8 + o] = fp[i] + 2.0 * r * W[o] * eu / CS2;
                }
            }
            if (thermal) {
                double gp[5];
                thermal_collide_node(p, &g[k * 5], u[0], u[1], gp);
                for (int j = 0; j < 5; ++j) {
                    int xt = x + TX[j], yt = y + TY[j];
                    int out_x = (xt < 0 || xt >= nx), out_y = (yt < 0 || yt >= ny);
                    if (out_x && p->bc_x == ORC_PERIODIC) { xt = (xt + nx) % nx; out_x = 0; }
                    if (out_y && p->bc_y == ORC_PERIODIC) { yt = (yt + ny) % ny; out_y = 0; }
                    if (!out_x && !out_y) {
                        gnew[((long)yt * nx + xt) * 5 + j] = gp[j];
                    } else if ((out_x && p->bc_x == ORC_NEE) || (out_y && p->bc_y == ORC_NEE)) {
                        /* rebuilt after streaming, as for f */
                    } else if (out_x) {
                        /* Dirichlet walls (hot x = 0, cold x = nx): anti-bounce-back */
                        double Tw = (xt < 0) ? p->Th : p->Tc;
                        gnew[k * 5 + opposite5(j)] = -gp[j] + 2.0 * wT * Tw;
                    } else {
                        /* adiabatic walls: bounce-back */
                        gnew[k * 5 + opposite5(j)] = gp[j];
                    }
                }
            }
        }
    }
    if (p->bc_x == ORC_NEE || p->bc_y == ORC_NEE) nee_walls(p, phi, K, Fphi, fnew, thermal ? gnew : NULL);
}

/* Eq. (22): equilibrium populations at porosity phi, pressure pres, velocity u. */
static void feq_eq22(const orc_params *p, double phi, double pres, double ux, double uy,
                     double feq[8])
{
    const double r = p->rho0;
    const double u2 = ux * ux + uy * uy;
    for (int i = 0; i < 8; ++i) {
        const double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = r * W[i] * (phi * pres / (r * CS2) + eu / CS2 + eu * eu / (2.0 * phi * CS2 * CS2) -
                             u2 / (2.0 * phi * CS2));
    }
}

/* Thermal equilibrium g^eq = N^-1 n^eq with n^eq of Eq. (B.6). */
static void geq_b6(const orc_params *p, double T, double ux, double uy, double geq[5])
{
    const double neq[5] = {T, ux * T / p->sigma, uy * T / p->sigma, p->varpi * T, 0.0};
    for (int j = 0; j < 5; ++j) {
        double acc = 0.0;
        for (int a = 0; a < 5; ++a) acc += NINV[j][a] * neq[a];
        geq[j] = acc;
    }
}

/* Non-equilibrium extrapolation at on-node walls (Sec. 3, Ref. [40]).
 * Every population of a wall node O is the equilibrium at the wall's state
 * plus the non-equilibrium part of the next node B inward along the normal
 * (diagonally inward at a corner), all at the same time:
 *   f(O) = f^eq(phi_O, p_O, u_w) + [f(B) - f^eq(phi_B, p_B, u_B)],
 * f^eq from Eq. (22), u_B and p_B from Eqs. (18)-(20) at B (with B's force),
 * the wall taking B's phi p (phi_O p_O = phi_B p_B) and the wall velocity
 * u_w: the lid velocity on the top wall away from on-node x walls (the top
 * corners of a cavity stay at rest), zero elsewhere. Temperature likewise:
 *   g(O) = g^eq(T_w, u_w) + [g(B) - g^eq(T_B, u_B)],
 * T_w = Th / Tc on the x walls (Dirichlet, corners included) and T_w = T_B
 * on the y walls (adiabatic). B is never a wall node (>= 3 nodes per axis). */
static void nee_walls(const orc_params *p, const double *phi, const double *K, const double *Fphi,
                      double *f, double *g)
{
    const int nx = p->nx, ny = p->ny;
    const int thermal = p->thermal && g;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const int wx = p->bc_x == ORC_NEE && (x == 0 || x == nx - 1);
            const int wy = p->bc_y == ORC_NEE && (y == 0 || y == ny - 1);
            if (!wx && !wy) continue;
            const int bx = wx ? (x == 0 ? 1 : nx - 2) : x;
            const int by = wy ? (y == 0 ? 1 : ny - 2) : y;
            const long ko = (long)y * nx + x, kb = (long)by * nx + bx;
            double ax = p->ax, ay = p->ay, TB = 0.0;
            if (thermal) {
                for (int j = 0; j < 5; ++j) TB += g[kb * 5 + j];
                ay += buoyancy_y(p, TB);
            }
            double uB[2], FB[2];
            orc_velocity(p, phi[kb], K[kb], Fphi[kb], ax, ay, &f[kb * 8], uB, FB);
            const double pB = orc_pressure(p, phi[kb], &f[kb * 8], uB[0], uB[1]);
            const double pO = phi[kb] * pB / phi[ko];
            const double uwx = (wy && y == ny - 1 && !wx) ? p->lid_ux : 0.0;
            double eO[8], eB[8];
            feq_eq22(p, phi[ko], pO, uwx, 0.0, eO);
            feq_eq22(p, phi[kb], pB, uB[0], uB[1], eB);
            for (int i = 0; i < 8; ++i) f[ko * 8 + i] = eO[i] + (f[kb * 8 + i] - eB[i]);
            if (thermal) {
                const double Tw = wx ? (x == 0 ? p->Th : p->Tc) : TB;
                double hO[5], hB[5];
                geq_b6(p, Tw, uwx, 0.0, hO);
                geq_b6(p, TB, uB[0], uB[1], hB);
                for (int j = 0; j < 5; ++j) g[ko * 5 + j] = hO[j] + (g[kb * 5 + j] - hB[j]);
            }
        }
    }
}

int orc_run(const orc_params *p, const double *phi, const double *K, const double *Fphi,
            double *f, double *g, long nsteps)
{
    const long n = (long)p->nx * p->ny;
    double *fb = (double *)malloc(sizeof(double) * 8 * n);
    double *gb = NULL;
    if (!fb) return -1;
    const int thermal = p->thermal && g;
    if (thermal) {
        gb = (double *)malloc(sizeof(double) * 5 * n);
        if (!gb) { free(fb); return -1; }
    }
    double *fa = f, *ga = g, *fo = fb, *go = gb;
    for (long t = 0; t < nsteps; ++t) {
        orc_step(p, phi, K, Fphi, fa, fo, thermal ? ga : NULL, thermal ? go : NULL);
        double *tf = fa; fa = fo; fo = tf;
        double *tg = ga; ga = go; go = tg;
    }
    if (fa != f) memcpy(f, fa, sizeof(double) * 8 * n);
    if (thermal && ga != g) memcpy(g, ga, sizeof(double) * 5 * n);
    free(fb);
    free(gb);
    return 0;
}

void orc_macroscopic(const orc_params *p, const double *phi, const double *K,
                     const double *Fphi, const double *f, const double *g,
                     double *ux, double *uy, double *pres, double *T)
{
    const long n = (long)p->nx * p->ny;
    for (long k = 0; k < n; ++k) {
        double ax = p->ax, ay = p->ay, Tk = 0.0;
        if (p->thermal && g) {
            for (int j = 0; j < 5; ++j) Tk += g[k * 5 + j];
            ay += buoyancy_y(p, Tk);
        }
        double u[2], F[2];
        orc_velocity(p, phi[k], K[k], Fphi[k], ax, ay, &f[k * 8], u, F);
        if (ux) ux[k] = u[0];
        if (uy) uy[k] = u[1];
        if (pres) pres[k] = orc_pressure(p, phi[k], &f[k * 8], u[0], u[1]);
        if (T) T[k] = Tk;
    }
}

void orc_rest_state(const orc_params *p, long n, double Pi0, double *f)
{
    /* Eq. (22) at u = 0: f_i = rho0 w_i phi p / (rho0 cs^2) with phi p = Pi0. */
    for (long k = 0; k < n; ++k)
        for (int i = 0; i < 8; ++i) f[k * 8 + i] = p->rho0 * W[i] * Pi0 / (p->rho0 * CS2);
}

void orc_thermal_rest_state(const orc_params *p, long n, const double *T, double *g)
{
    ensure_matrices();
    for (long k = 0; k < n; ++k) {
        double neq[5] = {T[k], 0.0, 0.0, p->varpi * T[k], 0.0};
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int a = 0; a < 5; ++a) acc += NINV[j][a] * neq[a];
            g[k * 5 + j] = acc;
        }
    }
}
