/*
 * FP64 CPU oracle for the D2Q8 porous MRT lattice Boltzmann scheme of
 * Liu & He, "Multiple-relaxation-time lattice Boltzmann modeling of
 * incompressible flows in porous media" (arXiv:1311.7239).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library includes, links
 * or calls this code; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark have an obviously correct reference to compare
 * the GPU path against. It shares no header, helper, table or constant with
 * the GPU path.
 *
 * Conventions (all from Sec. 2.2 and Sec. 3 of the paper):
 *   - lattice units: rho0 = 1 is a parameter, delta_t = delta_x = c = 1;
 *   - node (x, y), 0 <= x < nx, 0 <= y < ny, cell centre at (x+1/2, y+1/2);
 *   - populations stored node-major: f[(y*nx + x)*8 + i], i = 0..7 is the
 *     paper's f_1..f_8 (Eq. 7 ordering); thermal g[(y*nx + x)*5 + j], j = 0..4
 *     as in Eq. (B.3);
 *   - walls sit half a link outside the first/last node (halfway bounce-back).
 *
 * Readings of passages where the paper is silent or ambiguous are listed in
 * the repository's design notes; the ones that change arithmetic are repeated
 * at the function that implements them.
 */
#ifndef MRT_PAPER_ORACLE_H
#define MRT_PAPER_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* ORC_WALLS: halfway bounce-back, walls half a link outside the edge nodes.
 * ORC_NEE: the first and last node of the axis lie on the walls, treated by
 * non-equilibrium extrapolation (Sec. 3, its Ref. [40]); an axis with ORC_NEE
 * needs >= 3 nodes and the other axis ORC_PERIODIC or ORC_NEE. */
enum { ORC_PERIODIC = 0, ORC_WALLS = 1, ORC_NEE = 2 };

typedef struct {
    int nx, ny;
    int bc_x;        /* ORC_PERIODIC, ORC_WALLS (x = 0, x = nx) or ORC_NEE    */
    int bc_y;        /* ORC_PERIODIC, ORC_WALLS (y = 0, y = ny) or ORC_NEE    */
    double lid_ux;   /* x-velocity of the top wall (moving lid); 0 = rest     */
    double rho0;     /* mean density (Eq. 2)                                  */
    double nu;       /* fluid kinematic viscosity (Eq. 3)                     */
    double J;        /* viscosity ratio nu_e / nu (Eq. 5)                     */
    double s_e, s_q; /* s_2 and s_4 = s_6 of Eq. (13)                         */
    double alpha2, c1, c2, gamma1, gamma2, gamma3; /* Eq. (12) parameters     */
    double ax, ay;   /* uniform external acceleration a (Eq. 3)               */
    /* thermal D2Q5 model of Appendix B and the buoyancy of Sec. 3.4 */
    int thermal;     /* 0: isothermal; 1: couple T through a = g beta (T-T0) j */
    double sigma;    /* thermal capacity ratio (Eq. B.1)                      */
    double tau_T;    /* thermal relaxation time: zeta_1 = zeta_2 = 1/tau_T   */
    double zeta3, zeta4;
    double varpi;    /* Eq. (B.6) constant                                    */
    double Th, Tc;   /* Dirichlet temperatures of walls x = 0 and x = nx      */
    double T0;       /* reference temperature of the buoyancy term            */
    double gbeta;    /* g * beta                                              */
    int nthreads;    /* OpenMP threads for the node loops (<= 0: runtime default) */
    const double *Jcell; /* per-node viscosity ratio (NULL: J everywhere); the
                          * relaxation rate s_nu of a node follows its own J
                          * (Sec. 3.2, partially porous channel) */
} orc_params;

/* Fills params with the paper's constants: rho0 = 1, J = 1, s_e = 1.1,
 * s_q = 1.2 (Sec. 3), alpha2 = -1, c1 = c2 = -2, gamma2 = 0,
 * gamma1 = gamma3 = 2/3 (Sec. 2.2), zeta3 = zeta4 = 1.1, varpi = 0 (Sec. 3.4,
 * App. B). Geometry, viscosity and forces are left zero. */
void orc_default_params(orc_params *p);

/* M of Eq. (10) and its inverse (Gauss-Jordan, FP64), row-major 8x8. */
void orc_flow_matrices(double M[64], double Minv[64]);
/* N of Eq. (B.4) and its inverse, row-major 5x5. */
void orc_thermal_matrices(double N[25], double Ninv[25]);
/* Velocity set of Eq. (7) (c = 1) as integers, ex[i], ey[i]. */
void orc_velocities(int ex[8], int ey[8]);

/* Eq. (4): F_phi = 1.75/sqrt(150 phi^3), K = phi^3 dp^2 / (150 (1-phi)^2). */
void orc_ergun(long n, const double *phi, double dp, double *K, double *Fphi);

/* Per-node pieces of Eqs. (11)-(20), exposed for the pins. */
void orc_equilibrium_moments(const orc_params *p, double phi, double pres,
                             double ux, double uy, double meq[8]);
void orc_forcing_moments(const orc_params *p, double phi, double ux, double uy,
                         double Fx, double Fy, double S[8]);
/* Eqs. (17)-(19) and (3): velocity u and total force F from f. */
void orc_velocity(const orc_params *p, double phi, double K, double Fphi,
                  double ax, double ay, const double f[8], double u[2], double F[2]);
/* Eq. (20): pressure from f and u. */
double orc_pressure(const orc_params *p, double phi, const double f[8], double ux, double uy);
/* Eq. (14) and f+ = M^-1 m+: one node's collision; also returns u and p. */
void orc_collide_node(const orc_params *p, double phi, double K, double Fphi,
                      double ax, double ay, const double f[8], double fplus[8],
                      double u[2], double *pres);

/* One collide-and-stream step (Eqs. 14-15), push scheme, f -> fnew
 * (and g -> gnew when p->thermal). Arrays are node-major as above.
 * phi, K, Fphi are per node; K may be +inf (free fluid). With ORC_NEE axes
 * the wall nodes of fnew (and gnew) are rebuilt by non-equilibrium
 * extrapolation after streaming, so every stored state past t = 0 is whole. */
void orc_step(const orc_params *p, const double *phi, const double *K, const double *Fphi,
              const double *f, double *fnew, const double *g, double *gnew);
/* nsteps steps in place (internal double buffer). Returns 0, or -1 on
 * allocation failure. */
int orc_run(const orc_params *p, const double *phi, const double *K, const double *Fphi,
            double *f, double *g, long nsteps);
/* Macroscopic fields at the current time: u (Eq. 18), p (Eq. 20), T (Eq. B.5);
 * any output may be NULL. */
void orc_macroscopic(const orc_params *p, const double *phi, const double *K,
                     const double *Fphi, const double *f, const double *g,
                     double *ux, double *uy, double *pres, double *T);
/* Rest state used at t = 0 (Sec. 3.1): m = m^eq with u = 0 and phi*p = Pi0,
 * f_i = rho0 w_i Pi0/(rho0 cs^2) from Eq. (22); g_j = n^eq-state at T. */
void orc_rest_state(const orc_params *p, long n, double Pi0, double *f);
void orc_thermal_rest_state(const orc_params *p, long n, const double *T, double *g);

#ifdef __cplusplus
}
#endif
#endif
