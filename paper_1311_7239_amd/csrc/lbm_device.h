// Device-side building blocks of the D2Q8 porous MRT-LB step (Liu & He,
// arXiv:1311.7239) for gfx950: the per-node collision in moment space, the
// D2Q5 thermal collision (App. B), and the pull-scheme gather with periodic
// wrap and halfway bounce-back.
//
// Populations are stored as deviations from the rest state f_ref_i = 3 w_i Pi0.
// The collision never needs Pi0: with m = m_ref + dm and
// m_ref = (5/3 Pi0, -Pi0, 0, ..., 0), every term m - m^eq of Eq. (14) is a
// function of the deviations alone, so the kernels work on deviations
// throughout and only the output of the pressure adds Pi0 back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrt {

// Velocity set of Eq. (7), zero-based: index i holds the paper's f_{i+1}.
//   0:(1,0) 1:(0,1) 2:(-1,0) 3:(0,-1) 4:(1,1) 5:(-1,1) 6:(-1,-1) 7:(1,-1)
constexpr int EX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[8] = {0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[8] = {2, 3, 0, 1, 6, 7, 4, 5};
// D2Q5 of Eq. (B.3): 0 rest, 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
constexpr int TXv[5] = {0, 1, 0, -1, 0};
constexpr int TYv[5] = {0, 0, 1, 0, -1};
constexpr int TOPP[5] = {0, 3, 4, 1, 2};

// BC_WALLS: halfway bounce-back, walls half a link outside the edge nodes.
// BC_NEE: the first and last node of the axis lie on the walls
// (non-equilibrium extrapolation); the other axis is periodic or BC_NEE.
enum { BC_PERIODIC = 0, BC_WALLS = 1, BC_NEE = 2 };
enum { MED_UNIFORM = 0, MED_PHI_ERGUN = 1, MED_PHI_KAPPA = 2 };

// Everything a kernel needs to know about one domain. Passed by value as a
// kernel argument (single domain) or read from a device array (batch).
struct Dom {
    int32_t nx, ny, pitch;  // nodes; pitch = elements per stored row
    int32_t bc_x, bc_y;
    int64_t plane;          // elements between consecutive planes
    float lid6;             // 6 w_diag U_lid = U_lid / 6 (diagonal lid links)
    float lid_u;            // U_lid (velocity of on-node lid nodes)
    // relaxation (Eq. 13) and the (1 - s/2) factors of Eq. (14)
    float s_e, s_q, s_nu, h_e, h_q, h_nu;
    // medium
    int32_t medium;
    float phi0, inv_phi0, cd0, cf0;  // uniform: phi, 1/phi, phi nu kappa, phi F sqrt(kappa)
    float cd0h, cf0h;                // cd0 / 2, cf0 / 2 (exact halves)
    float nu;                        // fluid viscosity (per-cell drag)
    float kcoef;                     // 150 / dp^2 (Eq. 4): kappa = kcoef (1-phi)^2 / phi^3
    float cdk, cfk;                  // 150 nu / dp^2 and 1.75 / dp (Eq. 4 drag in closed form)
    float cdkh, cfkh;                // their exact halves
    float Fconst;                    // >= 0: constant F_phi; < 0: Eq. (4)
    float ax, ay;                    // uniform external acceleration
    float axh, ayh;                  // a / 2 (exact halves: the step works on half forces)
    // rates of the half-force forcing: 1.6 (1 - s_e/2), 2 (1 - s_q/2), and
    // 2 (1 - s_nu/2), 4 (1 - s_nu/2) (exact multiples of the float h_q, h_nu)
    float h_e16, h_q2, h_nu2, h_nu4;
    const float *phi;                // [ny][pitch] (MED_PHI_*)
    const float *kappa;              // [ny][pitch] (MED_PHI_KAPPA)
    const float *snu;                // [ny][pitch] per-node s_nu (NULL: s_nu everywhere)
    // thermal (App. B); deviations from wT*T0
    int32_t thermal;
    float zT, z3, z4;                // 1/tau_T, zeta3, zeta4
    float inv_sigma, T0, gbeta, gbetah;  // ..., g beta, g beta / 2
    float abbh, abbc;                // 2 wT (Th - T0), 2 wT (Tc - T0)
    float dTh, dTc;                  // Th - T0, Tc - T0 (on-node Dirichlet walls)
    // state buffers (storage type erased)
    const void *fin;
    void *fout;
    const float *gin;
    float *gout;
    float *urec;                     // optional record of step t: planes u_x, u_y, then
                                     // n7, n8 (with rec_stress) and dT (thermal)
    int32_t rec_stress;              // also record m7 - m7^eq and m8 - m8^eq (planes 2, 3)
    int32_t nt_store;                // store the state non-temporally (state buffers
                                     // larger than the Infinity Cache)
    float inv_nu;                    // 1 / nu (parameter gradients)
    float *uprev;                    // optional: u_x, u_y planes ([ny][pitch] each) of the
                                     // last collision of the pass, i.e. u(t - 1) once the
                                     // pass has advanced the state to t (steady residual)
};

// Square root and reciprocal by the hardware instructions (v_sqrt_f32,
// v_rcp_f32, about 1 ulp) instead of the correctly rounded library sequences
// (a dozen instructions each). They only enter drag coefficients, |u| and
// the velocity-recovery ratio, where an ulp is far below the FP32 noise of
// the populations, and they carry no systematic gain on a conserved moment.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// x * (p/q) for the rational constants of the transforms (1/6, 1/12, 3/5, ...),
// rounded once: the constant is split into its nearest float hi plus the float
// lo of the remainder, and x*hi + x*lo goes through one fused multiply-add.
// A bare x * float(1/6) is 3e-8 too large every time; through the
// back-transform and the next moment sum the momentum would gain that factor
// every step and settle ~1e-4 off in slowly relaxing flows.
__device__ __forceinline__ float mulc(float x, float hi, float lo) { return fmaf(x, hi, x * lo); }
#define MRT_C1_6 0x1.555556p-3f, -0x1.555556p-28f
#define MRT_C1_12 0x1.555556p-4f, -0x1.555556p-29f
#define MRT_C3_5 0x1.333334p-1f, -0x1.99999ap-26f
#define MRT_C2_5 0x1.99999ap-2f, -0x1.99999ap-28f
#define MRT_C4_5 0x1.99999ap-1f, -0x1.99999ap-27f
#define MRT_C1_5 0x1.99999ap-3f, -0x1.99999ap-29f
#define MRT_C1_20 0x1.99999ap-5f, -0x1.99999ap-31f

// Workgroup barrier for LDS exchange only: waits for this wave's LDS accesses
// (lgkmcnt) but not for its outstanding global stores, which no other wave of
// the workgroup reads (__syncthreads also drains those, stalling the
// recording kernels on their u stores). The memory clobber keeps the compiler
// from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Workgroups are dispatched round-robin over the 8 XCDs; this remaps the
// block id so that each XCD walks a contiguous run of tiles (neighbouring
// tiles share cache lines at the x-shifted loads and the halo rows).
__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
    constexpr int NUM_XCD = 8;
    const int q = nb / NUM_XCD;
    if (b >= q * NUM_XCD) return b;
    return (b % NUM_XCD) * q + b / NUM_XCD;
}

// Per-cell quantities of Eqs. (3), (4) and (19).
struct Cell {
    float phi, inv_phi;
    float cd;   // phi nu / K             (linear drag coefficient, Eq. 3)
    float cf;   // phi F_phi / sqrt(K)    (Forchheimer coefficient, Eq. 3)
    float cdh, cfh;    // cd / 2 and cf / 2 (exact halves; the step uses these)
    float s_nu, h_nu;  // s_7 = s_8 = 1/tau of the node's own J (Eq. 21) and 1 - s_nu/2
    float h_nu2, h_nu4;  // 2 h_nu = 2 - s_nu and 4 h_nu = 4 - 2 s_nu (exact)
};

// Ergun's F_phi (Eq. 4): 1.75 / sqrt(150 phi^3) = (1.75/sqrt(150)) phi^{-3/2}.
__device__ __forceinline__ float ergun_F(float inv_phi) {
    return 0.14288690166235206f * inv_phi * hw_sqrt(inv_phi);
}

// Eq. (4) substituted into Eq. (3): phi nu / K = (150 nu / dp^2)(1-phi)^2 / phi^2
// and phi F_phi / sqrt(K) = (1.75 / dp)(1-phi) / phi^2, without square roots.
__device__ __forceinline__ void ergun_closed(const Dom &d, float phi, Cell &c) {
    const float ip = hw_rcp(phi);
    c.phi = phi; c.inv_phi = ip;
    const float om = 1.0f - phi;
    const float t = om * (ip * ip);
    c.cdh = (d.cdkh * om) * t;
    c.cfh = d.cfkh * t;
    c.cd = c.cdh + c.cdh;   // the same bits as (cdk om) t and cfk t
    c.cf = c.cfh + c.cfh;
}

// Per-cell drag coefficients from the porosity (and 1/K when it has its own
// plane); kappa is ignored unless the medium is MED_PHI_KAPPA.
__device__ __forceinline__ Cell cell_from(const Dom &d, float phi, float kappa_plane) {
    Cell c;
    c.s_nu = d.s_nu; c.h_nu = d.h_nu; c.h_nu2 = d.h_nu2; c.h_nu4 = d.h_nu4;
    if (d.medium == MED_UNIFORM) {
        c.phi = d.phi0; c.inv_phi = d.inv_phi0; c.cd = d.cd0; c.cf = d.cf0;
        c.cdh = d.cd0h; c.cfh = d.cf0h;
        return c;
    }
    if (d.medium == MED_PHI_ERGUN && d.Fconst < 0.0f) {
        ergun_closed(d, phi, c);
        return c;
    }
    const float ip = hw_rcp(phi);
    c.phi = phi; c.inv_phi = ip;
    float kappa;
    if (d.medium == MED_PHI_ERGUN) {
        const float om = 1.0f - phi;
        kappa = d.kcoef * (om * om) * (ip * ip * ip);   // 1/K of Eq. (4)
    } else {
        kappa = kappa_plane;
    }
    const float F = (d.Fconst >= 0.0f) ? d.Fconst : ergun_F(ip);
    c.cd = phi * d.nu * kappa;
    c.cf = phi * F * hw_sqrt(kappa);
    c.cdh = 0.5f * c.cd;
    c.cfh = 0.5f * c.cf;
    return c;
}

// A node with its own viscosity ratio J (partially porous domains, where the
// porous part has nu_e = J nu and the free fluid nu_e = nu) relaxes its stress
// moments at its own rate; the plane holds s_nu and 1 - s_nu/2 follows here.
__device__ __forceinline__ void cell_viscosity(const Dom &d, Cell &c, int64_t idx) {
    if (d.snu) {
        const float s = d.snu[idx];
        c.s_nu = s;
        c.h_nu = 1.0f - 0.5f * s;
        c.h_nu2 = 2.0f - s;
        c.h_nu4 = fmaf(-2.0f, s, 4.0f);
    }
}

__device__ __forceinline__ Cell load_cell(const Dom &d, int64_t idx) {
    Cell c = (d.medium == MED_UNIFORM)
                 ? cell_from(d, 0.0f, 0.0f)
                 : cell_from(d, d.phi[idx], d.medium == MED_PHI_KAPPA ? d.kappa[idx] : 0.0f);
    cell_viscosity(d, c, idx);
    return c;
}

// Eqs. (18)-(19) in cancellation-free form. With d = cd/2, l0 = (1 + d)/2,
// l1 = cf/2, s = sqrt(l0^2 + l1|v|) and w = l0 + s, the denominator of Eq. (18)
// is w, and w^2 = (1 + d) w + l1|v|, so u = v / w = v - v q with
// q = 1 - 1/w = (d w + l1|v|) / w^2 = r (d + l1|v| r), r = 1/w: a sum of
// non-negative terms, so the small drag terms keep full relative precision
// instead of being rounded against 1 (one reciprocal). |u| = |v| (1 - q)
// comes with it.
__device__ __forceinline__ void velocity(const Cell &c, float vx, float vy, float &ux, float &uy,
                                         float &umag) {
    const float l0 = fmaf(0.5f, c.cdh, 0.5f);
    const float vmag = hw_sqrt(fmaf(vx, vx, vy * vy));
    const float t = c.cfh * vmag;
    const float r = hw_rcp(l0 + hw_sqrt(fmaf(l0, l0, t)));
    const float q = r * fmaf(t, r, c.cdh);
    ux = fmaf(-vx, q, vx);
    uy = fmaf(-vy, q, vy);
    umag = fmaf(-vmag, q, vmag);
}

__device__ __forceinline__ void velocity(const Cell &c, float vx, float vy, float &ux, float &uy) {
    float umag;
    velocity(c, vx, vy, ux, uy, umag);
}

// Moments m_1, m_3, m_5 of the deviations (rows 1, 3, 5 of Eq. 10).
__device__ __forceinline__ void conserved_moments(const float f[8], float &m1, float &m3,
                                                  float &m5) {
    const float a = f[0] + f[2], b = f[1] + f[3], cc = f[4] + f[6], dg = f[5] + f[7];
    const float x13 = f[0] - f[2], y24 = f[1] - f[3], p57 = f[4] - f[6], q68 = f[5] - f[7];
    m1 = (a + b) + (cc + dg);
    m3 = x13 + (p57 - q68);
    m5 = y24 + (p57 + q68);
}

// Velocity of a node from its pre-collision deviations (Eqs. 17-19);
// paxh/payh = phi * a / 2 (half the external force per unit mass).
__device__ __forceinline__ void node_velocity_h(const float f[8], const Cell &c, float paxh,
                                                float payh, float &ux, float &uy, float &m1) {
    float m3, m5;
    conserved_moments(f, m1, m3, m5);
    velocity(c, m3 + paxh, m5 + payh, ux, uy);
}

// The same with the full force pax/pay = phi * a (halving is exact).
__device__ __forceinline__ void node_velocity(const float f[8], const Cell &c, float pax,
                                              float pay, float &ux, float &uy, float &m1) {
    node_velocity_h(f, c, 0.5f * pax, 0.5f * pay, ux, uy, m1);
}

// One node's collision (Eq. 14) followed by f+ = M^-1 m+, in place on the
// deviations. Returns u. paxh/payh = phi * a / 2 (a may include buoyancy).
// Also returns the non-equilibrium stress moments n7 = m7 - m7^eq and
// n8 = m8 - m8^eq before relaxation (dropped by the compiler when unused).
// The step works on half forces Fh = F/2 (Eq. 3 scaled by 1/2: every drag and
// force term is an exact power-of-two multiple of the full one), which the
// forcing of Eq. (16) takes with doubled rates.
__device__ __forceinline__ void collide_h(float f[8], const Dom &d, const Cell &c, float paxh,
                                          float payh, float &ux, float &uy, float &n7, float &n8) {
    // m = M f (Eq. 8, rows of Eq. 10), shared sums first
    const float a = f[0] + f[2], b = f[1] + f[3], cc = f[4] + f[6], dg = f[5] + f[7];
    const float x13 = f[0] - f[2], y24 = f[1] - f[3], p57 = f[4] - f[6], q68 = f[5] - f[7];
    const float ab = a + b, cdg = cc + dg;
    const float m1 = ab + cdg;
    const float m2 = cdg - ab;
    const float pmq = p57 - q68, ppq = p57 + q68;
    const float m3 = x13 + pmq;
    const float m4 = fmaf(-2.0f, x13, pmq);
    const float m5 = y24 + ppq;
    const float m6 = fmaf(-2.0f, y24, ppq);
    const float m7 = a - b;
    const float m8 = cc - dg;

    // velocity (Eqs. 18-19) and half the total force (Eq. 3)
    float umag;
    velocity(c, m3 + paxh, m5 + payh, ux, uy, umag);
    const float dragh = fmaf(c.cfh, umag, c.cdh);
    const float Fx = fmaf(-dragh, ux, paxh);   // F_x / 2
    const float Fy = fmaf(-dragh, uy, payh);   // F_y / 2

    // relaxation toward m^eq (Eqs. 11-12) with forcing (Eq. 16); every 1/phi term
    // is formed from u/phi, so the products uy uy/phi, uy Fy/phi, uy Fx/phi serve
    // two terms each
    const float ip = c.inv_phi;
    const float uxi = ux * ip, uyi = uy * ip;  // u / phi
    const float yyi = uy * uyi, yFyi = uyi * Fy, yFxi = uyi * Fx;
    const float u2i = fmaf(ux, uxi, yyi);      // |u|^2 / phi
    const float uFi = fmaf(uxi, Fx, yFyi);     // u . F / (2 phi)
    // e - e^eq = dm2 + (3/5) dm1 - (2/5)|u|^2/phi  (Pi from Eq. 20, alpha2 = -1, gamma2 = 0);
    // e enters neither m1 nor j of f+, so single-rounded constants suffice here
    const float ne = fmaf(-0.4f, u2i, fmaf(0.6f, m1, m2));
    // S_2 = (4/5) u . F / phi: (1 - s_e/2) 4/5 S_2 = h_e16 (u . F/2) / phi
    const float m2p = fmaf(d.h_e16, uFi, fmaf(-d.s_e, ne, m2));
    // s1 = s3 = s5 = 1: m1+ = m1, j+ = rho0 u + F/2
    const float m3p = ux + Fx;
    const float m5p = uy + Fy;
    // q^eq = -u (c1 = c2 = -2), S_4 = -F_x (and S_6 = -F_y)
    const float m4p = fmaf(-d.h_q2, Fx, fmaf(-d.s_q, m4 + ux, m4));
    const float m6p = fmaf(-d.h_q2, Fy, fmaf(-d.s_q, m6 + uy, m6));
    // p_xx^eq = (ux^2 - uy^2)/phi, p_xy^eq = ux uy / phi (gamma1 = gamma3 = 2/3);
    // S_7 = 2 (ux Fx - uy Fy)/phi and S_8 = (ux Fy + uy Fx)/phi, in half forces
    const float pxx = fmaf(ux, uxi, -yyi);
    const float pxy = ux * uyi;
    const float Sxx4 = fmaf(uxi, Fx, -yFyi);   // S_7 / 4
    const float Sxy2 = fmaf(uxi, Fy, yFxi);    // S_8 / 2
    n7 = m7 - pxx;
    n8 = m8 - pxy;
    const float m7p = fmaf(c.h_nu4, Sxx4, fmaf(-c.s_nu, n7, m7));
    const float m8p = fmaf(c.h_nu2, Sxy2, fmaf(-c.s_nu, n8, m8));

    // f+ = M^T diag(1/8, 1/8, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m+; the 1/6 of the
    // momentum rows goes through the split constant (their rounding would bias
    // the momentum every step). The 1/12 of the energy-flux rows (which cancel
    // from mass and momentum) and the 1/4 of the stress rows are folded into the
    // fused multiply-adds that form the terms shared by two populations (with
    // X = j+_x/6 and Q_x = q+_x/12: X - 2 Q_x, X + Q_x, (A - B) +- m+_7/4,
    // (Y + Q_y) +- m+_8/4). Every population itself ends in an add, so no
    // kernel variant can merge its last rounding with the conversion to a
    // binary16 store (a mixed-precision multiply-add rounds once where the
    // separate instructions round twice).
    const float B = 0.125f * m2p;
    const float X = mulc(m3p, MRT_C1_6);
    const float Y = mulc(m5p, MRT_C1_6);
    const float amb = fmaf(0.125f, m1, -B), apb = fmaf(0.125f, m1, B);   // m1/8 -+ m2+/8
    const float xa = fmaf(-0x1.555556p-3f, m4p, X), ya = fmaf(-0x1.555556p-3f, m6p, Y);   // X - 2 Q
    const float xd = fmaf(0x1.555556p-4f, m4p, X), yd = fmaf(0x1.555556p-4f, m6p, Y);     // X + Q
    const float pa = fmaf(0.25f, m7p, amb), pm = fmaf(-0.25f, m7p, amb);   // A - B +- m+_7/4
    const float ypr = fmaf(0.25f, m8p, yd), ymr = fmaf(-0.25f, m8p, yd);   // Y + Q_y +- m+_8/4
    f[0] = pa + xa;
    f[2] = pa - xa;
    f[1] = pm + ya;
    f[3] = pm - ya;
    f[4] = (apb + xd) + ypr;
    f[5] = (apb - xd) + ymr;
    f[6] = (apb - xd) - ymr;
    f[7] = (apb + xd) - ypr;
}

// The same with the full force pax/pay = phi * a.
__device__ __forceinline__ void collide(float f[8], const Dom &d, const Cell &c, float pax,
                                        float pay, float &ux, float &uy, float &n7, float &n8) {
    collide_h(f, d, c, 0.5f * pax, 0.5f * pay, ux, uy, n7, n8);
}

__device__ __forceinline__ void collide(float f[8], const Dom &d, const Cell &c, float pax,
                                        float pay, float &ux, float &uy) {
    float n7, n8;
    collide(f, d, c, pax, pay, ux, uy, n7, n8);
}

// D2Q5 collision (Eq. B.2) on deviations dg = g - wT T0 (varpi = 0, so the
// rest distribution is T0/5 on every link), using the flow velocity u.
__device__ __forceinline__ void thermal_collide(float g[5], const Dom &d, float ux, float uy) {
    // n = N g (Eq. B.4)
    const float n0 = (g[0] + g[1]) + (g[2] + g[3]) + g[4];   // dT
    const float n1 = g[1] - g[3];
    const float n2 = g[2] - g[4];
    const float n3 = (g[1] + g[2]) + (g[3] + g[4]) - 4.0f * g[0];
    const float n4 = (g[1] - g[2]) + (g[3] - g[4]);
    const float T = d.T0 + n0;
    // n^eq = (T, ux T/sigma, uy T/sigma, varpi T, 0) with varpi = 0 (Eq. B.6)
    const float n1p = fmaf(-d.zT, n1 - ux * T * d.inv_sigma, n1);
    const float n2p = fmaf(-d.zT, n2 - uy * T * d.inv_sigma, n2);
    const float n3p = n3 - d.z3 * n3;
    const float n4p = n4 - d.z4 * n4;
    // g+ = N^T diag(1/5, 1/2, 1/2, 1/20, 1/4) n+
    const float a0 = mulc(n0, MRT_C1_5), a1 = 0.5f * n1p, a2 = 0.5f * n2p, a3 = mulc(n3p, MRT_C1_20),
                a4 = 0.25f * n4p;
    g[0] = a0 - 4.0f * a3;
    g[1] = (a0 + a3) + (a1 + a4);
    g[2] = (a0 + a3) + (a2 - a4);
    g[3] = (a0 + a3) - (a1 - a4);
    g[4] = (a0 + a3) - (a2 + a4);
}

// ---- storage ----------------------------------------------------------

template <typename S> struct Store;
template <> struct Store<float> {
    __device__ __forceinline__ static float ld(const float *p) { return *p; }
    __device__ __forceinline__ static void st(float *p, float v) { *p = v; }
};
template <> struct Store<_Float16> {
    __device__ __forceinline__ static float ld(const _Float16 *p) { return (float)(*p); }
    __device__ __forceinline__ static void st(_Float16 *p, float v) { *p = (_Float16)v; }
};

// NX consecutive values of a row; p is aligned to the element size only (the
// x-shifted planes start one element off a vector boundary).
template <typename S, int NX>
__device__ __forceinline__ void load_row(const S *p, float out[NX]) {
    S tmp[NX];
    __builtin_memcpy(tmp, p, sizeof(S) * NX);
#pragma unroll
    for (int k = 0; k < NX; ++k) out[k] = (float)tmp[k];
}

// NX consecutive values of a row to an address aligned to NX elements.
template <typename S, int NX>
__device__ __forceinline__ void store_row(S *p, const float in[NX]) {
    S tmp[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) tmp[k] = (S)in[k];
    S *q = (S *)__builtin_assume_aligned(p, sizeof(S) * NX);
    __builtin_memcpy(q, tmp, sizeof(S) * NX);
}

// The same values stored non-temporally (streaming past the caches).
template <typename S, int NX>
__device__ __forceinline__ void store_row_nt(S *p, const float in[NX]) {
    S *q = (S *)__builtin_assume_aligned(p, sizeof(S) * NX);
#pragma unroll
    for (int k = 0; k < NX; ++k) __builtin_nontemporal_store((S)in[k], q + k);
}

// ---- raw buffer access ------------------------------------------------

// CDNA buffer instructions: a 128-bit resource (base and byte size) lives in
// scalar registers, each lane adds a 32-bit byte offset and the wave a
// uniform one, so a gather of eight planes costs one vector offset instead of
// eight 64-bit address computations. Reads beyond the size return 0 and
// stores beyond it are dropped. Only for arrays below 4 GiB.
typedef __amdgpu_buffer_rsrc_t BufRes;

__device__ __forceinline__ BufRes buf_res(const void *base, uint32_t bytes) {
    // word 3 of the resource for gfx9-family raw (unformatted, unswizzled) access
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// Cache-policy operand of the buffer instructions: the non-temporal bit.
constexpr int CPOL_NT = 2;

template <typename S> struct BufIO;
template <> struct BufIO<float> {
    __device__ __forceinline__ static float ld(BufRes r, uint32_t vo, uint32_t so) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
    }
    __device__ __forceinline__ static void st(BufRes r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, (int)so, 0);
    }
    // non-temporal (streaming) store: the line is not kept in the caches
    __device__ __forceinline__ static void st_nt(BufRes r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, (int)so, CPOL_NT);
    }
};
template <> struct BufIO<_Float16> {
    __device__ __forceinline__ static float ld(BufRes r, uint32_t vo, uint32_t so) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0);
        _Float16 x;
        __builtin_memcpy(&x, &h, 2);
        return (float)x;
    }
    __device__ __forceinline__ static void st(BufRes r, uint32_t vo, uint32_t so, float v) {
        const _Float16 x = (_Float16)v;
        unsigned short h;
        __builtin_memcpy(&h, &x, 2);
        __builtin_amdgcn_raw_buffer_store_b16(h, r, (int)vo, (int)so, 0);
    }
    __device__ __forceinline__ static void st_nt(BufRes r, uint32_t vo, uint32_t so, float v) {
        const _Float16 x = (_Float16)v;
        unsigned short h;
        __builtin_memcpy(&h, &x, 2);
        __builtin_amdgcn_raw_buffer_store_b16(h, r, (int)vo, (int)so, CPOL_NT);
    }
};

// Buffer resources over a domain's per-node medium planes (porosity, 1/K,
// s_nu), each NULL plane given size 0.
struct CellPlanes {
    BufRes phi, kappa, snu;
};

__device__ __forceinline__ CellPlanes cell_planes(const Dom &d) {
    const uint32_t pb = (uint32_t)(d.plane * 4);
    CellPlanes r;
    // an absent plane gets a zero-size resource over a valid base: its loads are
    // out of range and return 0 without a memory access
    const void *any = d.fin;
    r.phi = d.phi ? buf_res(d.phi, pb) : buf_res(any, 0u);
    r.kappa = d.kappa ? buf_res(d.kappa, pb) : buf_res(any, 0u);
    r.snu = d.snu ? buf_res(d.snu, pb) : buf_res(any, 0u);
    return r;
}

// The raw per-node medium values of a node (porosity, 1/K, s_nu plane entries),
// fetched early so that the loads are in flight while other work runs.
struct CellRaw {
    float phi, kappa, snu;
};

__device__ __forceinline__ CellRaw load_cell_raw(const Dom &d, const CellPlanes &pl, uint32_t o4) {
    CellRaw r{0.0f, 0.0f, 0.0f};
    if (d.medium != MED_UNIFORM) r.phi = BufIO<float>::ld(pl.phi, o4, 0u);
    if (d.medium == MED_PHI_KAPPA) r.kappa = BufIO<float>::ld(pl.kappa, o4, 0u);
    if (d.snu) r.snu = BufIO<float>::ld(pl.snu, o4, 0u);
    return r;
}

// Same values with unconditional loads (an absent plane reads 0 through its
// zero-size resource): three loads issue back to back, without branches. The
// three-cycle and two-step adjoint kernels, which fetch several nodes' values
// ahead, measured faster this way; the one- and two-cycle kernels measured
// faster with the branches (uniform media then load nothing).
__device__ __forceinline__ CellRaw load_cell_raw_all(const CellPlanes &pl, uint32_t o4) {
    return CellRaw{BufIO<float>::ld(pl.phi, o4, 0u), BufIO<float>::ld(pl.kappa, o4, 0u),
                   BufIO<float>::ld(pl.snu, o4, 0u)};
}

// Same values as load_cell.
__device__ __forceinline__ Cell cell_of(const Dom &d, const CellRaw &r) {
    Cell c = cell_from(d, r.phi, r.kappa);
    if (d.snu) {
        c.s_nu = r.snu;
        c.h_nu = 1.0f - 0.5f * r.snu;
        c.h_nu2 = 2.0f - r.snu;
        c.h_nu4 = fmaf(-2.0f, r.snu, 4.0f);
    }
    return c;
}

// Where a kernel gets its per-node medium values, fixed at compile time.
// MK_ANY: every medium, with an optional per-node s_nu plane (branch-free loads,
// absent planes read 0). MK_ERGUN: the Ergun medium with the closed-form drag
// and one s_nu for all nodes; only the porosity plane is read, and the kernel
// holds fewer scalars (with MK_ANY the other medium parameters and plane
// resources spill to vector lanes in the three-cycle kernel). Both give the
// same values for an Ergun medium.
// MK_BRANCHED: every medium with the loads of load_cell_raw (branches; uniform
// media load nothing), which the one- and two-cycle kernels measured faster.
// MK_UNIFORM: a uniform medium and one s_nu; nothing is loaded.
enum { MK_ANY = 0, MK_ERGUN = 1, MK_BRANCHED = 2, MK_UNIFORM = 3 };

// The specialised kind a domain allows (MK_ANY when none applies); kernels
// without an instantiation for it use their generic kind.
__host__ __device__ inline int medium_kind(const Dom &d) {
    if (d.snu) return MK_ANY;
    if (d.medium == MED_PHI_ERGUN && d.Fconst < 0.0f) return MK_ERGUN;
    if (d.medium == MED_UNIFORM) return MK_UNIFORM;
    return MK_ANY;
}

template <int MK> struct MediumSrc;
template <> struct MediumSrc<MK_ANY> {
    CellPlanes pl;
    __device__ explicit MediumSrc(const Dom &d) : pl(cell_planes(d)) {}
    __device__ CellRaw load(uint32_t o4) const { return load_cell_raw_all(pl, o4); }
    __device__ Cell cell(const Dom &d, const CellRaw &r) const { return cell_of(d, r); }
};
template <> struct MediumSrc<MK_BRANCHED> {
    CellPlanes pl;
    int32_t medium;
    bool snu;
    __device__ explicit MediumSrc(const Dom &d) : pl(cell_planes(d)), medium(d.medium), snu(d.snu != nullptr) {}
    __device__ CellRaw load(uint32_t o4) const {
        CellRaw r{0.0f, 0.0f, 0.0f};
        if (medium != MED_UNIFORM) r.phi = BufIO<float>::ld(pl.phi, o4, 0u);
        if (medium == MED_PHI_KAPPA) r.kappa = BufIO<float>::ld(pl.kappa, o4, 0u);
        if (snu) r.snu = BufIO<float>::ld(pl.snu, o4, 0u);
        return r;
    }
    __device__ Cell cell(const Dom &d, const CellRaw &r) const { return cell_of(d, r); }
};
template <> struct MediumSrc<MK_UNIFORM> {
    __device__ explicit MediumSrc(const Dom &) {}
    __device__ CellRaw load(uint32_t) const { return CellRaw{0.0f, 0.0f, 0.0f}; }
    __device__ Cell cell(const Dom &d, const CellRaw &) const { return cell_from(d, 0.0f, 0.0f); }
};
template <> struct MediumSrc<MK_ERGUN> {
    BufRes phi;
    __device__ explicit MediumSrc(const Dom &d) : phi(buf_res(d.phi, (uint32_t)(d.plane * 4))) {}
    __device__ CellRaw load(uint32_t o4) const { return CellRaw{BufIO<float>::ld(phi, o4, 0u), 0.0f, 0.0f}; }
    __device__ Cell cell(const Dom &d, const CellRaw &r) const {
        Cell c;
        c.s_nu = d.s_nu;
        c.h_nu = d.h_nu;
        c.h_nu2 = d.h_nu2;
        c.h_nu4 = d.h_nu4;
        ergun_closed(d, r.phi, c);
        return c;
    }
};

// ---- gather (pull streaming, Eq. 15, with boundaries) -----------------

// Wraps (gx, gy) on periodic axes; false for a node beyond a wall.
__device__ __forceinline__ bool wrap_node(const Dom &d, int &gx, int &gy) {
    if (gx < 0 || gx >= d.nx) {
        if (d.bc_x != BC_PERIODIC) return false;
        gx = ((gx % d.nx) + d.nx) % d.nx;
    }
    if (gy < 0 || gy >= d.ny) {
        if (d.bc_y != BC_PERIODIC) return false;
        gy = ((gy % d.ny) + d.ny) % d.ny;
    }
    return true;
}


// f_i(x, t) = f_i+(x - e_i, t-1); a link whose source lies beyond a wall is
// replaced by the node's own opposite post-collision population plus the
// moving-wall term 6 w_i (e_i . u_w) when the wall crossed is the top one.
template <typename S>
__device__ __forceinline__ void gather_general(const Dom &d, const S *__restrict__ fin, int x,
                                               int y, float f[8]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int sx = x - EX[i], sy = y - EY[i];
        bool out = false, top = false;
        if (EX[i] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else out = true;
        }
        if (EY[i] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else { out = true; top = (sy >= d.ny); }
        }
        if (!out) {
            f[i] = Store<S>::ld(fin + i * d.plane + (int64_t)sy * d.pitch + sx);
        } else {
            float v = Store<S>::ld(fin + OPP[i] * d.plane + (int64_t)y * d.pitch + x);
            if (top) v += (float)EX[i] * d.lid6;
            f[i] = v;
        }
    }
}

// gather_general through a buffer resource over the eight planes: one 32-bit
// offset per link instead of a 64-bit address, so no per-plane base pointers
// stay live in scalar registers (the state buffer is below 4 GiB).
template <typename S>
__device__ __forceinline__ void gather_general_buf(const Dom &d, BufRes rin, int x, int y, float f[8]) {
    constexpr uint32_t ES = sizeof(S);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int sx = x - EX[i], sy = y - EY[i];
        bool out = false, top = false;
        if (EX[i] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else out = true;
        }
        if (EY[i] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else { out = true; top = (sy >= d.ny); }
        }
        const uint32_t idx = out ? (uint32_t)(OPP[i] * d.plane + y * d.pitch + x)
                                 : (uint32_t)(i * d.plane + sy * d.pitch + sx);
        float v = BufIO<S>::ld(rin, idx * ES, 0u);
        if (top) v += (float)EX[i] * d.lid6;
        f[i] = v;
    }
}

template <typename S>
__device__ __forceinline__ void load_own(const Dom &d, const S *__restrict__ fin, int x, int y,
                                         float f[8]) {
    const int64_t o = (int64_t)y * d.pitch + x;
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = Store<S>::ld(fin + i * d.plane + o);
}

// D2Q5 gather: Dirichlet walls at x = 0 / x = nx by anti-bounce-back,
// adiabatic walls at y = 0 / y = ny by bounce-back.
__device__ __forceinline__ void gather_thermal(const Dom &d, const float *__restrict__ gin,
                                               int x, int y, bool interior, float g[5]) {
    const int64_t o = (int64_t)y * d.pitch + x;
    g[0] = gin[o];
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        if (interior) {
            g[j] = gin[j * d.plane + o - TYv[j] * d.pitch - TXv[j]];
            continue;
        }
        int sx = x - TXv[j], sy = y - TYv[j];
        int kind = 0;  // 0 stream, 1 bounce-back, 2 hot ABB, 3 cold ABB
        if (TXv[j] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else kind = (sx < 0) ? 2 : 3;
        }
        if (TYv[j] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else kind = 1;
        }
        if (kind == 0) {
            g[j] = gin[j * d.plane + (int64_t)sy * d.pitch + sx];
        } else {
            const float v = gin[TOPP[j] * d.plane + o];
            g[j] = (kind == 1) ? v : ((kind == 2) ? d.abbh - v : d.abbc - v);
        }
    }
}

// gather_thermal's edge form through a buffer resource over the five planes
// (below 4 GiB).
__device__ __forceinline__ void gather_thermal_buf(const Dom &d, BufRes rg, int x, int y, float g[5]) {
    const uint32_t o = (uint32_t)(y * d.pitch + x);
    g[0] = BufIO<float>::ld(rg, o * 4u, 0u);
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        int sx = x - TXv[j], sy = y - TYv[j];
        int kind = 0;  // 0 stream, 1 bounce-back, 2 hot ABB, 3 cold ABB
        if (TXv[j] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else kind = (sx < 0) ? 2 : 3;
        }
        if (TYv[j] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else kind = 1;
        }
        const uint32_t idx = kind == 0 ? (uint32_t)(j * d.plane + sy * d.pitch + sx)
                                       : (uint32_t)(TOPP[j] * d.plane) + o;
        const float v = BufIO<float>::ld(rg, idx * 4u, 0u);
        g[j] = (kind <= 1) ? v : ((kind == 2) ? d.abbh - v : d.abbc - v);
    }
}

__device__ __forceinline__ void load_own_thermal(const Dom &d, const float *__restrict__ gin,
                                                 int x, int y, float g[5]) {
    const int64_t o = (int64_t)y * d.pitch + x;
#pragma unroll
    for (int j = 0; j < 5; ++j) g[j] = gin[j * d.plane + o];
}

// ---- on-node walls: non-equilibrium extrapolation (Sec. 3, Ref. [40]) ----

// Whether (x, y) lies on an on-node wall, and the next node inward along the
// wall normal (diagonally inward at a corner), which is never a wall node
// (>= 3 nodes per BC_NEE axis).
__device__ __forceinline__ bool nee_wall(const Dom &d, int x, int y, int &bx, int &by) {
    const bool wx = d.bc_x == BC_NEE && (x == 0 || x == d.nx - 1);
    const bool wy = d.bc_y == BC_NEE && (y == 0 || y == d.ny - 1);
    bx = wx ? (x == 0 ? 1 : d.nx - 2) : x;
    by = wy ? (y == 0 ? 1 : d.ny - 2) : y;
    return wx || wy;
}

// Deviation of the equilibrium of Eq. (22) from the rest state 3 w_i Pi0 at
// phi p = Pi0 + dPi (rho0 = 1):
//   w_i [3 dPi + 3 e.u + (9/2)(e.u)^2/phi - (3/2)|u|^2/phi].
__device__ __forceinline__ void feq_dev(float dPi, float ux, float uy, float ip, float out[8]) {
    const float u2 = 1.5f * (ux * ux + uy * uy) * ip;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float eu = (float)EX[i] * ux + (float)EY[i] * uy;
        const float v = 3.0f * dPi + 3.0f * eu + 4.5f * eu * eu * ip - u2;
        out[i] = (i < 4) ? v * (1.0f / 9.0f) : v * (1.0f / 36.0f);
    }
}

// Deviation of g^eq = N^-1 n^eq (Eq. B.6, varpi = 0) from T0/5 per link:
// dT/5 on every link plus +-u T/(2 sigma) along the axis links.
__device__ __forceinline__ void geq_dev(const Dom &d, float dT, float ux, float uy, float out[5]) {
    const float b = 0.2f * dT, T = d.T0 + dT;
    const float hx = 0.5f * ux * T * d.inv_sigma, hy = 0.5f * uy * T * d.inv_sigma;
    out[0] = b;
    out[1] = b + hx;
    out[2] = b + hy;
    out[3] = b - hx;
    out[4] = b - hy;
}

// Rebuilds the populations f(t) (and g(t)) of a wall node from those of its
// inner neighbour B at the same time t >= 1 (B's own gather from the
// post-collision buffer fin):
//   f(O) = f^eq(Pi_B, u_w; phi_O) + [f(B) - f^eq(Pi_B, u_B; phi_B)],
// with Pi = phi p taken over from B, u_B from Eqs. (18)-(19) with B's force,
// u_w = (U_lid, 0) on the top wall away from on-node x walls and zero
// elsewhere; g likewise with T_w = Th / Tc on x walls and T_B on y walls.
template <typename S, bool THERMAL>
__device__ __forceinline__ void nee_fixup(const Dom &d, const S *__restrict__ fin, int x, int y,
                                          float f[8], float g[5]) {
    int bx, by;
    if (!nee_wall(d, x, y, bx, by)) return;
    float fB[8], gB[5];
    gather_general<S>(d, fin, bx, by, fB);
    const Cell cB = load_cell(d, (int64_t)by * d.pitch + bx);
    const Cell cO = load_cell(d, (int64_t)y * d.pitch + x);
    float ay = d.ay, dTB = 0.0f;
    if (THERMAL) {
        gather_thermal(d, d.gin, bx, by, false, gB);
        dTB = (gB[0] + gB[1]) + (gB[2] + gB[3]) + gB[4];
        ay = d.ay + d.gbeta * dTB;
    }
    float uxB, uyB, m1B;
    node_velocity(fB, cB, cB.phi * d.ax, cB.phi * ay, uxB, uyB, m1B);
    // Eq. (20) on deviations: dPi = (3/5)(dm1 - (2/3)|u|^2/phi)
    const float dPi = mulc(m1B, MRT_C3_5) - mulc((uxB * uxB + uyB * uyB) * cB.inv_phi, MRT_C2_5);
    const bool wx = d.bc_x == BC_NEE && (x == 0 || x == d.nx - 1);
    const float uw = (d.bc_y == BC_NEE && y == d.ny - 1 && !wx) ? d.lid_u : 0.0f;
    float eO[8], eB[8];
    feq_dev(dPi, uw, 0.0f, cO.inv_phi, eO);
    feq_dev(dPi, uxB, uyB, cB.inv_phi, eB);
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = eO[i] + (fB[i] - eB[i]);
    if (THERMAL) {
        const float dTw = wx ? (x == 0 ? d.dTh : d.dTc) : dTB;
        float hO[5], hB[5];
        geq_dev(d, dTw, uw, 0.0f, hO);
        geq_dev(d, dTB, uxB, uyB, hB);
#pragma unroll
        for (int j = 0; j < 5; ++j) g[j] = hO[j] + (gB[j] - hB[j]);
    }
}

}  // namespace mrt
