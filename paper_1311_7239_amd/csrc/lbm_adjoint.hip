// Hand-written discrete adjoint of the fused D2Q8 porous MRT-LB step
// (Liu & He, arXiv:1311.7239, Eqs. 3, 4, 14-19) for gfx950.
//
// Forward: f(t+1) = G(C(f(t); phi)), with C the per-node collision
// (moments, velocity recovery, drag forcing, relaxation, back-transform) and
// G the pull streaming with halfway bounce-back. For a loss L(u(T)):
//   a(T)   = (du/df)^T dL/du,            g = (du/dphi)^T dL/du
//   b(t)   = G^T a(t+1)                  (adjoint of the post-collision state)
//   a(t)   = (dC/df)^T b(t),             g += (dC/dphi)^T b(t)
// G^T is a pull in the opposite direction: b_i(x) = a_i(x + e_i), or a_ibar(x)
// when the link x -> x + e_i crosses a wall (the lid's constant drops out).
// The Jacobian of C depends on f only through u (m^eq and S depend on m_1
// linearly and on u), so each backward step needs u(x, t) and the medium,
// which the checkpointed recomputation records; never f itself.
#include <hip/hip_runtime.h>

#include "lbm_launch.h"

namespace mrt {

constexpr int ABLOCK = 256;

// Adjoints of the intermediate medium quantities: phi*a (per component),
// cd = phi nu kappa, cf = phi F sqrt(kappa), and 1/phi.
struct ParamBar {
    float pax, pay, cd, cf, ip;
    float s;   // adjoint of the node's s_nu (s_7 = s_8)
};

// Per-thread sums of the adjoints of the scalar parameters: nu, a_x, a_y and
// the lid velocity.
struct ThetaSum {
    float nu, ax, ay, lid;
};

// A node's share of dL/dnu, dL/da_x, dL/da_y at one step: a enters as phi a;
// nu enters the linear drag cd = phi nu / K (Eq. 3) and s_nu = 1/(1/2 + 3 J nu)
// (Eq. 21), whose derivative is -s_nu (1 - s_nu/2) / nu for any J.
__device__ __forceinline__ void theta_add(const Dom &d, const Cell &c, const ParamBar &pb, ThetaSum &ts) {
    ts.ax += c.phi * pb.pax;
    ts.ay += c.phi * pb.pay;
    ts.nu += (pb.cd * c.cd - pb.s * c.s_nu * c.h_nu) * d.inv_nu;
}

// The lid term of the bounce-back gather adds (U/6) e_ix to links 6 and 7
// of a top-row node (e_iy = -1), so a(t) there carries (a_7 - a_6)/6 to dL/dU.
__device__ __forceinline__ float lid_share(const Dom &d, int y, float a6, float a7) {
    return (d.bc_y == BC_WALLS && y == d.ny - 1) ? (a7 - a6) * (1.0f / 6.0f) : 0.0f;
}

// Adds the block's sums of ts to slot[0..3] in a fixed order (bitwise
// reproducible); every thread of the block calls it.
template <int NT>
__device__ __forceinline__ void block_theta_add(const ThetaSum &ts, double *slot) {
    __shared__ double red[NT / 64][4];
    double v[4] = {ts.nu, ts.ax, ts.ay, ts.lid};
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[w][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double acc = 0.0;
            for (int j = 0; j < NT / 64; ++j) acc += red[j][k];
            slot[k] += acc;
        }
    }
}

// y -> M^T y with the paper's M (Eq. 10); y in moment order.
__device__ __forceinline__ void apply_MT(const float y[8], float f[8]) {
    const float amb = y[0] - y[1], apb = y[0] + y[1];
    const float xa = y[2] - 2.0f * y[3], ya = y[4] - 2.0f * y[5];
    const float xd = y[2] + y[3], yd = y[4] + y[5];
    f[0] = (amb + xa) + y[6];
    f[2] = (amb - xa) + y[6];
    f[1] = (amb + ya) - y[6];
    f[3] = (amb - ya) - y[6];
    f[4] = (apb + xd) + (yd + y[7]);
    f[5] = (apb - xd) + (yd - y[7]);
    f[6] = (apb - xd) - (yd - y[7]);
    f[7] = (apb + xd) - (yd + y[7]);
}

// Reverse mode of the velocity recovery u = v / D(|v|), D = l0 + sqrt(l0^2 + l1|v|)
// (Eqs. 18-19), given the total adjoint ub of u. Writes vb and adds the
// adjoints of cd and cf (through l0 = (1 + cd/2)/2, l1 = cf/2).
__device__ __forceinline__ void velocity_adjoint(const Cell &c, float ux, float uy, float ubx,
                                                 float uby, float &vbx, float &vby,
                                                 ParamBar &pb) {
    const float umag = hw_sqrt(fmaf(ux, ux, uy * uy));
    const float l0 = fmaf(0.25f, c.cd, 0.5f);
    const float l1 = 0.5f * c.cf;
    const float R = fmaf(l1, umag, l0);   // sqrt(l0^2 + l1|v|) on the solution
    const float D = l0 + R;               // = 2 l0 + l1 |u|
    const float uub = fmaf(ux, ubx, uy * uby);
    const float rR = hw_rcp(R), rD = hw_rcp(D);
    const float corr = (umag > 0.0f) ? (0.5f * l1 * rR) * uub * hw_rcp(umag) : 0.0f;
    vbx = fmaf(-corr, ux, ubx) * rD;
    vby = fmaf(-corr, uy, uby) * rD;
    const float w = -0.25f * uub * rR;
    pb.cd += w;
    pb.cf += w * umag;
    pb.pax = fmaf(0.5f, vbx, pb.pax);
    pb.pay = fmaf(0.5f, vby, pb.pay);
}

// Reverse mode of one node's collision (Eq. 14 and f+ = M^-1 m+): given the
// adjoint b of f+, returns the adjoint a of the pre-collision f and the
// medium adjoints. u is the node's velocity at this time step.
// n7, n8: the node's non-equilibrium stress moments before relaxation (only
// the adjoint of s_nu uses them).
// ubx0, uby0: adjoint of u from outside the flow collision (the thermal
// equilibrium), added before the velocity recovery.
__device__ __forceinline__ void collide_adjoint(const float b[8], const Dom &d, const Cell &c,
                                                float pax, float pay, float ux, float uy,
                                                float n7, float n8, float a[8], ParamBar &pb,
                                                float ubx0 = 0.0f, float uby0 = 0.0f) {
    // mbar+ = diag(1/8, 1/8, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) M b
    const float A1 = b[0] + b[2], B1 = b[1] + b[3], C1 = b[4] + b[6], D1 = b[5] + b[7];
    const float x13 = b[0] - b[2], y24 = b[1] - b[3], p57 = b[4] - b[6], q68 = b[5] - b[7];
    const float pmq = p57 - q68, ppq = p57 + q68;
    const float P1 = 0.125f * ((A1 + B1) + (C1 + D1));
    const float P2 = 0.125f * ((C1 + D1) - (A1 + B1));
    const float P3 = mulc(x13 + pmq, MRT_C1_6);
    const float P4 = mulc(pmq - 2.0f * x13, MRT_C1_12);
    const float P5 = mulc(y24 + ppq, MRT_C1_6);
    const float P6 = mulc(ppq - 2.0f * y24, MRT_C1_12);
    const float P7 = 0.25f * (A1 - B1);
    const float P8 = 0.25f * (C1 - D1);

    // forward quantities on this node
    const float ip = c.inv_phi;
    const float umag = hw_sqrt(fmaf(ux, ux, uy * uy));
    const float drag = fmaf(c.cf, umag, c.cd);
    const float Fx = fmaf(-drag, ux, pax), Fy = fmaf(-drag, uy, pay);
    const float u2 = fmaf(ux, ux, uy * uy), uF = fmaf(ux, Fx, uy * Fy);

    float mb[8];
    mb[0] = fmaf(-0.6f * d.s_e, P2, P1);
    mb[1] = (1.0f - d.s_e) * P2;
    mb[3] = (1.0f - d.s_q) * P4;
    mb[5] = (1.0f - d.s_q) * P6;
    mb[6] = (1.0f - c.s_nu) * P7;
    mb[7] = (1.0f - c.s_nu) * P8;

    // u and F enter m2+, m3+..m8+ directly (Eqs. 11-12, 16)
    const float se8 = 0.8f * d.s_e, he8 = 0.8f * d.h_e, s = c.s_nu, h = c.h_nu;
    const float Q2 = P2 * ip, Q7 = P7 * ip, Q8 = P8 * ip;
    float ubx = fmaf(Q2, fmaf(se8, ux, he8 * Fx),
                     fmaf(Q7, fmaf(2.0f * s, ux, 2.0f * h * Fx), fmaf(Q8, fmaf(s, uy, h * Fy), fmaf(-d.s_q, P4, P3))));
    float uby = fmaf(Q2, fmaf(se8, uy, he8 * Fy),
                     fmaf(-Q7, fmaf(2.0f * s, uy, 2.0f * h * Fy), fmaf(Q8, fmaf(s, ux, h * Fx), fmaf(-d.s_q, P6, P5))));
    const float hQ8 = h * Q8;
    const float Fbx = fmaf(ux, fmaf(he8, Q2, 2.0f * h * Q7), fmaf(hQ8, uy, fmaf(0.5f, P3, -d.h_q * P4)));
    const float Fby = fmaf(uy, fmaf(he8, Q2, -2.0f * h * Q7), fmaf(hQ8, ux, fmaf(0.5f, P5, -d.h_q * P6)));
    const float sxx = fmaf(ux, Fx, -(uy * Fy)), sxy = fmaf(ux, Fy, uy * Fx);
    // m7+ = m7 - s (m7 - m7^eq) + (1 - s/2) S7 (and m8+ alike): d/ds = -n7 - S7/2
    pb.s = fmaf(P7, -n7 - sxx * ip, P8 * (-n8 - 0.5f * sxy * ip));
    pb.ip = fmaf(fmaf(0.4f * d.s_e, u2, he8 * uF), P2,
                 fmaf(fmaf(s, fmaf(ux, ux, -(uy * uy)), 2.0f * h * sxx), P7, fmaf(s, ux * uy, h * sxy) * P8));

    // F = phi a - (cd + cf |u|) u  (Eq. 3)
    const float uFb = fmaf(ux, Fbx, uy * Fby);
    const float nl = (umag > 0.0f) ? c.cf * uFb * hw_rcp(umag) : 0.0f;
    ubx = fmaf(-drag, Fbx, fmaf(-nl, ux, ubx)) + ubx0;
    uby = fmaf(-drag, Fby, fmaf(-nl, uy, uby)) + uby0;
    pb.pax = Fbx;
    pb.pay = Fby;
    pb.cd = -uFb;
    pb.cf = -umag * uFb;

    float vbx, vby;
    velocity_adjoint(c, ux, uy, ubx, uby, vbx, vby, pb);
    mb[2] = vbx;
    mb[4] = vby;
    apply_MT(mb, a);
}

// d cd / d phi and d cf / d phi of a node (Eqs. 3-4; zero without a porosity plane).
template <int MK = MK_ANY>
__device__ __forceinline__ void cell_phi_derivs(const Dom &d, const Cell &c, float kappa, float &dcd,
                                                float &dcf) {
    const float phi = c.phi, ip = c.inv_phi;
    if (MK == MK_ERGUN || (d.medium == MED_PHI_ERGUN && d.Fconst < 0.0f)) {
        // the closed forms cd = (150 nu/dp^2)(1-phi)^2/phi^2, cf = (1.75/dp)(1-phi)/phi^2
        const float om = 1.0f - phi, ip2 = ip * ip;
        dcd = -2.0f * d.cdk * om * ip2 * ip;
        dcf = -fmaf(2.0f * c.cf, ip, d.cfk * ip2);
    } else if (d.medium == MED_PHI_ERGUN) {
        // kappa = kcoef (1-phi)^2 / phi^3; sqrt(kappa) = sk (1 - phi)
        const float om = 1.0f - phi;
        const float sk = hw_sqrt(d.kcoef) * ip * hw_sqrt(ip);
        const float F = (d.Fconst >= 0.0f) ? d.Fconst : ergun_F(ip);
        dcd = -2.0f * d.nu * d.kcoef * om * (ip * ip * ip);
        dcf = ((d.Fconst >= 0.0f) ? -0.5f : -2.0f) * c.cf * ip - phi * F * sk;
    } else if (d.medium == MED_PHI_KAPPA) {
        const float F = (d.Fconst >= 0.0f) ? d.Fconst : ergun_F(ip);
        dcd = d.nu * kappa;
        dcf = ((d.Fconst >= 0.0f) ? 1.0f : -0.5f) * F * hw_sqrt(kappa);
    } else {
        dcd = 0.0f;
        dcf = 0.0f;
    }
}

// Medium adjoints -> dL/dphi (and dL/dkappa with a kappa plane).
template <int MK = MK_ANY>
__device__ __forceinline__ void medium_gradient(const Dom &d, const Cell &c, float kappa,
                                                const ParamBar &pb, float ax, float ay,
                                                float &gphi, float &gkappa) {
    const float phi = c.phi, ip = c.inv_phi;
    float dcd, dcf;
    cell_phi_derivs<MK>(d, c, kappa, dcd, dcf);
    gkappa = 0.0f;
    if (MK == MK_ANY && d.medium == MED_PHI_KAPPA) {
        const float F = (d.Fconst >= 0.0f) ? d.Fconst : ergun_F(ip);
        const float sq = hw_sqrt(kappa);
        const float dcf_dk = (kappa > 0.0f) ? 0.5f * phi * F * hw_rcp(sq) : 0.0f;
        gkappa = pb.cd * phi * d.nu + pb.cf * dcf_dk;
    }
    gphi = ax * pb.pax + ay * pb.pay + pb.cd * dcd + pb.cf * dcf - pb.ip * ip * ip;
}

__device__ __forceinline__ float kappa_at(const Dom &d, int64_t o) {
    return d.medium == MED_PHI_KAPPA ? d.kappa[o] : 0.0f;
}

// a(T) and the direct medium gradient of u(T), from f(T) and dL/du(T). With
// THETA the block also adds its share of the parameter gradients to acc.
template <int SRC_T, bool THETA>
__global__ __launch_bounds__(ABLOCK) void k_adjoint_seed(Dom d, const float *__restrict__ dLdu,
                                                         float *__restrict__ lam,
                                                         float *__restrict__ gphi,
                                                         float *__restrict__ gkappa,
                                                         double *__restrict__ acc) {
    const int x = blockIdx.x * ABLOCK + threadIdx.x, y = blockIdx.y;
    ThetaSum ts{0.0f, 0.0f, 0.0f, 0.0f};
    if (x < d.nx) {
        float f[8];
        if (SRC_T == SRC_DIRECT) load_own<float>(d, (const float *)d.fin, x, y, f);
        else gather_general<float>(d, (const float *)d.fin, x, y, f);
        const int64_t o = (int64_t)y * d.pitch + x;
        const Cell c = load_cell(d, o);
        const float pax = c.phi * d.ax, pay = c.phi * d.ay;
        float ux, uy, m1;
        node_velocity(f, c, pax, pay, ux, uy, m1);
        const int64_t q = (int64_t)y * d.nx + x, n = (int64_t)d.nx * d.ny;
        ParamBar pb{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float vbx, vby;
        velocity_adjoint(c, ux, uy, dLdu[q], dLdu[n + q], vbx, vby, pb);
#pragma unroll
        for (int i = 0; i < 8; ++i) lam[i * d.plane + o] = (float)EX[i] * vbx + (float)EY[i] * vby;
        float gp, gk;
        medium_gradient(d, c, kappa_at(d, o), pb, d.ax, d.ay, gp, gk);
        gphi[o] = gp;
        if (gkappa) gkappa[o] = gk;
        if (THETA) theta_add(d, c, pb, ts);
    }
    if (THETA) block_theta_add<ABLOCK>(ts, acc + 4 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x));
}

__device__ __forceinline__ void gather_transposed(const Dom &d, const float *__restrict__ lam, int x,
                                                  int y, bool interior, float b[8]);

// One backward step at time t: lam_out = a(t), lam_in = a(t+1), u_t = u(t)
// (with THETA also the stress moments n7, n8 in planes 2 and 3).
template <bool THETA>
__global__ __launch_bounds__(ABLOCK) void k_adjoint_step(Dom d, const float *__restrict__ lam_in,
                                                         float *__restrict__ lam_out,
                                                         const float *__restrict__ u_t,
                                                         float *__restrict__ gphi,
                                                         float *__restrict__ gkappa,
                                                         int tiles_x, double *__restrict__ acc) {
    const int tx = blockIdx.x % tiles_x, y = blockIdx.x / tiles_x;
    const int x = tx * ABLOCK + threadIdx.x;
    ThetaSum ts{0.0f, 0.0f, 0.0f, 0.0f};
    if (x < d.nx) {
        const int64_t o = (int64_t)y * d.pitch + x;
        const bool interior = tx * ABLOCK >= 1 && tx * ABLOCK + ABLOCK <= d.nx - 1 && y >= 1 &&
                              y <= d.ny - 2;
        float b[8];
        gather_transposed(d, lam_in, x, y, interior, b);
        const Cell c = load_cell(d, o);
        const float ux = u_t[o], uy = u_t[d.plane + o];
        const float n7 = THETA ? u_t[2 * d.plane + o] : 0.0f, n8 = THETA ? u_t[3 * d.plane + o] : 0.0f;
        float a[8];
        ParamBar pb;
        collide_adjoint(b, d, c, c.phi * d.ax, c.phi * d.ay, ux, uy, n7, n8, a, pb);
#pragma unroll
        for (int i = 0; i < 8; ++i) lam_out[i * d.plane + o] = a[i];
        float gp, gk;
        medium_gradient(d, c, kappa_at(d, o), pb, d.ax, d.ay, gp, gk);
        gphi[o] += gp;
        if (gkappa) gkappa[o] += gk;
        if (THETA) {
            theta_add(d, c, pb, ts);
            if (y == d.ny - 1) ts.lid += lid_share(d, y, lam_in[6 * d.plane + o], lam_in[7 * d.plane + o]);
        }
    }
    if (THETA) block_theta_add<ABLOCK>(ts, acc + 4 * (int64_t)blockIdx.x);
}

// b_i(x) = a_i(x + e_i), or a_ibar(x) across a wall: the transpose of the
// pull gather, read from HBM for node (x, y).
__device__ __forceinline__ void gather_transposed(const Dom &d, const float *__restrict__ lam, int x,
                                                  int y, bool interior, float b[8]) {
    const int64_t o = (int64_t)y * d.pitch + x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (interior) {
            b[i] = lam[i * d.plane + o + EY[i] * d.pitch + EX[i]];
            continue;
        }
        int sx = x + EX[i], sy = y + EY[i];
        bool out = false;
        if (EX[i] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else out = true;
        }
        if (EY[i] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else out = true;
        }
        b[i] = out ? lam[OPP[i] * d.plane + o] : lam[i * d.plane + (int64_t)sy * d.pitch + sx];
    }
}

// gather_transposed's edge form through a buffer resource over the eight
// planes of a (below 4 GiB): 32-bit offsets, no per-plane base pointers.
__device__ __forceinline__ void gather_transposed_buf(const Dom &d, BufRes rlam, int x, int y, float b[8]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int sx = x + EX[i], sy = y + EY[i];
        bool out = false;
        if (EX[i] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else out = true;
        }
        if (EY[i] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else out = true;
        }
        const uint32_t idx = out ? (uint32_t)(OPP[i] * d.plane + y * d.pitch + x)
                                 : (uint32_t)(i * d.plane + sy * d.pitch + sx);
        b[i] = BufIO<float>::ld(rlam, idx * 4u, 0u);
    }
}

// Reverse mode of the D2Q5 collision (Eq. B.2 with varpi = 0, deviations from
// T0/5): given the adjoint bg of g+, the adjoint ag of the pre-collision g
// (through n = N g, T = T0 + n_0 and n^eq of Eq. B.6) and the adjoint of the
// flow velocity it uses, added to ubx, uby.
__device__ __forceinline__ void thermal_collide_adjoint(const float bg[5], const Dom &d, float ux, float uy,
                                                        float dT, float ag[5], float &ubx, float &uby) {
    // adjoint of n+: diag(1/5, 1/2, 1/2, 1/20, 1/4) N bg (g+ = N^T diag(...) n+)
    const float nb0 = 0.2f * ((bg[0] + bg[1]) + (bg[2] + bg[3]) + bg[4]);
    const float nb1 = 0.5f * (bg[1] - bg[3]);
    const float nb2 = 0.5f * (bg[2] - bg[4]);
    const float nb3 = 0.05f * ((bg[1] + bg[2]) + (bg[3] + bg[4]) - 4.0f * bg[0]);
    const float nb4 = 0.25f * ((bg[1] - bg[2]) + (bg[3] - bg[4]));
    const float T = d.T0 + dT;
    // n1+ = n1 - zT (n1 - ux T / sigma), T = T0 + n0; n0+ = n0; n3, n4 relax to 0
    const float nbar0 = nb0 + d.zT * (ux * nb1 + uy * nb2) * d.inv_sigma;
    const float nbar1 = (1.0f - d.zT) * nb1, nbar2 = (1.0f - d.zT) * nb2;
    const float nbar3 = (1.0f - d.z3) * nb3, nbar4 = (1.0f - d.z4) * nb4;
    ubx += d.zT * T * d.inv_sigma * nb1;
    uby += d.zT * T * d.inv_sigma * nb2;
    // ag = N^T nbar
    ag[0] = nbar0 - 4.0f * nbar3;
    ag[1] = (nbar0 + nbar1) + (nbar3 + nbar4);
    ag[2] = (nbar0 + nbar2) + (nbar3 - nbar4);
    ag[3] = (nbar0 - nbar1) + (nbar3 + nbar4);
    ag[4] = (nbar0 - nbar2) + (nbar3 - nbar4);
}

// gather_thermal_transposed's edge form through a buffer resource over the
// five planes of a_g (below 4 GiB).
__device__ __forceinline__ void gather_thermal_transposed_buf(const Dom &d, BufRes rg, int x, int y, float b[5]) {
    const uint32_t o = (uint32_t)(y * d.pitch + x);
    b[0] = BufIO<float>::ld(rg, o * 4u, 0u);
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        int sx = x + TXv[j], sy = y + TYv[j];
        int kind = 0;  // 0 stream, 1 bounce-back, 2 anti-bounce-back
        if (TXv[j] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else kind = 2;
        }
        if (TYv[j] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else kind = 1;
        }
        const uint32_t idx = kind == 0 ? (uint32_t)(j * d.plane + sy * d.pitch + sx)
                                       : (uint32_t)(TOPP[j] * d.plane) + o;
        const float v = BufIO<float>::ld(rg, idx * 4u, 0u);
        b[j] = (kind == 2) ? -v : v;
    }
}

// Two backward steps per pass: a(t) on a 64 x 16 tile plus a one-node ring
// from a(t+1) in HBM into LDS (phase A), then a(t-1) on the tile from LDS
// (phase B); the medium gradient of both steps is added in one
// read-modify-write, in the order of two single steps, so the result is
// bitwise that of two k_adjoint_step launches.
constexpr int ATW = 64, ATH = 16, ANT = 512;

template <bool THETA, int MK, bool THERMAL>
__global__ __launch_bounds__(ANT) __attribute__((amdgpu_waves_per_eu(THERMAL ? 4 : 6))) void k_adjoint_step2(
                                                       Dom d, const float *__restrict__ lam_in,
                                                       float *__restrict__ lam_out,
                                                       const float *__restrict__ lamg_in,
                                                       float *__restrict__ lamg_out,
                                                       const float *__restrict__ u_t,
                                                       const float *__restrict__ u_tm1,
                                                       float *__restrict__ gphi,
                                                       float *__restrict__ gkappa, int tiles_x,
                                                       int swz, double *__restrict__ acc) {
    constexpr int EW = ATW + 2, EH = ATH + 2, EN = EW * EH;
    constexpr int NB = (ATW * ATH + ANT - 1) / ANT;
    __shared__ float lds[8][EH][EW];
    __shared__ float ldsg[THERMAL ? 5 * EH * EW : 1];   // a_g(t) of the D2Q5 links
    __shared__ float gA[ATH][ATW];
    __shared__ float gkA[ATH][ATW];
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    const int x0 = (b % tiles_x) * ATW, y0 = (b / tiles_x) * ATH;
    const bool interior = x0 >= 2 && x0 + ATW + 2 <= d.nx && y0 >= 2 && y0 + ATH + 2 <= d.ny;
    // every buffer is below 4 GiB (the host runs two steps per pass only then):
    // byte offsets go through buffer resources
    const uint32_t pb4 = (uint32_t)(d.plane * 4);
    const BufRes rlin = buf_res(lam_in, 8 * pb4), rlout = buf_res(lam_out, 8 * pb4);
    const BufRes rut = buf_res(u_t, 5 * pb4), rutm = buf_res(u_tm1, 5 * pb4);
    const BufRes rg = buf_res(gphi, pb4), rgk = buf_res(gkappa, gkappa ? pb4 : 0u);
    const BufRes rgin = buf_res(THERMAL ? lamg_in : nullptr, THERMAL ? 5 * pb4 : 0u);
    const BufRes rgout = buf_res(THERMAL ? lamg_out : nullptr, THERMAL ? 5 * pb4 : 0u);
    const MediumSrc<MK> med(d);
    ThetaSum ts{0.0f, 0.0f, 0.0f, 0.0f};

    // phase A: a(t) on the tile plus a one-node ring, from a(t+1) in HBM
    auto finish_a = [&](float (&bb)[8], const float (&bg)[5], const CellRaw &r, const float (&uu)[4], float dT,
                        int ex, int ey, int gx, int gy) {
        const int64_t o = (int64_t)gy * d.pitch + gx;
        const Cell c = med.cell(d, r);
        float a[8];
        ParamBar pb;
        // thermal: the D2Q5 reverse mode first (it adds to the adjoint of u), then
        // the flow collision with the node's buoyancy, then the buoyancy's adjoint
        // returned to every thermal link
        float ag[5], ubx = 0.0f, uby = 0.0f;
        if (THERMAL) thermal_collide_adjoint(bg, d, uu[0], uu[1], dT, ag, ubx, uby);
        const float ay = THERMAL ? d.ay + d.gbeta * dT : d.ay;
        collide_adjoint(bb, d, c, c.phi * d.ax, c.phi * ay, uu[0], uu[1], uu[2], uu[3], a, pb, ubx, uby);
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[i][ey][ex] = a[i];
        if (THERMAL) {
            const float Tb = c.phi * d.gbeta * pb.pay;
#pragma unroll
            for (int j = 0; j < 5; ++j) ldsg[(j * EH + ey) * EW + ex] = ag[j] + Tb;
        }
        if (ex >= 1 && ex <= ATW && ey >= 1 && ey <= ATH && x0 - 1 + ex < d.nx && y0 - 1 + ey < d.ny) {
            float gp, gk;
            medium_gradient<MK>(d, c, r.kappa, pb, d.ax, ay, gp, gk);
            gA[ey - 1][ex - 1] = gp;
            gkA[ey - 1][ex - 1] = gk;
            if (THETA) {
                theta_add(d, c, pb, ts);
                if (gy == d.ny - 1) {
                    const uint32_t o4 = (uint32_t)(o * 4);
                    ts.lid += lid_share(d, gy, BufIO<float>::ld(rlin, o4, 6 * pb4), BufIO<float>::ld(rlin, o4, 7 * pb4));
                }
            }
        }
    };
    if (interior) {
        // b_i(x) = a_i(x + e_i): the lane's offset of (gx - 1, gy - 1) plus a uniform,
        // non-negative per-link offset; the next node's loads are issued before this
        // node's reverse-mode collision (software pipeline)
        auto fetch = [&](int e, float (&bb)[8], float (&bg)[5], CellRaw &r, float (&uu)[4], float &dT) {
            const int gx = x0 - 1 + e % EW, gy = y0 - 1 + e / EW;
            const uint32_t vo = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * 4);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                bb[i] = BufIO<float>::ld(rlin, vo, (uint32_t)((i * d.plane + (1 + EY[i]) * d.pitch + (1 + EX[i])) * 4));
            if (THERMAL) {
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    bg[j] = BufIO<float>::ld(rgin, vo, (uint32_t)((j * d.plane + (1 + TYv[j]) * d.pitch + (1 + TXv[j])) * 4));
            }
            const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
            r = med.load(o4);
            uu[0] = BufIO<float>::ld(rut, o4, 0u);
            uu[1] = BufIO<float>::ld(rut, o4, pb4);
            uu[2] = THETA ? BufIO<float>::ld(rut, o4, 2 * pb4) : 0.0f;
            uu[3] = THETA ? BufIO<float>::ld(rut, o4, 3 * pb4) : 0.0f;
            dT = THERMAL ? BufIO<float>::ld(rut, o4, 4 * pb4) : 0.0f;
        };
        float bn[8], gn[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, un[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dn = 0.0f;
        CellRaw rn{0.0f, 0.0f, 0.0f};
        if ((int)threadIdx.x < EN) fetch(threadIdx.x, bn, gn, rn, un, dn);
        for (int e = threadIdx.x; e < EN; e += ANT) {
            float bb[8], bg[5], uu[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) bb[i] = bn[i];
#pragma unroll
            for (int j = 0; j < 5; ++j) bg[j] = gn[j];
#pragma unroll
            for (int k = 0; k < 4; ++k) uu[k] = un[k];
            const CellRaw r = rn;
            const float dT = dn;
            if (e + ANT < EN) fetch(e + ANT, bn, gn, rn, un, dn);
            const int ex = e % EW, ey = e / EW;
            finish_a(bb, bg, r, uu, dT, ex, ey, x0 - 1 + ex, y0 - 1 + ey);
        }
    } else {
        for (int e = threadIdx.x; e < EN; e += ANT) {
            const int ex = e % EW, ey = e / EW;
            int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            if (gx < 0 || gx >= d.nx) {
                if (d.bc_x != BC_PERIODIC) continue;
                gx = ((gx % d.nx) + d.nx) % d.nx;
            }
            if (gy < 0 || gy >= d.ny) {
                if (d.bc_y != BC_PERIODIC) continue;
                gy = ((gy % d.ny) + d.ny) % d.ny;
            }
            float bb[8], bg[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            gather_transposed_buf(d, rlin, gx, gy, bb);
            if (THERMAL) gather_thermal_transposed_buf(d, rgin, gx, gy, bg);
            const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
            float uu[4] = {BufIO<float>::ld(rut, o4, 0u), BufIO<float>::ld(rut, o4, pb4), 0.0f, 0.0f};
            if (THETA) {
                uu[2] = BufIO<float>::ld(rut, o4, 2 * pb4);
                uu[3] = BufIO<float>::ld(rut, o4, 3 * pb4);
            }
            const float dT = THERMAL ? BufIO<float>::ld(rut, o4, 4 * pb4) : 0.0f;
            finish_a(bb, bg, med.load(o4), uu, dT, ex, ey, gx, gy);
        }
    }
    __syncthreads();

    // phase B: a(t-1) on the tile from LDS. The vector-memory counter retires
    // loads and stores in order, so both nodes' inputs are fetched before the
    // first node's stores.
    const float *flat = &lds[0][0][0];
    CellRaw rawB[NB];
    float uB[NB][4], dTB[NB], gB[NB], gkB[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int q = threadIdx.x + k * ANT;
        const int gx = x0 + q % ATW, gy = y0 + q / ATW;
        if (q >= ATW * ATH || gx >= d.nx || gy >= d.ny) continue;
        const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
        rawB[k] = med.load(o4);
        uB[k][0] = BufIO<float>::ld(rutm, o4, 0u);
        uB[k][1] = BufIO<float>::ld(rutm, o4, pb4);
        uB[k][2] = THETA ? BufIO<float>::ld(rutm, o4, 2 * pb4) : 0.0f;
        uB[k][3] = THETA ? BufIO<float>::ld(rutm, o4, 3 * pb4) : 0.0f;
        dTB[k] = THERMAL ? BufIO<float>::ld(rutm, o4, 4 * pb4) : 0.0f;
        gB[k] = BufIO<float>::ld(rg, o4, 0u);
        gkB[k] = gkappa ? BufIO<float>::ld(rgk, o4, 0u) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int q = threadIdx.x + k * ANT;
        if (q >= ATW * ATH) continue;
        const int lx = q % ATW, ly = q / ATW;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= d.nx || gy >= d.ny) continue;
        const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
        float bb[8];
        if (interior) {
            const int base = (ly + 1) * EW + lx + 1;
#pragma unroll
            for (int i = 0; i < 8; ++i) bb[i] = flat[base + i * EH * EW + EY[i] * EW + EX[i]];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                bool out = false;
                const int sx = gx + EX[i], sy = gy + EY[i];
                if (EX[i] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) out = true;
                if (EY[i] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) out = true;
                const int src = out ? (OPP[i] * EH + ly + 1) * EW + lx + 1
                                    : (i * EH + ly + 1 + EY[i]) * EW + lx + 1 + EX[i];
                bb[i] = flat[src];
            }
        }
        float bg[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (THERMAL) {
            // b_j(x) = a_g,j(x + e_j); across a wall the node's own opposite link,
            // with the sign flipped at the isothermal (anti-bounce-back) walls
            bg[0] = ldsg[(ly + 1) * EW + lx + 1];
#pragma unroll
            for (int j = 1; j < 5; ++j) {
                int kind = 0;
                if (!interior) {
                    const int sx = gx + TXv[j], sy = gy + TYv[j];
                    if (TXv[j] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) kind = 2;
                    if (TYv[j] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) kind = 1;
                }
                const int src = kind == 0 ? (j * EH + ly + 1 + TYv[j]) * EW + lx + 1 + TXv[j]
                                          : (TOPP[j] * EH + ly + 1) * EW + lx + 1;
                const float v = ldsg[src];
                bg[j] = kind == 2 ? -v : v;
            }
        }
        const Cell c = med.cell(d, rawB[k]);
        float a[8];
        ParamBar pb;
        float ag[5], ubx = 0.0f, uby = 0.0f;
        if (THERMAL) thermal_collide_adjoint(bg, d, uB[k][0], uB[k][1], dTB[k], ag, ubx, uby);
        const float ay = THERMAL ? d.ay + d.gbeta * dTB[k] : d.ay;
        collide_adjoint(bb, d, c, c.phi * d.ax, c.phi * ay, uB[k][0], uB[k][1], uB[k][2], uB[k][3], a, pb, ubx, uby);
#pragma unroll
        for (int i = 0; i < 8; ++i) BufIO<float>::st(rlout, o4, (uint32_t)i * pb4, a[i]);
        if (THERMAL) {
            const float Tb = c.phi * d.gbeta * pb.pay;
#pragma unroll
            for (int j = 0; j < 5; ++j) BufIO<float>::st(rgout, o4, (uint32_t)j * pb4, ag[j] + Tb);
        }
        float gp, gk;
        medium_gradient<MK>(d, c, rawB[k].kappa, pb, d.ax, ay, gp, gk);
        BufIO<float>::st(rg, o4, 0u, (gB[k] + gA[ly][lx]) + gp);
        if (gkappa) BufIO<float>::st(rgk, o4, 0u, (gkB[k] + gkA[ly][lx]) + gk);
        if (THETA) {
            theta_add(d, c, pb, ts);
            if (gy == d.ny - 1)
                ts.lid += lid_share(d, gy, lds[6][ly + 1][lx + 1], lds[7][ly + 1][lx + 1]);
        }
    }
    if (THETA) block_theta_add<ANT>(ts, acc + 4 * (int64_t)b);
}

// Three backward steps per pass, the adjoint of the three-cycle forward pass:
// a(t) on a 64 x 16 tile plus a two-node ring from a(t+1) in HBM into LDS
// (phase A), a(t-1) on the tile plus a one-node ring from LDS, kept in
// registers and written back to the same LDS in a smaller layout (phase B),
// then a(t-2) on the tile to HBM (phase C). The three steps' medium gradients
// of a tile node are added in one read-modify-write, in the order of three
// single steps, so the result is bitwise that of three k_adjoint_step
// launches. KAPPA: the gradient with respect to a 1/K plane is accumulated too.
template <bool THETA, int MK, bool KAPPA>
__global__ __launch_bounds__(ANT) __attribute__((amdgpu_waves_per_eu(KAPPA ? 4 : 6))) void k_adjoint_step3(
    Dom d, const float *__restrict__ lam_in, float *__restrict__ lam_out, const float *__restrict__ u_t,
    const float *__restrict__ u_tm1, const float *__restrict__ u_tm2, float *__restrict__ gphi,
    float *__restrict__ gkappa, int tiles_x, int swz, double *__restrict__ acc) {
    constexpr int AW = ATW + 4, AH = ATH + 4, AN = AW * AH;
    constexpr int BW = ATW + 2, BH = ATH + 2, BN = BW * BH;
    constexpr int NBB = (BN + ANT - 1) / ANT;
    constexpr int NC = (ATW * ATH + ANT - 1) / ANT;
    constexpr int NG = KAPPA ? 4 : 2;   // gradient partials of steps t and t-1 (phi, then 1/K)
    __shared__ float lds[8 * AH * AW];
    __shared__ float gpart[NG][ATH][ATW];
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    const int x0 = (b % tiles_x) * ATW, y0 = (b / tiles_x) * ATH;
    const bool interior = x0 >= 3 && x0 + ATW + 3 <= d.nx && y0 >= 3 && y0 + ATH + 3 <= d.ny;
    // every buffer is below 4 GiB (the host runs multi-step passes only then)
    const uint32_t pb4 = (uint32_t)(d.plane * 4);
    const BufRes rlin = buf_res(lam_in, 8 * pb4), rlout = buf_res(lam_out, 8 * pb4);
    const BufRes rg = buf_res(gphi, pb4), rgk = buf_res(KAPPA ? gkappa : nullptr, KAPPA ? pb4 : 0u);
    const MediumSrc<MK> med(d);
    ThetaSum ts{0.0f, 0.0f, 0.0f, 0.0f};

    // phase A: a(t) on the tile plus a two-node ring, from a(t+1) in HBM
    {
        const BufRes rut = buf_res(u_t, 5 * pb4);
        auto finish_a = [&](float (&bb)[8], const CellRaw &r, const float (&uu)[4], int ex, int ey, int gx,
                            int gy) {
            const Cell c = med.cell(d, r);
            float a[8];
            ParamBar pb;
            collide_adjoint(bb, d, c, c.phi * d.ax, c.phi * d.ay, uu[0], uu[1], uu[2], uu[3], a, pb);
#pragma unroll
            for (int i = 0; i < 8; ++i) lds[(i * AH + ey) * AW + ex] = a[i];
            if (ex >= 2 && ex < ATW + 2 && ey >= 2 && ey < ATH + 2 && x0 - 2 + ex < d.nx && y0 - 2 + ey < d.ny) {
                float gp, gk;
                medium_gradient<MK>(d, c, r.kappa, pb, d.ax, d.ay, gp, gk);
                gpart[0][ey - 2][ex - 2] = gp;
                if (KAPPA) gpart[KAPPA ? 2 : 0][ey - 2][ex - 2] = gk;
                if (THETA) {
                    theta_add(d, c, pb, ts);
                    if (gy == d.ny - 1) {
                        const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
                        ts.lid += lid_share(d, gy, BufIO<float>::ld(rlin, o4, 6 * pb4),
                                            BufIO<float>::ld(rlin, o4, 7 * pb4));
                    }
                }
            }
        };
        if (interior) {
            // b_i(x) = a_i(x + e_i) at constant per-link offsets; the next node's loads
            // are issued before this node's reverse-mode collision
            auto fetch = [&](int e, float (&bb)[8], CellRaw &r, float (&uu)[4]) {
                const int gx = x0 - 2 + e % AW, gy = y0 - 2 + e / AW;
                const uint32_t vo = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * 4);
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    bb[i] = BufIO<float>::ld(rlin, vo, (uint32_t)((i * d.plane + (1 + EY[i]) * d.pitch + (1 + EX[i])) * 4));
                const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
                r = med.load(o4);
                uu[0] = BufIO<float>::ld(rut, o4, 0u);
                uu[1] = BufIO<float>::ld(rut, o4, pb4);
                uu[2] = THETA ? BufIO<float>::ld(rut, o4, 2 * pb4) : 0.0f;
                uu[3] = THETA ? BufIO<float>::ld(rut, o4, 3 * pb4) : 0.0f;
            };
            float bn[8], un[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            CellRaw rn{0.0f, 0.0f, 0.0f};
            if ((int)threadIdx.x < AN) fetch(threadIdx.x, bn, rn, un);
            for (int e = threadIdx.x; e < AN; e += ANT) {
                float bb[8], uu[4];
#pragma unroll
                for (int i = 0; i < 8; ++i) bb[i] = bn[i];
#pragma unroll
                for (int k = 0; k < 4; ++k) uu[k] = un[k];
                const CellRaw r = rn;
                if (e + ANT < AN) fetch(e + ANT, bn, rn, un);
                const int ex = e % AW, ey = e / AW;
                finish_a(bb, r, uu, ex, ey, x0 - 2 + ex, y0 - 2 + ey);
            }
        } else {
            for (int e = threadIdx.x; e < AN; e += ANT) {
                const int ex = e % AW, ey = e / AW;
                int gx = x0 - 2 + ex, gy = y0 - 2 + ey;
                if (!wrap_node(d, gx, gy)) continue;
                float bb[8];
                gather_transposed_buf(d, rlin, gx, gy, bb);
                const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
                float uu[4] = {BufIO<float>::ld(rut, o4, 0u), BufIO<float>::ld(rut, o4, pb4), 0.0f, 0.0f};
                if (THETA) {
                    uu[2] = BufIO<float>::ld(rut, o4, 2 * pb4);
                    uu[3] = BufIO<float>::ld(rut, o4, 3 * pb4);
                }
                finish_a(bb, med.load(o4), uu, ex, ey, gx, gy);
            }
        }
    }
    __syncthreads();

    // phase B: a(t-1) on the tile plus a one-node ring, from LDS, kept in registers
    float ab[NBB][8];
    int slot[NBB];
    {
        const BufRes rutm = buf_res(u_tm1, 5 * pb4);
        CellRaw rawB[NBB];
        float uB[NBB][4];
#pragma unroll
        for (int k = 0; k < NBB; ++k) {
            slot[k] = -1;
            const int e = threadIdx.x + k * ANT;
            if (e >= BN) continue;
            int gx = x0 - 1 + e % BW, gy = y0 - 1 + e / BW;
            if (!interior && !wrap_node(d, gx, gy)) continue;
            const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
            rawB[k] = med.load(o4);
            uB[k][0] = BufIO<float>::ld(rutm, o4, 0u);
            uB[k][1] = BufIO<float>::ld(rutm, o4, pb4);
            uB[k][2] = THETA ? BufIO<float>::ld(rutm, o4, 2 * pb4) : 0.0f;
            uB[k][3] = THETA ? BufIO<float>::ld(rutm, o4, 3 * pb4) : 0.0f;
            slot[k] = e;
        }
#pragma unroll
        for (int k = 0; k < NBB; ++k) {
            if (slot[k] < 0) continue;
            const int bx = slot[k] % BW, by = slot[k] / BW;
            const int gx = x0 - 1 + bx, gy = y0 - 1 + by;   // unwrapped: wall tests only
            const int cx = bx + 1, cy = by + 1;              // position in the phase-A layout
            float bb[8];
            if (interior) {
#pragma unroll
                for (int i = 0; i < 8; ++i) bb[i] = lds[(i * AH + cy + EY[i]) * AW + cx + EX[i]];
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bool out = false;
                    const int sx = gx + EX[i], sy = gy + EY[i];
                    if (EX[i] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) out = true;
                    if (EY[i] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) out = true;
                    const int src = out ? (OPP[i] * AH + cy) * AW + cx : (i * AH + cy + EY[i]) * AW + cx + EX[i];
                    bb[i] = lds[src];
                }
            }
            const Cell c = med.cell(d, rawB[k]);
            ParamBar pb;
            collide_adjoint(bb, d, c, c.phi * d.ax, c.phi * d.ay, uB[k][0], uB[k][1], uB[k][2], uB[k][3], ab[k], pb);
            if (bx >= 1 && bx <= ATW && by >= 1 && by <= ATH && gx < d.nx && gy < d.ny) {
                float gp, gk;
                medium_gradient<MK>(d, c, rawB[k].kappa, pb, d.ax, d.ay, gp, gk);
                gpart[1][by - 1][bx - 1] = gp;
                if (KAPPA) gpart[KAPPA ? 3 : 1][by - 1][bx - 1] = gk;
                if (THETA) {
                    theta_add(d, c, pb, ts);
                    if (gy == d.ny - 1)
                        ts.lid += lid_share(d, gy, lds[(6 * AH + cy) * AW + cx], lds[(7 * AH + cy) * AW + cx]);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NBB; ++k) {
        if (slot[k] < 0) continue;
        const int bx = slot[k] % BW, by = slot[k] / BW;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[(i * BH + by) * BW + bx] = ab[k][i];
    }
    __syncthreads();

    // phase C: a(t-2) on the tile, to HBM. The vector-memory counter retires loads
    // and stores in order, so every input is fetched before the first store.
    {
        const BufRes rutm2 = buf_res(u_tm2, 5 * pb4);
        CellRaw rawC[NC];
        float uC[NC][4], gC[NC], gkC[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int q = threadIdx.x + k * ANT;
            const int gx = x0 + q % ATW, gy = y0 + q / ATW;
            if (q >= ATW * ATH || gx >= d.nx || gy >= d.ny) continue;
            const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
            rawC[k] = med.load(o4);
            uC[k][0] = BufIO<float>::ld(rutm2, o4, 0u);
            uC[k][1] = BufIO<float>::ld(rutm2, o4, pb4);
            uC[k][2] = THETA ? BufIO<float>::ld(rutm2, o4, 2 * pb4) : 0.0f;
            uC[k][3] = THETA ? BufIO<float>::ld(rutm2, o4, 3 * pb4) : 0.0f;
            gC[k] = BufIO<float>::ld(rg, o4, 0u);
            gkC[k] = KAPPA ? BufIO<float>::ld(rgk, o4, 0u) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int q = threadIdx.x + k * ANT;
            if (q >= ATW * ATH) continue;
            const int lx = q % ATW, ly = q / ATW;
            const int gx = x0 + lx, gy = y0 + ly;
            if (gx >= d.nx || gy >= d.ny) continue;
            const uint32_t o4 = (uint32_t)(((int64_t)gy * d.pitch + gx) * 4);
            const int cx = lx + 1, cy = ly + 1;
            float bb[8];
            if (interior) {
#pragma unroll
                for (int i = 0; i < 8; ++i) bb[i] = lds[(i * BH + cy + EY[i]) * BW + cx + EX[i]];
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bool out = false;
                    const int sx = gx + EX[i], sy = gy + EY[i];
                    if (EX[i] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) out = true;
                    if (EY[i] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) out = true;
                    const int src = out ? (OPP[i] * BH + cy) * BW + cx : (i * BH + cy + EY[i]) * BW + cx + EX[i];
                    bb[i] = lds[src];
                }
            }
            const Cell c = med.cell(d, rawC[k]);
            float a[8];
            ParamBar pb;
            collide_adjoint(bb, d, c, c.phi * d.ax, c.phi * d.ay, uC[k][0], uC[k][1], uC[k][2], uC[k][3], a, pb);
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<float>::st(rlout, o4, (uint32_t)i * pb4, a[i]);
            float gp, gk;
            medium_gradient<MK>(d, c, rawC[k].kappa, pb, d.ax, d.ay, gp, gk);
            BufIO<float>::st(rg, o4, 0u, ((gC[k] + gpart[0][ly][lx]) + gpart[1][ly][lx]) + gp);
            if (KAPPA)
                BufIO<float>::st(rgk, o4, 0u,
                                 ((gkC[k] + gpart[KAPPA ? 2 : 0][ly][lx]) + gpart[KAPPA ? 3 : 1][ly][lx]) + gk);
            if (THETA) {
                theta_add(d, c, pb, ts);
                if (gy == d.ny - 1)
                    ts.lid += lid_share(d, gy, lds[(6 * BH + cy) * BW + cx], lds[(7 * BH + cy) * BW + cx]);
            }
        }
    }
    if (THETA) block_theta_add<ANT>(ts, acc + 4 * (int64_t)b);
}

hipError_t launch_adjoint_step3(const Dom &d, const float *lam_in, float *lam_out, const float *u_t,
                                const float *u_tm1, const float *u_tm2, float *gphi, float *gkappa, double *acc,
                                hipStream_t st) {
    const int tiles_x = (d.nx + ATW - 1) / ATW, tiles_y = (d.ny + ATH - 1) / ATH;
    const dim3 grid((unsigned)(tiles_x * tiles_y));
    const int mk = medium_kind(d) == MK_ERGUN ? MK_ERGUN : MK_ANY;
    const bool kap = gkappa != nullptr;
#define MRT_ADJ3(TH, MK, KP) \
    hipLaunchKernelGGL((k_adjoint_step3<TH, MK, KP>), grid, dim3(ANT), 0, st, d, lam_in, lam_out, u_t, u_tm1, \
                       u_tm2, gphi, gkappa, tiles_x, 1, acc)
    if (kap) {
        if (acc) MRT_ADJ3(true, MK_ANY, true);
        else MRT_ADJ3(false, MK_ANY, true);
    } else if (mk == MK_ERGUN) {
        if (acc) MRT_ADJ3(true, MK_ERGUN, false);
        else MRT_ADJ3(false, MK_ERGUN, false);
    } else {
        if (acc) MRT_ADJ3(true, MK_ANY, false);
        else MRT_ADJ3(false, MK_ANY, false);
    }
#undef MRT_ADJ3
    return hipGetLastError();
}

hipError_t launch_adjoint_step2(const Dom &d, const float *lam_in, float *lam_out, const float *u_t,
                                const float *u_tm1, float *gphi, float *gkappa, double *acc, hipStream_t st) {
    const int tiles_x = (d.nx + ATW - 1) / ATW, tiles_y = (d.ny + ATH - 1) / ATH;
    const dim3 grid((unsigned)(tiles_x * tiles_y));
    const bool ergun = medium_kind(d) == MK_ERGUN;
    const float *no_g = nullptr;
    float *no_gout = nullptr;
#define MRT_ADJ2(TH, MK) \
    hipLaunchKernelGGL((k_adjoint_step2<TH, MK, false>), grid, dim3(ANT), 0, st, d, lam_in, lam_out, no_g, no_gout, \
                       u_t, u_tm1, gphi, gkappa, tiles_x, 1, acc)
    if (acc && ergun) MRT_ADJ2(true, MK_ERGUN);
    else if (acc) MRT_ADJ2(true, MK_ANY);
    else if (ergun) MRT_ADJ2(false, MK_ERGUN);
    else MRT_ADJ2(false, MK_ANY);
#undef MRT_ADJ2
    return hipGetLastError();
}

hipError_t launch_adjoint_step2_thermal(const Dom &d, const float *lam_in, float *lam_out, const float *lamg_in,
                                        float *lamg_out, const float *u_t, const float *u_tm1, float *gphi,
                                        float *gkappa, double *acc, hipStream_t st) {
    const int tiles_x = (d.nx + ATW - 1) / ATW, tiles_y = (d.ny + ATH - 1) / ATH;
    const dim3 grid((unsigned)(tiles_x * tiles_y));
    const bool ergun = medium_kind(d) == MK_ERGUN;
#define MRT_ADJ2T(TH, MK) \
    hipLaunchKernelGGL((k_adjoint_step2<TH, MK, true>), grid, dim3(ANT), 0, st, d, lam_in, lam_out, lamg_in, \
                       lamg_out, u_t, u_tm1, gphi, gkappa, tiles_x, 1, acc)
    if (acc && ergun) MRT_ADJ2T(true, MK_ERGUN);
    else if (acc) MRT_ADJ2T(true, MK_ANY);
    else if (ergun) MRT_ADJ2T(false, MK_ERGUN);
    else MRT_ADJ2T(false, MK_ANY);
#undef MRT_ADJ2T
    return hipGetLastError();
}

hipError_t launch_adjoint_seed(const Dom &d, Source src, const float *dLdu, float *lam,
                               float *gphi, float *gkappa, double *acc, hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + ABLOCK - 1) / ABLOCK), (unsigned)d.ny);
    if (src == SRC_DIRECT) {
        if (acc) hipLaunchKernelGGL((k_adjoint_seed<SRC_DIRECT, true>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, gphi, gkappa, acc);
        else hipLaunchKernelGGL((k_adjoint_seed<SRC_DIRECT, false>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, gphi, gkappa, acc);
    } else {
        if (acc) hipLaunchKernelGGL((k_adjoint_seed<SRC_GATHER, true>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, gphi, gkappa, acc);
        else hipLaunchKernelGGL((k_adjoint_seed<SRC_GATHER, false>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, gphi, gkappa, acc);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const Dom &d, const float *lam_in, float *lam_out,
                               const float *u_t, float *gphi, float *gkappa, double *acc, hipStream_t st) {
    const int tiles_x = (d.nx + ABLOCK - 1) / ABLOCK;
    const dim3 grid((unsigned)(tiles_x * d.ny));
    if (acc)
        hipLaunchKernelGGL(k_adjoint_step<true>, grid, dim3(ABLOCK), 0, st, d, lam_in, lam_out, u_t, gphi,
                           gkappa, tiles_x, acc);
    else
        hipLaunchKernelGGL(k_adjoint_step<false>, grid, dim3(ABLOCK), 0, st, d, lam_in, lam_out, u_t, gphi,
                           gkappa, tiles_x, acc);
    return hipGetLastError();
}

// ------------------------------------------------------ thermal coupling


// Transpose of the D2Q5 gather: b_j(x) = a_j(x + e_j), or across a wall the
// node's own a of the opposite link, negated on the Dirichlet walls
// (anti-bounce-back g = const - g+) and kept on the adiabatic ones.
__device__ __forceinline__ void gather_thermal_transposed(const Dom &d, const float *__restrict__ lamg, int x,
                                                          int y, float b[5]) {
    const int64_t o = (int64_t)y * d.pitch + x;
    b[0] = lamg[o];
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        int sx = x + TXv[j], sy = y + TYv[j];
        int kind = 0;  // 0 stream, 1 bounce-back, 2 anti-bounce-back
        if (TXv[j] != 0 && (sx < 0 || sx >= d.nx)) {
            if (d.bc_x == BC_PERIODIC) sx = (sx < 0) ? d.nx - 1 : 0;
            else kind = 2;
        }
        if (TYv[j] != 0 && (sy < 0 || sy >= d.ny)) {
            if (d.bc_y == BC_PERIODIC) sy = (sy < 0) ? d.ny - 1 : 0;
            else kind = 1;
        }
        if (kind == 0) {
            b[j] = lamg[j * d.plane + (int64_t)sy * d.pitch + sx];
        } else {
            const float v = lamg[TOPP[j] * d.plane + o];
            b[j] = (kind == 1) ? v : -v;
        }
    }
}

// Seed of the coupled adjoint: a_f(T) and a_g(T) from dL/du(T) (u(T) depends on
// g(T) through the buoyancy of Sec. 3.4), and the direct medium gradient.
template <int SRC_T, bool THETA>
__global__ __launch_bounds__(ABLOCK) void k_adjoint_seed_thermal(Dom d, const float *__restrict__ dLdu,
                                                                 float *__restrict__ lam, float *__restrict__ lamg,
                                                                 float *__restrict__ gphi,
                                                                 float *__restrict__ gkappa,
                                                                 double *__restrict__ acc) {
    const int x = blockIdx.x * ABLOCK + threadIdx.x, y = blockIdx.y;
    ThetaSum ts{0.0f, 0.0f, 0.0f, 0.0f};
    if (x < d.nx) {
        float f[8], g[5];
        if (SRC_T == SRC_DIRECT) {
            load_own<float>(d, (const float *)d.fin, x, y, f);
            load_own_thermal(d, d.gin, x, y, g);
        } else {
            gather_general<float>(d, (const float *)d.fin, x, y, f);
            gather_thermal(d, d.gin, x, y, false, g);
        }
        const float dT = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
        const int64_t o = (int64_t)y * d.pitch + x;
        const Cell c = load_cell(d, o);
        const float ay = d.ay + d.gbeta * dT;
        float ux, uy, m1;
        node_velocity(f, c, c.phi * d.ax, c.phi * ay, ux, uy, m1);
        const int64_t q = (int64_t)y * d.nx + x, n = (int64_t)d.nx * d.ny;
        ParamBar pb{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float vbx, vby;
        velocity_adjoint(c, ux, uy, dLdu[q], dLdu[n + q], vbx, vby, pb);
#pragma unroll
        for (int i = 0; i < 8; ++i) lam[i * d.plane + o] = (float)EX[i] * vbx + (float)EY[i] * vby;
        const float Tb = c.phi * d.gbeta * pb.pay;   // pay = phi (a_y + g beta dT)
#pragma unroll
        for (int j = 0; j < 5; ++j) lamg[j * d.plane + o] = Tb;
        float gp, gk;
        medium_gradient(d, c, kappa_at(d, o), pb, d.ax, ay, gp, gk);
        gphi[o] = gp;
        if (gkappa) gkappa[o] = gk;
        if (THETA) theta_add(d, c, pb, ts);
    }
    if (THETA) block_theta_add<ABLOCK>(ts, acc + 4 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x));
}

// One backward step of the coupled D2Q8 + D2Q5 scheme at time t: a(t) from
// a(t+1) for both distributions, using u(t) and dT(t) recorded in planes 0, 1
// and 4 of u_t (n7, n8 in planes 2, 3 with THETA).
template <bool THETA>
__global__ __launch_bounds__(ABLOCK) void k_adjoint_step_thermal(Dom d, const float *__restrict__ lam_in,
                                                                 float *__restrict__ lam_out,
                                                                 const float *__restrict__ lamg_in,
                                                                 float *__restrict__ lamg_out,
                                                                 const float *__restrict__ u_t,
                                                                 float *__restrict__ gphi,
                                                                 float *__restrict__ gkappa,
                                                                 int tiles_x, double *__restrict__ acc) {
    const int tx = blockIdx.x % tiles_x, y = blockIdx.x / tiles_x;
    const int x = tx * ABLOCK + threadIdx.x;
    ThetaSum ts{0.0f, 0.0f, 0.0f, 0.0f};
    if (x < d.nx) {
        const int64_t o = (int64_t)y * d.pitch + x;
        float b[8], bg[5];
        gather_transposed(d, lam_in, x, y, false, b);
        gather_thermal_transposed(d, lamg_in, x, y, bg);
        const Cell c = load_cell(d, o);
        const float ux = u_t[o], uy = u_t[d.plane + o], dT = u_t[4 * d.plane + o];
        const float n7 = THETA ? u_t[2 * d.plane + o] : 0.0f, n8 = THETA ? u_t[3 * d.plane + o] : 0.0f;
        float ag[5], ubx = 0.0f, uby = 0.0f;
        thermal_collide_adjoint(bg, d, ux, uy, dT, ag, ubx, uby);
        const float ay = d.ay + d.gbeta * dT;
        float a[8];
        ParamBar pb;
        collide_adjoint(b, d, c, c.phi * d.ax, c.phi * ay, ux, uy, n7, n8, a, pb, ubx, uby);
        const float Tb = c.phi * d.gbeta * pb.pay;
#pragma unroll
        for (int i = 0; i < 8; ++i) lam_out[i * d.plane + o] = a[i];
#pragma unroll
        for (int j = 0; j < 5; ++j) lamg_out[j * d.plane + o] = ag[j] + Tb;
        float gp, gk;
        medium_gradient(d, c, kappa_at(d, o), pb, d.ax, ay, gp, gk);
        gphi[o] += gp;
        if (gkappa) gkappa[o] += gk;
        if (THETA) {
            theta_add(d, c, pb, ts);
            if (y == d.ny - 1) ts.lid += lid_share(d, y, lam_in[6 * d.plane + o], lam_in[7 * d.plane + o]);
        }
    }
    if (THETA) block_theta_add<ABLOCK>(ts, acc + 4 * (int64_t)blockIdx.x);
}

hipError_t launch_adjoint_seed_thermal(const Dom &d, Source src, const float *dLdu, float *lam, float *lamg,
                                       float *gphi, float *gkappa, double *acc, hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + ABLOCK - 1) / ABLOCK), (unsigned)d.ny);
    if (src == SRC_DIRECT) {
        if (acc) hipLaunchKernelGGL((k_adjoint_seed_thermal<SRC_DIRECT, true>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, lamg, gphi, gkappa, acc);
        else hipLaunchKernelGGL((k_adjoint_seed_thermal<SRC_DIRECT, false>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, lamg, gphi, gkappa, acc);
    } else {
        if (acc) hipLaunchKernelGGL((k_adjoint_seed_thermal<SRC_GATHER, true>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, lamg, gphi, gkappa, acc);
        else hipLaunchKernelGGL((k_adjoint_seed_thermal<SRC_GATHER, false>), grid, dim3(ABLOCK), 0, st, d, dLdu, lam, lamg, gphi, gkappa, acc);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_step_thermal(const Dom &d, const float *lam_in, float *lam_out, const float *lamg_in,
                                       float *lamg_out, const float *u_t, float *gphi, float *gkappa, double *acc,
                                       hipStream_t st) {
    const int tiles_x = (d.nx + ABLOCK - 1) / ABLOCK;
    const dim3 grid((unsigned)(tiles_x * d.ny));
    if (acc)
        hipLaunchKernelGGL(k_adjoint_step_thermal<true>, grid, dim3(ABLOCK), 0, st, d, lam_in, lam_out, lamg_in,
                           lamg_out, u_t, gphi, gkappa, tiles_x, acc);
    else
        hipLaunchKernelGGL(k_adjoint_step_thermal<false>, grid, dim3(ABLOCK), 0, st, d, lam_in, lam_out, lamg_in,
                           lamg_out, u_t, gphi, gkappa, tiles_x, acc);
    return hipGetLastError();
}

// ---------------------------------------------------------------- tangent

// Forward mode of the velocity recovery (Eqs. 18-19) on the solution: with
// D = 2 l0 + l1 |u| and R = l0 + l1 |u|, du/dv = (I - (l1 / (2 R |u|)) u u^T) / D,
// du/dcd = -u / (4 R) and du/dcf = -|u| u / (4 R) (the transposes of the maps
// velocity_adjoint applies).
__device__ __forceinline__ void velocity_tangent(const Cell &c, float ux, float uy, float vdx, float vdy,
                                                 float dcd, float dcf, float &udx, float &udy) {
    const float umag = hw_sqrt(ux * ux + uy * uy);
    const float l0 = 0.5f * (1.0f + 0.5f * c.cd);
    const float l1 = 0.5f * c.cf;
    const float R = l0 + l1 * umag;
    const float D = l0 + R;
    const float rR = hw_rcp(R), rD = hw_rcp(D);
    const float corr = (umag > 0.0f) ? (0.5f * l1 * rR) * (ux * vdx + uy * vdy) * hw_rcp(umag) : 0.0f;
    const float w = 0.25f * (dcd + umag * dcf) * rR;
    udx = (vdx - corr * ux) * rD - w * ux;
    udy = (vdy - corr * uy) * rD - w * uy;
}

// Tangents of the node's inputs: phi a (per component), cd, cf, 1/phi and s_nu.
struct TanIn {
    float dpax, dpay, dcd, dcf, dip, ds;
};

__device__ __forceinline__ TanIn tangent_inputs(const Dom &d, const Cell &c, float kappa, float dphi,
                                                float dnu, float dax, float day) {
    float dcd_dphi, dcf_dphi;
    cell_phi_derivs(d, c, kappa, dcd_dphi, dcf_dphi);
    TanIn t;
    t.dpax = dphi * d.ax + c.phi * dax;
    t.dpay = dphi * d.ay + c.phi * day;
    t.dcd = dcd_dphi * dphi + c.cd * dnu * d.inv_nu;
    t.dcf = dcf_dphi * dphi;
    t.dip = -c.inv_phi * c.inv_phi * dphi;
    t.ds = -c.s_nu * c.h_nu * dnu * d.inv_nu;   // s_nu = 1/(1/2 + 3 J nu)
    return t;
}

// Forward mode of one node's collision (Eq. 14 and f+ = M^-1 m+): given f and
// its tangent ft, returns the tangent of f+.
__device__ __forceinline__ void collide_tangent(const float f[8], const float ft[8], const Dom &d,
                                                const Cell &c, float pax, float pay, const TanIn &ti,
                                                float out[8]) {
    auto moments = [](const float g[8], float m[8]) {
        const float a = g[0] + g[2], b = g[1] + g[3], cc = g[4] + g[6], dg = g[5] + g[7];
        const float x13 = g[0] - g[2], y24 = g[1] - g[3], p57 = g[4] - g[6], q68 = g[5] - g[7];
        const float pmq = p57 - q68, ppq = p57 + q68;
        m[0] = (a + b) + (cc + dg);
        m[1] = (cc + dg) - (a + b);
        m[2] = x13 + pmq;
        m[3] = fmaf(-2.0f, x13, pmq);
        m[4] = y24 + ppq;
        m[5] = fmaf(-2.0f, y24, ppq);
        m[6] = a - b;
        m[7] = cc - dg;
    };
    float m[8], dm[8];
    moments(f, m);
    moments(ft, dm);
    // forward quantities, as in collide
    float ux, uy;
    velocity(c, fmaf(0.5f, pax, m[2]), fmaf(0.5f, pay, m[4]), ux, uy);
    const float umag = hw_sqrt(fmaf(ux, ux, uy * uy));
    const float drag = fmaf(c.cf, umag, c.cd);
    const float Fx = fmaf(-drag, ux, pax), Fy = fmaf(-drag, uy, pay);
    const float ip = c.inv_phi;
    // tangents of u, |u| and F (Eq. 3)
    float udx, udy;
    velocity_tangent(c, ux, uy, dm[2] + 0.5f * ti.dpax, dm[4] + 0.5f * ti.dpay, ti.dcd, ti.dcf, udx, udy);
    const float dumag = (umag > 0.0f) ? (ux * udx + uy * udy) * hw_rcp(umag) : 0.0f;
    const float ddrag = ti.dcd + ti.dcf * umag + c.cf * dumag;
    const float dFx = ti.dpax - ddrag * ux - drag * udx;
    const float dFy = ti.dpay - ddrag * uy - drag * udy;
    // relaxation (Eq. 14) differentiated term by term
    const float u2 = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
    const float du2 = 2.0f * (ux * udx + uy * udy);
    const float duF = (udx * Fx + ux * dFx) + (udy * Fy + uy * dFy);
    float mp[8];
    mp[0] = dm[0];
    mp[1] = dm[1] - d.s_e * (dm[1] + 0.6f * dm[0] - 0.4f * (du2 * ip + u2 * ti.dip)) +
            0.8f * d.h_e * (duF * ip + uF * ti.dip);
    mp[2] = udx + 0.5f * dFx;
    mp[4] = udy + 0.5f * dFy;
    mp[3] = dm[3] - d.s_q * (dm[3] + udx) - d.h_q * dFx;
    mp[5] = dm[5] - d.s_q * (dm[5] + udy) - d.h_q * dFy;
    const float pxx = (ux * ux - uy * uy) * ip, pxy = ux * uy * ip;
    const float Sxx = 2.0f * (ux * Fx - uy * Fy) * ip, Sxy = (ux * Fy + uy * Fx) * ip;
    const float dpxx = 2.0f * (ux * udx - uy * udy) * ip + (ux * ux - uy * uy) * ti.dip;
    const float dpxy = (udx * uy + ux * udy) * ip + ux * uy * ti.dip;
    const float dSxx = 2.0f * ((udx * Fx + ux * dFx) - (udy * Fy + uy * dFy)) * ip +
                       2.0f * (ux * Fx - uy * Fy) * ti.dip;
    const float dSxy = ((udx * Fy + ux * dFy) + (udy * Fx + uy * dFx)) * ip + (ux * Fy + uy * Fx) * ti.dip;
    mp[6] = dm[6] - c.s_nu * (dm[6] - dpxx) + c.h_nu * dSxx - ti.ds * ((m[6] - pxx) + 0.5f * Sxx);
    mp[7] = dm[7] - c.s_nu * (dm[7] - dpxy) + c.h_nu * dSxy - ti.ds * ((m[7] - pxy) + 0.5f * Sxy);
    // f+ tangent = M^T diag(1/8, 1/8, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m+ tangent
    const float y[8] = {0.125f * mp[0], 0.125f * mp[1], mp[2] * (1.0f / 6.0f), mp[3] * (1.0f / 12.0f),
                        mp[4] * (1.0f / 6.0f), mp[5] * (1.0f / 12.0f), 0.25f * mp[6], 0.25f * mp[7]};
    apply_MT(y, out);
}

// One cycle of the state and its tangent: d streams the state (fin -> fout),
// dt the tangent (same geometry, its own buffers, lid6 = dU/6 so that the
// moving-wall term's tangent enters the bounce-back). dphi: tangent porosity
// plane (pitched, may be NULL); dnu, dax, day: tangent parameters.
__global__ __launch_bounds__(ABLOCK) void k_tangent_step(Dom d, Dom dt, int src, const float *__restrict__ dphi,
                                                         float dnu, float dax, float day) {
    const int x = blockIdx.x * ABLOCK + threadIdx.x, y = blockIdx.y;
    if (x >= d.nx) return;
    float f[8], ft[8];
    if (src == SRC_DIRECT) {
        load_own<float>(d, (const float *)d.fin, x, y, f);
        load_own<float>(dt, (const float *)dt.fin, x, y, ft);
    } else {
        gather_general<float>(d, (const float *)d.fin, x, y, f);
        gather_general<float>(dt, (const float *)dt.fin, x, y, ft);
    }
    const int64_t o = (int64_t)y * d.pitch + x;
    const Cell c = load_cell(d, o);
    const TanIn ti = tangent_inputs(d, c, kappa_at(d, o), dphi ? dphi[o] : 0.0f, dnu, dax, day);
    float fpt[8];
    collide_tangent(f, ft, d, c, c.phi * d.ax, c.phi * d.ay, ti, fpt);
    float ux, uy;
    collide(f, d, c, c.phi * d.ax, c.phi * d.ay, ux, uy);
    float *fo = (float *)d.fout, *fto = (float *)dt.fout;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        fo[i * d.plane + o] = f[i];
        fto[i * d.plane + o] = fpt[i];
    }
}

// Tangent of u at the state's time into du [2][ny][nx] (unpitched).
__global__ __launch_bounds__(ABLOCK) void k_tangent_u(Dom d, Dom dt, int src, const float *__restrict__ dphi,
                                                      float dnu, float dax, float day, float *__restrict__ du) {
    const int x = blockIdx.x * ABLOCK + threadIdx.x, y = blockIdx.y;
    if (x >= d.nx) return;
    float f[8], ft[8];
    if (src == SRC_DIRECT) {
        load_own<float>(d, (const float *)d.fin, x, y, f);
        load_own<float>(dt, (const float *)dt.fin, x, y, ft);
    } else {
        gather_general<float>(d, (const float *)d.fin, x, y, f);
        gather_general<float>(dt, (const float *)dt.fin, x, y, ft);
    }
    const int64_t o = (int64_t)y * d.pitch + x;
    const Cell c = load_cell(d, o);
    const TanIn ti = tangent_inputs(d, c, kappa_at(d, o), dphi ? dphi[o] : 0.0f, dnu, dax, day);
    float ux, uy, m1, dux, duy, dm1;
    node_velocity(f, c, c.phi * d.ax, c.phi * d.ay, ux, uy, m1);
    float dm3, dm5;
    conserved_moments(ft, dm1, dm3, dm5);
    velocity_tangent(c, ux, uy, dm3 + 0.5f * ti.dpax, dm5 + 0.5f * ti.dpay, ti.dcd, ti.dcf, dux, duy);
    const int64_t q = (int64_t)y * d.nx + x, n = (int64_t)d.nx * d.ny;
    du[q] = dux;
    du[n + q] = duy;
}

hipError_t launch_tangent_step(const Dom &d, const Dom &dt, Source src, const float *dphi, float dnu,
                               float dax, float day, hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + ABLOCK - 1) / ABLOCK), (unsigned)d.ny);
    hipLaunchKernelGGL(k_tangent_step, grid, dim3(ABLOCK), 0, st, d, dt, (int)src, dphi, dnu, dax, day);
    return hipGetLastError();
}

hipError_t launch_tangent_u(const Dom &d, const Dom &dt, Source src, const float *dphi, float dnu, float dax,
                            float day, float *du, hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + ABLOCK - 1) / ABLOCK), (unsigned)d.ny);
    hipLaunchKernelGGL(k_tangent_u, grid, dim3(ABLOCK), 0, st, d, dt, (int)src, dphi, dnu, dax, day, du);
    return hipGetLastError();
}

// Sum of per-block parameter partials over n slots of 4 doubles, in a fixed
// order (one workgroup): out[k] = sum_j slots[4 j + k].
__global__ __launch_bounds__(256) void k_theta_final(const double *__restrict__ slots, int64_t n,
                                                     double *__restrict__ out) {
    __shared__ double red[256][4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t j = threadIdx.x; j < n; j += 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += slots[4 * j + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[threadIdx.x][k] += red[threadIdx.x + w][k];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = red[0][threadIdx.x];
}

hipError_t launch_theta_final(const double *slots, int64_t n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_theta_final, dim3(1), dim3(256), 0, st, slots, n, out);
    return hipGetLastError();
}

int64_t adjoint_theta_slots(int nx, int ny) {
    const int64_t seed = (int64_t)((nx + ABLOCK - 1) / ABLOCK) * ny;
    const int64_t step = seed;
    const int64_t step2 = (int64_t)((nx + ATW - 1) / ATW) * ((ny + ATH - 1) / ATH);
    return seed + step + step2;
}

int64_t adjoint_theta_offset(int nx, int ny, int which) {
    const int64_t seed = (int64_t)((nx + ABLOCK - 1) / ABLOCK) * ny;
    return which == 0 ? 0 : (which == 1 ? seed : 2 * seed);
}

}  // namespace mrt
