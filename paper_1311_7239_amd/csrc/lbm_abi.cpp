// C ABI of the gfx950 porous MRT-LB library: descriptor validation,
// workspace carving, state bookkeeping (time, ping-pong buffers,
// checkpoints) and kernel launches. Declarations and the contract of every
// entry point are in include/lbm.h.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "lbm_launch.h"

using namespace mrt;

// Device scratch of lbm_reduce_static: the FP64 partial sums of the reduction
// (three per workgroup, at most kReduceMaxBlocks workgroups) followed by the
// three final sums. One copy per GPU, held until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives per device.
constexpr int kReduceMaxBlocks = 4096;
constexpr int kScratchDoubles = 3 * kReduceMaxBlocks + 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int64_t round_up64(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Workspace layout of one domain, as byte offsets from its base.
struct Layout {
    int32_t pitch = 0;   // elements per stored row
    int64_t plane = 0;   // elements between planes (same for every plane type)
    int esize = 4;       // bytes per stored population
    size_t f_bytes = 0;  // one population buffer (8 planes)
    size_t g_bytes = 0;  // one thermal buffer (5 planes, FP32)
    size_t p_bytes = 0;  // one FP32 plane
    size_t off_f[2] = {0, 0}, off_g[2] = {0, 0};
    size_t off_phi = 0, off_kappa = 0, off_snu = 0, off_part = 0, off_res = 0;
    size_t off_uprev = 0;  // u(t - 1): two FP32 planes written by the last pass of lbm_step
    int red_blocks = 0;
    // recording for the adjoint
    int64_t nck = 0, ring = 0;
    size_t off_ck = 0, off_urec = 0, off_lam[2] = {0, 0}, off_gphi = 0, off_gkappa = 0;
    size_t off_theta = 0, theta_slots = 0;  // parameter-gradient slots (4 doubles each) + 4 results
    size_t off_rf[2] = {0, 0};  // recomputation buffers (the forward state stays put)
    size_t ck_slot = 0;         // bytes per checkpoint: populations (+ thermal populations)
    size_t off_lamg[2] = {0, 0}, off_rg[2] = {0, 0};  // thermal adjoint and recomputation
    size_t total = 0;
};

Layout make_layout(const lbm_desc &d, int64_t max_rec) {
    Layout L;
    L.esize = (d.storage == LBM_FP16_DEV) ? 2 : 4;
    L.pitch = (int32_t)round_up64(d.nx, 64);
    L.plane = round_up64((int64_t)d.ny * L.pitch, 128);
    L.f_bytes = (size_t)L.plane * L.esize * 8;
    L.g_bytes = (size_t)L.plane * 4 * 5;
    L.p_bytes = (size_t)L.plane * 4;
    size_t o = 0;
    auto carve = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, ALIGN);
        return at;
    };
    L.off_f[0] = carve(L.f_bytes);
    L.off_f[1] = carve(L.f_bytes);
    if (d.thermal.enabled) {
        L.off_g[0] = carve(L.g_bytes);
        L.off_g[1] = carve(L.g_bytes);
    }
    if (d.medium != LBM_MEDIUM_UNIFORM) L.off_phi = carve(L.p_bytes);
    if (d.medium == LBM_MEDIUM_PHI_KAPPA) L.off_kappa = carve(L.p_bytes);
    if (d.j_plane) L.off_snu = carve(L.p_bytes);
    L.red_blocks = reduce_blocks(d.nx, d.ny);
    L.off_part = carve(sizeof(double) * 3 * (size_t)L.red_blocks);
    L.off_res = carve(sizeof(double) * 4);
    L.off_uprev = carve(L.p_bytes * 2);
    if (d.ckpt_every > 0) {
        L.nck = max_rec / d.ckpt_every + 1;
        L.ring = d.ckpt_every;
        L.ck_slot = L.f_bytes + (d.thermal.enabled ? L.g_bytes : 0);
        L.off_ck = carve(L.ck_slot * (size_t)L.nck);
        // per recorded step: u_x, u_y, the two stress moments (parameter gradients)
        // and the temperature deviation (thermal coupling)
        L.off_urec = carve(L.p_bytes * 5 * (size_t)L.ring);
        L.off_lam[0] = carve(L.p_bytes * 8);
        L.off_lam[1] = carve(L.p_bytes * 8);
        L.off_gphi = carve(L.p_bytes);
        L.off_gkappa = carve(L.p_bytes);
        L.off_rf[0] = carve(L.f_bytes);
        L.off_rf[1] = carve(L.f_bytes);
        if (d.thermal.enabled) {
            L.off_lamg[0] = carve(L.g_bytes);
            L.off_lamg[1] = carve(L.g_bytes);
            L.off_rg[0] = carve(L.g_bytes);
            L.off_rg[1] = carve(L.g_bytes);
        }
        L.theta_slots = (size_t)adjoint_theta_slots(d.nx, d.ny);
        L.off_theta = carve(sizeof(double) * 4 * (L.theta_slots + 1));
    }
    L.total = o;
    return L;
}

int validate(const lbm_desc *d) {
    if (!d) return fail(LBM_EINVAL, "descriptor is NULL");
    if (d->nx < 1 || d->ny < 1) return fail(LBM_EINVAL, "nx and ny must be >= 1 (got %d, %d)", d->nx, d->ny);
    if ((int64_t)d->nx * d->ny > (int64_t)1 << 31)
        return fail(LBM_EINVAL, "nx*ny exceeds 2^31 nodes");
    auto bc_ok = [](int32_t b) { return b == LBM_PERIODIC || b == LBM_WALLS || b == LBM_WALLS_NEE; };
    if (!bc_ok(d->bc_x)) return fail(LBM_EINVAL, "bc_x must be LBM_PERIODIC, LBM_WALLS or LBM_WALLS_NEE");
    if (!bc_ok(d->bc_y)) return fail(LBM_EINVAL, "bc_y must be LBM_PERIODIC, LBM_WALLS or LBM_WALLS_NEE");
    if (d->bc_x == LBM_WALLS && d->nx < 2) return fail(LBM_EINVAL, "a walled x axis needs nx >= 2");
    if (d->bc_y == LBM_WALLS && d->ny < 2) return fail(LBM_EINVAL, "a walled y axis needs ny >= 2");
    if (d->bc_x == LBM_WALLS_NEE && d->nx < 3) return fail(LBM_EINVAL, "an on-node walled x axis needs nx >= 3");
    if (d->bc_y == LBM_WALLS_NEE && d->ny < 3) return fail(LBM_EINVAL, "an on-node walled y axis needs ny >= 3");
    if ((d->bc_x == LBM_WALLS && d->bc_y == LBM_WALLS_NEE) || (d->bc_x == LBM_WALLS_NEE && d->bc_y == LBM_WALLS))
        return fail(LBM_ENOTSUP, "bounce-back and on-node walls cannot be mixed");
    if (d->lid_ux != 0.0 && d->bc_y == LBM_PERIODIC) return fail(LBM_EINVAL, "lid_ux needs walls in y");
    if (!std::isfinite(d->lid_ux)) return fail(LBM_EINVAL, "lid_ux must be finite");
    if (!(d->nu > 0.0) || !std::isfinite(d->nu)) return fail(LBM_EINVAL, "nu must be > 0 (tau > 1/2)");
    if (!(d->J > 0.0) || !std::isfinite(d->J)) return fail(LBM_EINVAL, "J must be > 0");
    if (!(d->s_e > 0.0 && d->s_e < 2.0)) return fail(LBM_EINVAL, "s_e must lie in (0, 2)");
    if (!(d->s_q > 0.0 && d->s_q < 2.0)) return fail(LBM_EINVAL, "s_q must lie in (0, 2)");
    if (d->medium < LBM_MEDIUM_UNIFORM || d->medium > LBM_MEDIUM_PHI_KAPPA) return fail(LBM_EINVAL, "unknown medium");
    if (d->medium == LBM_MEDIUM_UNIFORM) {
        if (!(d->phi0 > 0.0 && d->phi0 <= 1.0)) return fail(LBM_EINVAL, "phi0 must lie in (0, 1]");
        if (!(d->kappa0 >= 0.0) || !std::isfinite(d->kappa0)) return fail(LBM_EINVAL, "kappa0 must be finite and >= 0");
    }
    if (d->medium == LBM_MEDIUM_PHI_ERGUN && !(d->dp > 0.0 && std::isfinite(d->dp)))
        return fail(LBM_EINVAL, "dp must be > 0 for LBM_MEDIUM_PHI_ERGUN");
    if (!std::isfinite(d->F_eps)) return fail(LBM_EINVAL, "F_eps must be finite");
    if (!std::isfinite(d->ax) || !std::isfinite(d->ay) || !std::isfinite(d->Pi0))
        return fail(LBM_EINVAL, "ax, ay and Pi0 must be finite");
    if (d->storage != LBM_FP32_DEV && d->storage != LBM_FP16_DEV) return fail(LBM_EINVAL, "unknown storage");
    if (d->ckpt_every < 0) return fail(LBM_EINVAL, "ckpt_every must be >= 0");
    if (d->j_plane != 0 && d->j_plane != 1) return fail(LBM_EINVAL, "j_plane must be 0 or 1");
    if (d->thermal.enabled) {
        const lbm_thermal &t = d->thermal;
        if (!(t.tau_T > 0.5) || !std::isfinite(t.tau_T)) return fail(LBM_EINVAL, "thermal tau_T must be > 1/2");
        if (!(t.sigma > 0.0) || !std::isfinite(t.sigma)) return fail(LBM_EINVAL, "thermal sigma must be > 0");
        if (!(t.zeta3 > 0.0 && t.zeta3 < 2.0) || !(t.zeta4 > 0.0 && t.zeta4 < 2.0))
            return fail(LBM_EINVAL, "thermal zeta3, zeta4 must lie in (0, 2)");
        if (!std::isfinite(t.Th) || !std::isfinite(t.Tc) || !std::isfinite(t.T0) || !std::isfinite(t.g_beta))
            return fail(LBM_EINVAL, "thermal temperatures and g_beta must be finite");
    }
    return LBM_OK;
}

// Per-domain constants in single precision, computed in double on the host
// (the same code for single and batched contexts, so both see identical bits).
Dom make_dom(const lbm_desc &d, const Layout &L) {
    Dom o;
    std::memset(&o, 0, sizeof(o));
    o.nx = d.nx; o.ny = d.ny; o.pitch = L.pitch; o.plane = L.plane;
    o.bc_x = d.bc_x; o.bc_y = d.bc_y;
    o.lid6 = (float)(d.lid_ux / 6.0);
    o.lid_u = (float)d.lid_ux;
    const double tau = 0.5 + 3.0 * d.J * d.nu;  // Eq. (21), cs^2 = 1/3
    const double s_nu = 1.0 / tau;
    o.s_e = (float)d.s_e; o.s_q = (float)d.s_q; o.s_nu = (float)s_nu;
    o.h_e = (float)(1.0 - 0.5 * d.s_e); o.h_q = (float)(1.0 - 0.5 * d.s_q);
    // from the rounded rate, as the kernels form 1 - s/2 for a per-node rate
    o.h_nu = (float)(1.0 - 0.5 * (double)o.s_nu);
    o.h_e16 = (float)(1.6 * (1.0 - 0.5 * d.s_e));
    o.h_q2 = 2.0f * o.h_q;
    o.h_nu2 = 2.0f * o.h_nu;
    o.h_nu4 = 4.0f * o.h_nu;
    o.medium = d.medium;
    o.nu = (float)d.nu;
    o.inv_nu = (float)(1.0 / d.nu);
    o.Fconst = (float)d.F_eps;
    if (d.medium == LBM_MEDIUM_UNIFORM) {
        const double F = d.F_eps >= 0.0 ? d.F_eps : 1.75 / std::sqrt(150.0 * d.phi0 * d.phi0 * d.phi0);
        o.phi0 = (float)d.phi0;
        o.inv_phi0 = (float)(1.0 / d.phi0);
        o.cd0 = (float)(d.phi0 * d.nu * d.kappa0);
        o.cf0 = (float)(d.phi0 * F * std::sqrt(d.kappa0));
        o.cd0h = 0.5f * o.cd0;
        o.cf0h = 0.5f * o.cf0;
    }
    if (d.medium == LBM_MEDIUM_PHI_ERGUN) {
        o.kcoef = (float)(150.0 / (d.dp * d.dp));
        o.cdk = (float)(150.0 * d.nu / (d.dp * d.dp));
        o.cfk = (float)(1.75 / d.dp);
        o.cdkh = 0.5f * o.cdk;
        o.cfkh = 0.5f * o.cfk;
    }
    o.ax = (float)d.ax; o.ay = (float)d.ay;
    o.axh = 0.5f * o.ax; o.ayh = 0.5f * o.ay;
    if (d.thermal.enabled) {
        const lbm_thermal &t = d.thermal;
        o.thermal = 1;
        o.zT = (float)(1.0 / t.tau_T);
        o.z3 = (float)t.zeta3; o.z4 = (float)t.zeta4;
        o.inv_sigma = (float)(1.0 / t.sigma);
        o.T0 = (float)t.T0;
        o.gbeta = (float)t.g_beta;
        o.gbetah = 0.5f * o.gbeta;
        o.abbh = (float)(0.4 * (t.Th - t.T0));  // 2 w_T (T_w - T0), w_T = 1/5
        o.abbc = (float)(0.4 * (t.Tc - t.T0));
        o.dTh = (float)(t.Th - t.T0);
        o.dTc = (float)(t.Tc - t.T0);
    }
    return o;
}

struct Domain {
    lbm_desc desc;
    Layout L;
    char *base = nullptr;
    Dom dom;  // constants and medium planes; buffers filled per launch
};

}  // namespace

struct lbm_ctx {
    std::vector<Domain> dom;
    hipStream_t stream = nullptr;
    int64_t t = 0;
    int cur = 0;  // index of the buffer holding the state at t
    bool poisoned = false;
    bool batch = false;
    bool batch_thermal = false;  // every batch domain carries the D2Q5 field
    bool batch_uniform = false;  // every batch domain has a uniform medium and one s_nu
    Schedule sched{128, 1, 2, 1};
    // recording (single domain)
    bool rec_valid = false;
    int64_t rec_cap = 0;
    // batched stepping
    Dom *d_doms = nullptr;
    Dom *d_doms_rec = nullptr;  // the same descriptors with u(t - 1) recording (last pass of a call)
    int4 *d_tiles = nullptr;
    int ntiles = 0;
    int grid = 0;
    int storage = ST_F32;
    std::vector<Dom> h_doms;    // host copies (kept alive for the async upload)
    std::vector<int4> h_tiles;
    int4 *d_tiles2 = nullptr;   // tiles of the two-cycle kernel (64 x tb_rows)
    int ntiles2 = 0;
    int grid2 = 0;
    int grid3 = 0;              // grid of the batched three-cycle kernel (64 x 16 tiles of d_tiles2)
    int4 *d_tiles4 = nullptr;   // tiles of the batched four-cycle kernel (64 x 26, one workgroup each)
    int ntiles4 = 0;
    bool four_ok = false;       // an isothermal batch with bounce-back walls: four cycles available
    std::vector<int4> h_tiles4;
    std::vector<int4> h_tiles2;
    // steps replayed from one hand-built HIP graph (0: launch each step);
    // one executable graph per starting buffer parity
    int graph_steps = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    // cycles per HBM pass of a single-domain isothermal context (1 or 2), and
    // the two-cycle kernel's workgroup size and tile rows
    int tblock = 1;
    int tb_threads = 512;
    int tb_rows = 16;
    int device = 0;  // the device current at creation (the static scratch's copy)
};

namespace {

bool on_node_walls(const lbm_desc &d) { return d.bc_x == LBM_WALLS_NEE || d.bc_y == LBM_WALLS_NEE; }

bool any_on_node_walls(const lbm_ctx *c) {
    for (const Domain &D : c->dom)
        if (on_node_walls(D.desc)) return true;
    return false;
}

// The multi-cycle kernels address a state buffer (and a thermal buffer) with
// 32-bit byte offsets.
bool buffer_below_4gib(const Layout &L) {
    return L.f_bytes < ((size_t)1 << 32) && L.g_bytes < ((size_t)1 << 32);
}

// Two cycles per pass: halfway walls, buffers below 4 GiB, with or without the
// D2Q5 field.
bool two_cycle_possible(const lbm_ctx *c) {
    for (const Domain &D : c->dom)
        if (on_node_walls(D.desc) || !buffer_below_4gib(D.L)) return false;
    return true;
}

// Three cycles per pass: single domains (with or without the D2Q5 field) and
// isothermal batches.
bool three_cycle_possible(const lbm_ctx *c) {
    return two_cycle_possible(c) && !(c->batch && c->batch_thermal);
}

// A failed HIP call: poisons the context (if any) and reads the thread's
// stored HIP error, which HIP keeps from any failed call until it is read, so
// that the next launch check of another context does not report it again.
int device_fail(lbm_ctx *c, hipError_t e, const char *what) {
    if (c) c->poisoned = true;
    (void)hipGetLastError();
    return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

Dom dom_for(const Domain &D, int cur) {
    Dom d = D.dom;
    d.fin = D.base + D.L.off_f[cur];
    d.fout = D.base + D.L.off_f[cur ^ 1];
    if (D.desc.thermal.enabled) {
        d.gin = (const float *)(D.base + D.L.off_g[cur]);
        d.gout = (float *)(D.base + D.L.off_g[cur ^ 1]);
    }
    return d;
}

// The descriptor of the last pass of an lbm_step call: its last collision
// writes u into the domain's two u(t - 1) planes for the steady residual.
Dom dom_rec(const Domain &D, int cur) {
    Dom d = dom_for(D, cur);
    d.uprev = (float *)(D.base + D.L.off_uprev);
    return d;
}

Source src_now(int64_t t) { return t == 0 ? SRC_DIRECT : SRC_GATHER; }

// Contexts returned by lbm_create / lbm_create_batch and not yet destroyed.
// Every entry point looks a handle up here before touching it, so a destroyed
// (or never created) handle is refused and a second lbm_destroy is harmless.
std::mutex g_live_mu;
std::unordered_set<const lbm_ctx *> g_live;

void register_live(const lbm_ctx *c) {
    std::lock_guard<std::mutex> lock(g_live_mu);
    g_live.insert(c);
}

int check_handle(const lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    std::lock_guard<std::mutex> lock(g_live_mu);
    if (!g_live.count(c)) return fail(LBM_EINVAL, "not a live context (destroyed, or never created)");
    return LBM_OK;
}

int check_ctx(lbm_ctx *c) {
    if (int rc = check_handle(c)) return rc;
    if (c->poisoned) return fail(LBM_EDEVICE, "context is poisoned by an earlier device error");
    return LBM_OK;
}

int check_domain(lbm_ctx *c, int32_t k) {
    if (k < 0 || k >= (int32_t)c->dom.size()) return fail(LBM_EINVAL, "domain %d out of range", k);
    return LBM_OK;
}

// Zeroed rest state (deviations 0) in buffer `cur` of one domain, medium
// planes copied in.
hipError_t init_domain(Domain &D, int cur, const float *phi, const float *kappa, hipStream_t st) {
    hipError_t e = launch_fill_zero(D.base + D.L.off_f[cur], D.L.f_bytes, st);
    if (e == hipSuccess && D.desc.thermal.enabled) e = launch_fill_zero(D.base + D.L.off_g[cur], D.L.g_bytes, st);
    if (e == hipSuccess && D.desc.medium != LBM_MEDIUM_UNIFORM) {
        // keep the row padding defined: fill first, then copy the rows
        e = launch_fill_zero(D.base + D.L.off_phi, align_up(D.L.p_bytes, 16), st);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(D.base + D.L.off_phi, (size_t)D.L.pitch * 4, phi, (size_t)D.desc.nx * 4,
                                 (size_t)D.desc.nx * 4, (size_t)D.desc.ny, hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess && D.desc.medium == LBM_MEDIUM_PHI_KAPPA) {
        e = launch_fill_zero(D.base + D.L.off_kappa, align_up(D.L.p_bytes, 16), st);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(D.base + D.L.off_kappa, (size_t)D.L.pitch * 4, kappa, (size_t)D.desc.nx * 4,
                                 (size_t)D.desc.nx * 4, (size_t)D.desc.ny, hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess && D.desc.j_plane) {
        // every node starts at the descriptor's J
        e = launch_fill_zero(D.base + D.L.off_snu, align_up(D.L.p_bytes, 16), st);
        if (e == hipSuccess)
            e = launch_snu_plane(nullptr, D.desc.J, D.desc.nu, (float *)(D.base + D.L.off_snu), D.L.pitch,
                                 D.desc.nx, D.desc.ny, nullptr, st);
    }
    return e;
}

// The step kernels store the state non-temporally once a state buffer outgrows
// the 256 MB Infinity Cache (8192^2 FP32: about 2% faster in the three-cycle
// pass, 3% in the one-cycle pass; with two 134 MB buffers at 2048^2 the cached
// stores are 5% faster). A batch decides on the sum over its domains.
constexpr size_t kCacheBytes = (size_t)256 << 20;

int setup_domain(Domain &D, const lbm_desc *d, const float *phi, const float *kappa, char *base) {
    D.desc = *d;
    D.L = make_layout(*d, 0);
    D.base = base;
    D.dom = make_dom(*d, D.L);
    D.dom.nt_store = D.L.f_bytes + D.L.g_bytes >= kCacheBytes ? 1 : 0;
    if (d->medium != LBM_MEDIUM_UNIFORM) {
        if (!phi) return fail(LBM_EINVAL, "phi plane required for this medium");
        D.dom.phi = (const float *)(base + D.L.off_phi);
    }
    if (d->medium == LBM_MEDIUM_PHI_KAPPA) {
        if (!kappa) return fail(LBM_EINVAL, "kappa plane required for LBM_MEDIUM_PHI_KAPPA");
        D.dom.kappa = (const float *)(base + D.L.off_kappa);
    }
    if (d->j_plane) D.dom.snu = (const float *)(base + D.L.off_snu);
    return LBM_OK;
}

hipError_t checkpoint(lbm_ctx *c) {
    Domain &D = c->dom[0];
    const int64_t k = D.desc.ckpt_every;
    if (!c->rec_valid || k <= 0 || c->t % k != 0) return hipSuccess;
    const int64_t slot = c->t / k;
    if (slot >= D.L.nck) return hipSuccess;  // beyond capacity: backward will refuse
    char *dst = D.base + D.L.off_ck + (size_t)slot * D.L.ck_slot;
    hipError_t e = hipMemcpyAsync(dst, D.base + D.L.off_f[c->cur], D.L.f_bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && D.desc.thermal.enabled)
        e = hipMemcpyAsync(dst + D.L.f_bytes, D.base + D.L.off_g[c->cur], D.L.g_bytes, hipMemcpyDeviceToDevice,
                           c->stream);
    return e;
}

}  // namespace

namespace {

// cycles advanced by one kernel node of the step graph
int graph_node_steps(const lbm_ctx *c) { return c->tblock; }

// cycles one graph replay advances (a whole number of kernel nodes)
int64_t graph_cycles(const lbm_ctx *c) {
    return (int64_t)(c->graph_steps / graph_node_steps(c)) * graph_node_steps(c);
}

void reset_graphs(lbm_ctx *c) {
    for (auto &g : c->gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// A chain of graph_steps kernel nodes, alternating the buffer parity, built
// node by node (no stream capture, so any stream, including the null stream,
// can launch it). Contains kernel nodes only.
hipError_t build_graph(lbm_ctx *c, int parity) {
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t prev = nullptr;
    const int nodes = c->graph_steps / graph_node_steps(c);
    for (int k = 0; k < nodes && e == hipSuccess; ++k) {
        int p = parity ^ (k & 1);
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        kp.blockDim = dim3(256);
        Dom d;
        int tx = 0, ty = 0, swz = c->sched.swizzle;
        void *args_b[4] = {&c->d_doms, &c->d_tiles, &c->ntiles, &p};
        void *args_s[3] = {&d, &tx, &swz};
        float *no_rec = nullptr;
        void *args_s2[4] = {&d, &tx, &swz, &no_rec};
        void *args_s3[5] = {&d, &tx, &swz, &no_rec, &no_rec};
        void *args_b2[4] = {&c->d_doms, &c->d_tiles2, &c->ntiles2, &p};
        void *args_b4[3] = {&c->d_doms, &c->d_tiles4, &p};
        if (c->batch && c->tblock == 4) {
            kp.func = (void *)step4_batch_kernel_fn(c->storage, c->batch_uniform);
            kp.gridDim = dim3((unsigned)c->ntiles4);
            kp.blockDim = dim3((unsigned)step4_threads());
            kp.kernelParams = args_b4;
        } else if (c->batch && c->tblock == 3) {
            const int g = c->grid3 < c->ntiles2 ? c->grid3 : c->ntiles2;
            kp.func = (void *)step3_batch_kernel_fn(c->storage, c->batch_uniform, g == c->ntiles2);
            kp.gridDim = dim3((unsigned)g);
            kp.blockDim = dim3((unsigned)step3_threads());
            kp.kernelParams = args_b2;
        } else if (c->batch && c->tblock == 2) {
            const int g = c->grid2 < c->ntiles2 ? c->grid2 : c->ntiles2;
            kp.func = (void *)step2_batch_kernel_fn(c->storage, c->batch_thermal, c->batch_uniform, g == c->ntiles2,
                                                    c->tb_threads, c->tb_rows);
            kp.gridDim = dim3((unsigned)g);
            kp.blockDim = dim3((unsigned)c->tb_threads);
            kp.kernelParams = args_b2;
        } else if (c->batch) {
            kp.func = (void *)batch_kernel_fn(c->storage, c->batch_thermal, c->sched);
            kp.gridDim = dim3((unsigned)c->grid);
            kp.kernelParams = args_b;
        } else if (c->tblock == 4) {
            Domain &D = c->dom[0];
            d = dom_for(D, p);
            step4_tiles(D.dom, &tx, &ty);
            kp.func = (void *)step4_kernel_fn(D.dom, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32);
            kp.gridDim = dim3((unsigned)(tx * ty));
            kp.blockDim = dim3((unsigned)step4_threads());
            kp.kernelParams = args_s;
        } else if (c->tblock == 3) {
            Domain &D = c->dom[0];
            d = dom_for(D, p);
            step3_tiles(D.dom, false, &tx, &ty);
            kp.func = (void *)step3_kernel_fn(D.dom, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32, false);
            kp.gridDim = dim3((unsigned)(tx * ty));
            kp.blockDim = dim3((unsigned)step3_single_threads(D.dom, false));
            kp.kernelParams = args_s3;
        } else if (c->tblock == 2) {
            Domain &D = c->dom[0];
            d = dom_for(D, p);
            step2_tiles(D.desc.nx, D.desc.ny, c->tb_rows, &tx, &ty);
            kp.func = (void *)step2_kernel_fn(D.dom, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32, c->tb_threads,
                                              c->tb_rows, false);
            kp.gridDim = dim3((unsigned)(tx * ty));
            kp.blockDim = dim3((unsigned)c->tb_threads);
            kp.kernelParams = args_s2;
        } else {
            Domain &D = c->dom[0];
            d = dom_for(D, p);
            tile_counts(c->sched, D.desc.nx, D.desc.ny, &tx, &ty);
            kp.func = (void *)step_kernel_fn(D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32,
                                             D.desc.thermal.enabled != 0, c->sched);
            kp.gridDim = dim3((unsigned)(tx * ty));
            kp.kernelParams = args_s;
        }
        if (!kp.func) { e = hipErrorInvalidValue; break; }
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        prev = node;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

}  // namespace

// =================================================================== ABI

extern "C" {

int lbm_desc_defaults(lbm_desc *d) {
    if (!d) return fail(LBM_EINVAL, "descriptor is NULL");
    std::memset(d, 0, sizeof(*d));
    d->J = 1.0;
    d->s_e = 1.1;
    d->s_q = 1.2;
    d->phi0 = 1.0;
    d->F_eps = -1.0;
    d->Pi0 = 1.0;
    d->storage = LBM_FP32_DEV;
    d->thermal.sigma = 1.0;
    d->thermal.zeta3 = 1.1;
    d->thermal.zeta4 = 1.1;
    d->thermal.tau_T = 1.0;
    return LBM_OK;
}

int lbm_workspace_size(const lbm_desc *d, int64_t max_steps_recorded, size_t *bytes) {
    int rc = validate(d);
    if (rc) return rc;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    if (d->ckpt_every > 0 && max_steps_recorded < 0) return fail(LBM_EINVAL, "max_steps_recorded must be >= 0");
    *bytes = make_layout(*d, d->ckpt_every > 0 ? max_steps_recorded : 0).total;
    return LBM_OK;
}

int lbm_create(const lbm_desc *d, const float *phi, const float *kappa, void *workspace,
               size_t ws_bytes, void *stream, lbm_ctx **out) {
    int rc = validate(d);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % ALIGN) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    if (d->medium != LBM_MEDIUM_UNIFORM && !phi) return fail(LBM_EINVAL, "phi plane required for this medium");
    if (d->medium == LBM_MEDIUM_PHI_KAPPA && !kappa) return fail(LBM_EINVAL, "kappa plane required");
    // recording capacity follows from the workspace the caller sized
    int64_t cap = 0;
    if (d->ckpt_every > 0) {
        const size_t base = make_layout(*d, 0).total;
        if (ws_bytes < base) return fail(LBM_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, base);
        // largest max_rec with total <= ws_bytes (monotone in max_rec)
        int64_t lo = 0, hi = 1;
        while (make_layout(*d, hi).total <= ws_bytes && hi < ((int64_t)1 << 40)) hi *= 2;
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (make_layout(*d, mid).total <= ws_bytes) lo = mid; else hi = mid;
        }
        cap = lo;
    }
    const Layout L = make_layout(*d, cap);
    if (ws_bytes < L.total) return fail(LBM_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, L.total);

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_EINVAL, "host allocation failed");
    c->stream = (hipStream_t)stream;
    (void)hipGetDevice(&c->device);
    c->dom.resize(1);
    Domain &D = c->dom[0];
    rc = setup_domain(D, d, phi, kappa, (char *)workspace);
    if (rc) { delete c; return rc; }
    D.L = L;
    c->rec_cap = cap;
    // several cycles per pass (the multi-cycle kernels implement bounce-back walls
    // only): from 2^20 nodes isothermal domains take three (8192^2: FP32 177 against
    // 146 GLUPS for two, FP16 190 against 188) and from 2^23 four (8192^2 in 20-step
    // calls: FP32 232 against 201 GLUPS for three, FP16 258 against 251; 4096^2: 227
    // against 196, 247 against 230-240), thermal domains three from 2^22
    // nodes (their 13 LDS planes leave two workgroups per CU: convection 2048^2 92
    // against 84 GLUPS, 4096^2 105 against 88, but 1024^2 80 against 87) and two
    // below; smaller domains take two with 64 x 8 tiles, which keep more workgroups
    // in flight (512^2 cavity: 81 GLUPS against 52 for one cycle per pass and 71
    // for three)
    const int64_t nodes = (int64_t)d->nx * d->ny;
    if (!two_cycle_possible(c)) {
        c->tblock = 1;
    } else if (!d->thermal.enabled && nodes >= ((int64_t)1 << 23)) {
        c->tblock = 4;
    } else if (nodes >= ((int64_t)1 << 20)) {
        const bool three = three_cycle_possible(c) && (!d->thermal.enabled || nodes >= ((int64_t)1 << 22));
        c->tblock = three ? 3 : 2;
    } else {
        c->tblock = 2;
        c->tb_rows = 8;
    }
    // thermal tiles carry 13 LDS planes: 8-row tiles keep four workgroups per CU
    // (measured 86 against 75 GLUPS for 16 rows at 1024^2)
    if (d->thermal.enabled) c->tb_rows = 8;
    if (d->storage == LBM_FP16_DEV) c->sched = Schedule{64, 2, 2, 1};
    hipError_t e = init_domain(D, 0, phi, kappa, c->stream);
    if (e != hipSuccess) {
        rc = device_fail(nullptr, e, "initialisation");
        delete c;
        return rc;
    }
    c->rec_valid = d->ckpt_every > 0;
    e = checkpoint(c);
    if (e != hipSuccess) {
        rc = device_fail(nullptr, e, "checkpoint");
        delete c;
        return rc;
    }
    register_live(c);
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t n) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    // The last pass of every call (the one that brings n to 0) records the
    // velocity of its last collision, u(t - 1) of the final time t, for
    // lbm_reduce's residual; graph replays never end a call.
    while (n > 0) {
        hipError_t e;
        if (c->t == 0) {
            // collide-only first cycle of every domain
            for (Domain &D : c->dom) {
                const Dom d = n == 1 ? dom_rec(D, c->cur) : dom_for(D, c->cur);
                e = launch_step(d, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32, SRC_DIRECT, false, c->sched,
                                c->stream);
                if (e != hipSuccess) return device_fail(c, e, "step launch");
            }
            c->cur ^= 1;
            c->t = 1;
            n -= 1;
            if ((e = checkpoint(c)) != hipSuccess) return device_fail(c, e, "checkpoint copy");
            continue;
        }
        const bool recording = c->rec_valid && c->dom[0].desc.ckpt_every > 0;
        // several cycles per pass where they fit; when recording, a pass never
        // steps over a checkpoint time (the checkpoint needs the state there)
        const bool fused = c->tblock >= 2;
        const int64_t next_ck = recording ? (c->t / c->dom[0].desc.ckpt_every + 1) * c->dom[0].desc.ckpt_every
                                          : INT64_MAX;
        const int64_t gcyc = graph_cycles(c);
        if (gcyc > 0 && !recording && n - 1 >= gcyc) {
            if (!c->gexec[c->cur]) {
                if ((e = build_graph(c, c->cur)) != hipSuccess) return device_fail(c, e, "graph build");
            }
            if ((e = hipGraphLaunch(c->gexec[c->cur], c->stream)) != hipSuccess)
                return device_fail(c, e, "graph launch");
            const int nodes = c->graph_steps / graph_node_steps(c);
            c->cur ^= (nodes & 1);
            c->t += gcyc;
            n -= gcyc;
            continue;
        }
        Domain &D = c->dom[0];
        const int st = D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32;
        int cycles = 1;
        if (fused && c->tblock == 4 && n >= 4 && c->t + 4 <= next_ck) cycles = 4;
        else if (fused && c->tblock >= 3 && n >= 3 && c->t + 3 <= next_ck) cycles = 3;
        else if (fused && n >= 2 && c->t + 2 <= next_ck) cycles = 2;
        const bool last = (n == cycles);
        const Dom d = last ? dom_rec(D, c->cur) : dom_for(D, c->cur);
        Dom *doms = last ? c->d_doms_rec : c->d_doms;
        if (cycles == 4) {
            if (c->batch)
                e = launch_step4_batch(doms, c->d_tiles4, c->ntiles4, c->cur, c->storage, c->batch_uniform, c->stream);
            else
                e = launch_step4(d, st, c->sched.swizzle, c->stream);
        } else if (cycles == 3) {
            if (c->batch)
                e = launch_step3_batch(doms, c->d_tiles2, c->ntiles2, c->cur, c->storage, c->batch_uniform, c->grid3,
                                       c->stream);
            else
                e = launch_step3(d, st, c->sched.swizzle, nullptr, nullptr, c->stream);
        } else if (cycles == 2) {
            if (c->batch)
                e = launch_step2_batch(doms, c->d_tiles2, c->ntiles2, c->cur, c->storage, c->batch_thermal,
                                       c->batch_uniform, c->tb_threads, c->tb_rows, c->grid2, c->stream);
            else
                e = launch_step2(d, st, c->sched.swizzle, c->tb_threads, c->tb_rows, nullptr, c->stream);
        } else {
            if (c->batch)
                e = launch_step_batch(doms, c->d_tiles, c->ntiles, c->cur, c->storage, c->batch_thermal, c->sched,
                                      c->grid, c->stream);
            else
                e = launch_step(d, st, SRC_GATHER, false, c->sched, c->stream);
        }
        if (e != hipSuccess) return device_fail(c, e, "step launch");
        c->cur ^= 1;
        c->t += cycles;
        n -= cycles;
        if ((e = checkpoint(c)) != hipSuccess) return device_fail(c, e, "checkpoint copy");
    }
    return LBM_OK;
}

int lbm_time(const lbm_ctx *c, int64_t *t) {
    if (int rc = check_handle(c)) return rc;
    if (!t) return fail(LBM_EINVAL, "NULL argument");
    *t = c->t;
    return LBM_OK;
}

int lbm_macroscopic(lbm_ctx *c, int32_t k, float *p, float *u, float *T) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = check_domain(c, k))) return rc;
    Domain &D = c->dom[k];
    if (T && !D.desc.thermal.enabled) return fail(LBM_EINVAL, "T requested without thermal model");
    if (!p && !u && !T) return LBM_OK;
    const Dom d = dom_for(D, c->cur);
    const int64_t n = (int64_t)D.desc.nx * D.desc.ny;
    hipError_t e = launch_macroscopic(d, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32, src_now(c->t),
                                      (float)D.desc.Pi0, p, u, u ? u + n : nullptr, T, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "macroscopic launch");
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx *c, int32_t k, float *df, float *dg) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = check_domain(c, k))) return rc;
    if (!df) return fail(LBM_EINVAL, "df is NULL");
    Domain &D = c->dom[k];
    if (dg && !D.desc.thermal.enabled) return fail(LBM_EINVAL, "dg requested without thermal model");
    const Dom d = dom_for(D, c->cur);
    hipError_t e = launch_get_populations(d, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32,
                                          src_now(c->t), df, dg, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "get_populations launch");
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx *c, int32_t k, const float *df, const float *dg) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = check_domain(c, k))) return rc;
    if (!df) return fail(LBM_EINVAL, "df is NULL");
    if (c->batch && c->t != 0) return fail(LBM_ESTATE, "batch domains take a new state only at t = 0");
    Domain &D = c->dom[k];
    if (dg && !D.desc.thermal.enabled) return fail(LBM_EINVAL, "dg given without thermal model");
    // write f(0) into the buffer that becomes current at t = 0
    Dom d = dom_for(D, c->cur ^ 1);  // fout/gout point at buffer `cur`
    hipError_t e = launch_set_populations(d, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32, df, dg,
                                          c->stream);
    if (e != hipSuccess) return device_fail(c, e, "set_populations launch");
    c->t = 0;
    c->rec_valid = D.desc.ckpt_every > 0;
    e = checkpoint(c);
    if (e != hipSuccess) return device_fail(c, e, "checkpoint copy");
    return LBM_OK;
}

}  // extern "C"

namespace {

// The reductions of lbm_reduce with the partial sums (3 doubles per workgroup)
// and the three final sums in the given device memory.
int reduce_into(lbm_ctx *c, int32_t k, double *mass, double *residual, double *partials, double *result) {
    Domain &D = c->dom[k];
    const Dom cur = dom_for(D, c->cur);
    // u(t - 1) was recorded by the last pass of the last lbm_step call
    const float *uprev = c->t >= 1 ? (const float *)(D.base + D.L.off_uprev) : nullptr;
    hipError_t e = launch_reduce(cur, src_now(c->t), uprev, D.desc.storage == LBM_FP16_DEV ? ST_F16 : ST_F32,
                                 partials, result, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "reduce launch");
    double h[3];
    e = hipMemcpyAsync(h, result, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "reduce copy");
    const double n = (double)D.desc.nx * D.desc.ny;
    const double m = n * (5.0 / 3.0) * D.desc.Pi0 + h[0];  // sum_i f_ref_i = (5/3) Pi0 per node
    const double r = (c->t == 0) ? NAN : std::sqrt(h[1]) / std::sqrt(h[2]);
    if (mass) *mass = m;
    if (residual) *residual = r;
    if (!std::isfinite(m) || !std::isfinite(h[1]) || !std::isfinite(h[2]))
        return fail(LBM_EUNSTABLE, "non-finite mass or residual (t = %lld)", (long long)c->t);
    return LBM_OK;
}

// Device address of `scratch` on each device, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int lbm_reduce(lbm_ctx *c, int32_t k, double *mass, double *residual) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = check_domain(c, k))) return rc;
    Domain &D = c->dom[k];
    return reduce_into(c, k, mass, residual, (double *)(D.base + D.L.off_part), (double *)(D.base + D.L.off_res));
}

int lbm_reduce_static(lbm_ctx *c, int32_t k, double *mass, double *residual) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = check_domain(c, k))) return rc;
    const Domain &D = c->dom[k];
    const int nb = reduce_blocks(D.desc.nx, D.desc.ny);
    if (nb > kReduceMaxBlocks)
        return fail(LBM_EINVAL, "the reduction needs %d workgroups of partial sums; the static scratch holds %d",
                    nb, kReduceMaxBlocks);
    double *ptr = nullptr;
    hipError_t e = scratch_on(c->device, &ptr);
    if (e != hipSuccess) return device_fail(c, e, "static scratch address");
    // every partial and final sum is written before it is read: nothing to clear
    return reduce_into(c, k, mass, residual, ptr, ptr + 3 * kReduceMaxBlocks);
}

int lbm_state_bytes(const lbm_ctx *c, size_t *bytes) {
    if (int rc = check_handle(c)) return rc;
    if (!bytes) return fail(LBM_EINVAL, "NULL argument");
    if (c->batch) return fail(LBM_ENOTSUP, "save/load is per single-domain context");
    const Domain &D = c->dom[0];
    *bytes = 64 + D.L.f_bytes + (D.desc.thermal.enabled ? D.L.g_bytes : 0) + 2 * D.L.p_bytes;
    return LBM_OK;
}

namespace {
// FNV-1a over every descriptor field that gives a saved state its meaning,
// field by field (struct padding never enters): grid, boundaries, lid,
// viscosity, J and its plane, relaxation rates, medium, forcing, Pi0, storage
// and, with the thermal model on, every thermal parameter. ckpt_every only
// decides recording and is left out.
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void *v, size_t n) {
        const unsigned char *p = (const unsigned char *)v;
        for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ull; }
    }
    void i32(int32_t v) { add(&v, sizeof(v)); }
    void f64(double v) { add(&v, sizeof(v)); }
};

uint64_t desc_hash(const lbm_desc &d) {
    Fnv f;
    f.i32(d.nx); f.i32(d.ny); f.i32(d.bc_x); f.i32(d.bc_y); f.f64(d.lid_ux);
    f.f64(d.nu); f.f64(d.J); f.f64(d.s_e); f.f64(d.s_q);
    f.i32(d.medium); f.f64(d.phi0); f.f64(d.kappa0); f.f64(d.dp); f.f64(d.F_eps);
    f.f64(d.ax); f.f64(d.ay); f.f64(d.Pi0); f.i32(d.storage); f.i32(d.j_plane);
    const lbm_thermal &t = d.thermal;
    f.i32(t.enabled);
    if (t.enabled) {
        f.f64(t.tau_T); f.f64(t.sigma); f.f64(t.zeta3); f.f64(t.zeta4);
        f.f64(t.Th); f.f64(t.Tc); f.f64(t.T0); f.f64(t.g_beta);
    }
    return f.h;
}

// Snapshot header (64 bytes): magic, descriptor hash, t, payload bytes; then
// the populations f (and g) in the current buffer's layout and the two u(t - 1)
// planes.
constexpr uint64_t kSnapMagic = 0x4d52544c424d3032ull;  // "MRTLBM02"
}  // namespace

int lbm_save(lbm_ctx *c, void *host_buf, size_t bytes) {
    int rc = check_ctx(c);
    if (rc) return rc;
    size_t need;
    if ((rc = lbm_state_bytes(c, &need))) return rc;
    if (!host_buf || bytes < need) return fail(LBM_EINVAL, "host buffer too small (%zu < %zu)", bytes, need);
    Domain &D = c->dom[0];
    char *h = (char *)host_buf;
    std::memset(h, 0, 64);
    const uint64_t hash = desc_hash(D.desc), payload = need - 64;
    std::memcpy(h, &kSnapMagic, 8);
    std::memcpy(h + 8, &hash, 8);
    std::memcpy(h + 16, &c->t, 8);
    std::memcpy(h + 24, &payload, 8);
    size_t o = 64;
    hipError_t e = hipMemcpyAsync(h + o, D.base + D.L.off_f[c->cur], D.L.f_bytes, hipMemcpyDeviceToHost, c->stream);
    o += D.L.f_bytes;
    if (e == hipSuccess && D.desc.thermal.enabled) {
        e = hipMemcpyAsync(h + o, D.base + D.L.off_g[c->cur], D.L.g_bytes, hipMemcpyDeviceToHost, c->stream);
        o += D.L.g_bytes;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(h + o, D.base + D.L.off_uprev, 2 * D.L.p_bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "save");
    return LBM_OK;
}

int lbm_load(lbm_ctx *c, const void *host_buf, size_t bytes) {
    int rc = check_ctx(c);
    if (rc) return rc;
    size_t need;
    if ((rc = lbm_state_bytes(c, &need))) return rc;
    if (!host_buf || bytes < 64) return fail(LBM_EINVAL, "snapshot too small (%zu bytes)", bytes);
    Domain &D = c->dom[0];
    const char *h = (const char *)host_buf;
    uint64_t magic, hash, payload;
    int64_t t;
    std::memcpy(&magic, h, 8);
    std::memcpy(&hash, h + 8, 8);
    std::memcpy(&t, h + 16, 8);
    std::memcpy(&payload, h + 24, 8);
    if (magic != kSnapMagic) return fail(LBM_EINVAL, "not a snapshot of this library");
    if (hash != desc_hash(D.desc)) return fail(LBM_EINVAL, "snapshot was taken with a different descriptor");
    if (payload != need - 64)
        return fail(LBM_EINVAL, "snapshot holds %llu bytes of state, this context %zu", (unsigned long long)payload,
                    need - 64);
    if (bytes < need) return fail(LBM_EINVAL, "snapshot too small (%zu < %zu)", bytes, need);
    if (t < 0) return fail(LBM_EINVAL, "corrupt snapshot time");
    size_t o = 64;
    hipError_t e = hipMemcpyAsync(D.base + D.L.off_f[c->cur], h + o, D.L.f_bytes, hipMemcpyHostToDevice, c->stream);
    o += D.L.f_bytes;
    if (e == hipSuccess && D.desc.thermal.enabled) {
        e = hipMemcpyAsync(D.base + D.L.off_g[c->cur], h + o, D.L.g_bytes, hipMemcpyHostToDevice, c->stream);
        o += D.L.g_bytes;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(D.base + D.L.off_uprev, h + o, 2 * D.L.p_bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "load");
    c->t = t;
    c->rec_valid = false;  // the recorded trajectory no longer leads here
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *c) {
    if (!c) return LBM_OK;
    {
        std::lock_guard<std::mutex> lock(g_live_mu);
        if (!g_live.erase(c)) return fail(LBM_EINVAL, "not a live context (destroyed, or never created)");
    }
    reset_graphs(c);
    delete c;
    return LBM_OK;
}

const char *lbm_strerror(int s) {
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ESTATE: return "invalid state for this call";
    case LBM_EDEVICE: return "device error (context poisoned)";
    case LBM_EUNSTABLE: return "non-finite mass or residual";
    case LBM_ENOTSUP: return "not supported";
    default: return "unknown status";
    }
}

const char *lbm_last_error(void) { return g_last_error.c_str(); }

int lbm_schedule(const lbm_ctx *c, int32_t *tile_w, int32_t *vec, int32_t *rows, int32_t *grid) {
    if (int rc = check_handle(c)) return rc;
    if (tile_w) *tile_w = c->sched.tile_w;
    if (vec) *vec = c->sched.vec;
    if (rows) *rows = c->sched.rows;
    if (grid) {
        if (c->batch) *grid = c->grid;
        else {
            int tx, ty;
            tile_counts(c->sched, c->dom[0].desc.nx, c->dom[0].desc.ny, &tx, &ty);
            *grid = tx * ty;
        }
    }
    return LBM_OK;
}

int lbm_time_blocking(const lbm_ctx *c, int32_t *cycles_per_pass, int32_t *threads, int32_t *rows,
                      int32_t *grid) {
    if (int rc = check_handle(c)) return rc;
    int32_t nt = c->tb_threads, nr = c->tb_rows, ng = 0;
    if (c->batch && c->tblock == 4) {
        nt = step4_threads();
        nr = step4_rows();
        ng = c->ntiles4;
    } else if (c->batch) {
        if (c->tblock == 3) nt = step3_threads();
        ng = c->tblock == 3 ? c->grid3 : c->grid2;
    } else if (c->tblock == 4) {
        int tx, ty;
        step4_tiles(c->dom[0].dom, &tx, &ty);
        nt = step4_threads();
        nr = step4_rows();
        ng = tx * ty;
    } else if (c->tblock == 3) {
        const Dom &d = c->dom[0].dom;
        int tx, ty;
        step3_tiles(d, false, &tx, &ty);
        nt = step3_single_threads(d, false);
        nr = step3_single_rows(d, false);
        ng = tx * ty;
    } else {
        int tx, ty;
        step2_tiles(c->dom[0].desc.nx, c->dom[0].desc.ny, c->tb_rows, &tx, &ty);
        ng = tx * ty;
    }
    if (cycles_per_pass) *cycles_per_pass = c->tblock;
    if (threads) *threads = nt;
    if (rows) *rows = nr;
    if (grid) *grid = ng;
    return LBM_OK;
}

int lbm_set_schedule(lbm_ctx *c, int32_t tile_w, int32_t vec, int32_t rows, int32_t swizzle) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(LBM_ENOTSUP, "a batch's schedule is chosen by its autotuner");
    const Schedule s{tile_w, vec, rows, swizzle ? 1 : 0};
    if (!schedule_supported(s))
        return fail(LBM_EINVAL, "unsupported schedule %d x %d x %d", tile_w, vec, rows);
    c->sched = s;
    reset_graphs(c);
    return LBM_OK;
}

namespace {
hipError_t upload_tiles2(lbm_ctx *c, int rows);
}  // namespace

int lbm_set_time_blocking(lbm_ctx *c, int32_t cycles_per_pass) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (cycles_per_pass < 1 || cycles_per_pass > 4) return fail(LBM_EINVAL, "cycles per pass must be 1, 2, 3 or 4");
    if (cycles_per_pass == 4 && (c->batch ? c->batch_thermal : c->dom[0].desc.thermal.enabled != 0))
        return fail(LBM_ENOTSUP, "four cycles per pass take isothermal domains");
    if (cycles_per_pass == 3 && c->batch && c->batch_thermal)
        return fail(LBM_ENOTSUP, "thermal batches advance one or two cycles per pass");
    if (cycles_per_pass >= 2 && any_on_node_walls(c))
        return fail(LBM_ENOTSUP, "on-node (extrapolated) walls advance one cycle per pass");
    if (cycles_per_pass >= 2 && !two_cycle_possible(c))
        return fail(LBM_ENOTSUP, "a population buffer of 4 GiB or more advances one cycle per pass");
    if (cycles_per_pass == 2 && c->batch && c->grid2 <= 0)
        return fail(LBM_ENOTSUP, "this batch has no tuned two-cycle schedule");
    if (cycles_per_pass == 4 && c->batch && !c->four_ok)
        return fail(LBM_ENOTSUP, "this batch has no four-cycle tile table");
    if (cycles_per_pass >= 3 && c->batch) {
        if (c->grid3 <= 0) return fail(LBM_ENOTSUP, "this batch has no tuned three-cycle schedule");
        if (c->tb_rows != 16) {
            // the three-cycle kernel walks 64 x 16 tiles (also for the three-cycle
            // passes of mode 4); the two-cycle kernel then uses the same table
            c->tb_rows = 16;
            hipError_t e = upload_tiles2(c, 16);
            if (e != hipSuccess) return device_fail(c, e, "tile table upload");
        }
    }
    c->tblock = cycles_per_pass;
    reset_graphs(c);
    return LBM_OK;
}

int lbm_set_two_cycle_tile(lbm_ctx *c, int32_t threads, int32_t rows) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!step2_shape_supported(threads, rows))
        return fail(LBM_EINVAL, "unsupported two-cycle tile: %d threads, %d rows", threads, rows);
    if (c->batch) return fail(LBM_ENOTSUP, "a batch's two-cycle tile is chosen by its autotuner");
    c->tb_threads = threads;
    c->tb_rows = rows;
    reset_graphs(c);
    return LBM_OK;
}

int lbm_set_viscosity_ratio(lbm_ctx *c, int32_t k, const float *J) {
    int rc = check_ctx(c);
    if (rc) return rc;
    rc = check_domain(c, k);
    if (rc) return rc;
    Domain &D = c->dom[k];
    if (!D.desc.j_plane) return fail(LBM_ESTATE, "domain %d was created without a viscosity-ratio plane (j_plane = 0)", k);
    if (!J) return fail(LBM_EINVAL, "J is NULL");
    if (c->rec_valid && c->t > 0)
        return fail(LBM_ESTATE, "the recorded forward pass has started; set J at t = 0");
    // check on the device first, so that a rejected plane leaves the old one in place
    int *flag = (int *)(D.base + D.L.off_part);
    hipError_t e = launch_fill_zero(flag, 16, c->stream);
    if (e == hipSuccess)
        e = launch_snu_plane(J, 0.0, D.desc.nu, nullptr, D.L.pitch, D.desc.nx, D.desc.ny, flag, c->stream);
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "viscosity ratio");
    if (bad) return fail(LBM_EINVAL, "J must be finite and > 0 at every node");
    e = launch_snu_plane(J, 0.0, D.desc.nu, (float *)(D.base + D.L.off_snu), D.L.pitch, D.desc.nx,
                         D.desc.ny, nullptr, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "viscosity ratio");
    return LBM_OK;
}

int lbm_set_graph_steps(lbm_ctx *c, int32_t steps) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (steps < 0 || steps > 4096) return fail(LBM_EINVAL, "graph steps must lie in [0, 4096]");
    c->graph_steps = steps;
    reset_graphs(c);
    return LBM_OK;
}

}  // extern "C"

// ============================================================ batches

namespace {

const Schedule kCandidates[] = {{256, 1, 1, 0}, {256, 1, 2, 0}, {128, 1, 1, 0}, {128, 1, 2, 0},
                                {64, 1, 2, 0},  {64, 1, 4, 0},  {128, 2, 1, 0}, {64, 2, 2, 0},
                                {64, 4, 1, 0},  {32, 4, 2, 0},  {64, 4, 2, 0},  {16, 4, 4, 0}};

int validate_batch(int32_t n, const lbm_desc *descs) {
    if (n < 1) return fail(LBM_EINVAL, "batch needs n >= 1 domains");
    if (!descs) return fail(LBM_EINVAL, "descs is NULL");
    for (int32_t k = 0; k < n; ++k) {
        int rc = validate(&descs[k]);
        if (rc) return fail(rc, "domain %d: %s", k, g_last_error.c_str());
        if ((descs[k].thermal.enabled != 0) != (descs[0].thermal.enabled != 0))
            return fail(LBM_ENOTSUP, "domain %d: a batch is thermal in every domain or in none", k);
        if (descs[k].ckpt_every != 0) return fail(LBM_ENOTSUP, "domain %d: batches do not record for the adjoint", k);
        if (descs[k].storage != descs[0].storage) return fail(LBM_EINVAL, "domain %d: storage differs from domain 0", k);
    }
    return LBM_OK;
}

int64_t batch_tiles(int32_t n, const lbm_desc *descs, const Schedule &s) {
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) {
        int tx, ty;
        tile_counts(s, descs[k].nx, descs[k].ny, &tx, &ty);
        total += (int64_t)tx * ty;
    }
    return total;
}

struct BatchLayout {
    std::vector<size_t> off;  // per-domain base offsets
    size_t off_doms = 0, off_tiles = 0, off_tiles2 = 0, off_tiles4 = 0, total = 0;
    int64_t max_tiles = 0, max_tiles2 = 0, tiles4 = 0;
};

const int kTwoCycleShapes[][2] = {{256, 16}, {512, 16}, {256, 8}, {512, 8}};

int64_t batch_tiles2(int32_t n, const lbm_desc *descs, int rows) {
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) {
        int tx, ty;
        step2_tiles(descs[k].nx, descs[k].ny, rows, &tx, &ty);
        total += (int64_t)tx * ty;
    }
    return total;
}

BatchLayout batch_layout(int32_t n, const lbm_desc *descs) {
    BatchLayout B;
    size_t o = 0;
    for (int32_t k = 0; k < n; ++k) {
        B.off.push_back(o);
        o = align_up(o + make_layout(descs[k], 0).total, ALIGN);
    }
    for (const Schedule &s : kCandidates) {
        const int64_t t = batch_tiles(n, descs, s);
        if (t > B.max_tiles) B.max_tiles = t;
    }
    B.off_doms = o;
    o = align_up(o + sizeof(Dom) * 4 * (size_t)n, ALIGN);  // two per parity: plain and recording
    B.off_tiles = o;
    o = align_up(o + sizeof(int4) * (size_t)B.max_tiles, ALIGN);
    for (const auto &sh : kTwoCycleShapes) {
        const int64_t t = batch_tiles2(n, descs, sh[1]);
        if (t > B.max_tiles2) B.max_tiles2 = t;
    }
    B.off_tiles2 = o;
    o = align_up(o + sizeof(int4) * (size_t)B.max_tiles2, ALIGN);
    B.tiles4 = batch_tiles2(n, descs, step4_rows());
    B.off_tiles4 = o;
    o = align_up(o + sizeof(int4) * (size_t)B.tiles4, ALIGN);
    B.total = o;
    return B;
}

void fill_tiles(const lbm_ctx *c, const Schedule &s, std::vector<int4> &out) {
    out.clear();
    for (size_t k = 0; k < c->dom.size(); ++k) {
        int tx, ty;
        tile_counts(s, c->dom[k].desc.nx, c->dom[k].desc.ny, &tx, &ty);
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) out.push_back(make_int4((int)k, x, y, 0));
    }
}

hipError_t upload_tiles2(lbm_ctx *c, int rows) {
    c->h_tiles2.clear();
    for (size_t k = 0; k < c->dom.size(); ++k) {
        int tx, ty;
        step2_tiles(c->dom[k].desc.nx, c->dom[k].desc.ny, rows, &tx, &ty);
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) c->h_tiles2.push_back(make_int4((int)k, x, y, 0));
    }
    c->ntiles2 = (int)c->h_tiles2.size();
    hipError_t e = hipMemcpyAsync(c->d_tiles2, c->h_tiles2.data(), sizeof(int4) * c->h_tiles2.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

// the 64 x 26 tiles of the batched four-cycle kernel, in their own table
hipError_t upload_tiles4(lbm_ctx *c) {
    c->h_tiles4.clear();
    for (size_t k = 0; k < c->dom.size(); ++k) {
        int tx, ty;
        step4_tiles(c->dom[k].dom, &tx, &ty);
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) c->h_tiles4.push_back(make_int4((int)k, x, y, 0));
    }
    c->ntiles4 = (int)c->h_tiles4.size();
    hipError_t e = hipMemcpyAsync(c->d_tiles4, c->h_tiles4.data(), sizeof(int4) * c->h_tiles4.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

uint64_t batch_signature(const lbm_ctx *c) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) { h ^= (uint64_t)((v >> (8 * b)) & 0xff); h *= 1099511628211ull; }
    };
    mix((int64_t)c->dom.size());
    mix(c->storage);
    mix(c->batch_thermal ? 1 : 0);
    for (const Domain &D : c->dom) {
        mix(D.desc.nx); mix(D.desc.ny); mix(D.desc.bc_x); mix(D.desc.bc_y); mix(D.desc.medium);
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        for (const char *p = prop.gcnArchName; *p; ++p) mix(*p);
        mix(prop.multiProcessorCount);
    }
    return h;
}

// One tuning result: the one-cycle schedule and grid, the two-cycle shape
// and grid, the three-cycle grid, whether the four-cycle pass (one workgroup
// per tile) was timed, and which mode is fastest.
struct Tuned {
    Schedule s{128, 1, 2, 0};
    int grid = 0;
    int tblock = 1, tb_threads = 512, tb_rows = 16, grid2 = 0, grid3 = 0, four = 0;
};

bool cache_lookup(const char *path, uint64_t sig, Tuned &out) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        unsigned long long key;
        int tw, v, r, g, tb, tt, tr, g2, g3, f4;
        if (sscanf(line, "%llx %d %d %d %d %d %d %d %d %d %d", &key, &tw, &v, &r, &g, &tb, &tt, &tr, &g2, &g3,
                   &f4) != 11)
            continue;
        const Schedule cand{tw, v, r, 0};
        if (key == sig && schedule_supported(cand) && g > 0 && tb >= 1 && tb <= 4 &&
            step2_shape_supported(tt, tr) && g2 > 0 && g3 >= 0 && (f4 == 0 || f4 == 1) &&
            (tb < 3 || (g3 > 0 && tr == 16)) && (tb < 4 || f4 == 1)) {
            out.s = cand; out.grid = g; out.tblock = tb; out.tb_threads = tt; out.tb_rows = tr; out.grid2 = g2;
            out.grid3 = g3;
            out.four = f4;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, uint64_t sig, const Tuned &t) {
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%016llx %d %d %d %d %d %d %d %d %d %d\n", (unsigned long long)sig, t.s.tile_w, t.s.vec, t.s.rows,
            t.grid, t.tblock, t.tb_threads, t.tb_rows, t.grid2, t.grid3, t.four);
    fclose(f);
}

hipError_t upload_tiles(lbm_ctx *c, const Schedule &s) {
    fill_tiles(c, s, c->h_tiles);
    c->ntiles = (int)c->h_tiles.size();
    hipError_t e = hipMemcpyAsync(c->d_tiles, c->h_tiles.data(), sizeof(int4) * c->h_tiles.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

// Times every (schedule, grid) candidate on the batch. Each timing launch
// reads buffer 0 (the rest state f(0)) and writes buffer 1, which the first
// real cycle overwrites, so tuning leaves the state untouched.
hipError_t autotune(lbm_ctx *c, Tuned &best) {
    int dev = 0, ncu = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) { (void)hipEventDestroy(a); return e; }
    auto time_it = [&](auto launch, float &ms) -> hipError_t {
        hipError_t r = hipSuccess;
        for (int w = 0; w < 2 && r == hipSuccess; ++w) r = launch();
        if (r == hipSuccess) r = hipEventRecord(a, c->stream);
        for (int w = 0; w < 5 && r == hipSuccess; ++w) r = launch();
        if (r == hipSuccess) r = hipEventRecord(b, c->stream);
        if (r == hipSuccess) r = hipEventSynchronize(b);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, a, b);
        return r;
    };
    float best1 = 1e30f, best2 = 1e30f;  // ms per cycle
    for (const Schedule &s : kCandidates) {
        if ((e = upload_tiles(c, s)) != hipSuccess) break;
        const int grids[5] = {2 * ncu, 4 * ncu, 8 * ncu, 16 * ncu, c->ntiles};
        for (int g : grids) {
            if (g > c->ntiles) g = c->ntiles;
            float ms = 0.0f;
            e = time_it([&] { return launch_step_batch(c->d_doms, c->d_tiles, c->ntiles, 0, c->storage,
                                                       c->batch_thermal, s, g,
                                                       c->stream); }, ms);
            if (e != hipSuccess) break;
            if (ms < best1) { best1 = ms; best.s = s; best.grid = g; }
        }
        if (e != hipSuccess) break;
    }
    const bool two_cycle_ok = two_cycle_possible(c);
    for (const auto &sh : kTwoCycleShapes) {
        if (e != hipSuccess || !two_cycle_ok) break;
        if ((e = upload_tiles2(c, sh[1])) != hipSuccess) break;
        const int grids[4] = {2 * ncu, 4 * ncu, 8 * ncu, c->ntiles2};
        for (int g : grids) {
            if (g > c->ntiles2) g = c->ntiles2;
            float ms = 0.0f;
            e = time_it([&] { return launch_step2_batch(c->d_doms, c->d_tiles2, c->ntiles2, 0, c->storage, c->batch_thermal,
                                                        c->batch_uniform, sh[0], sh[1], g, c->stream); }, ms);
            if (e != hipSuccess) break;
            if (0.5f * ms < best2) {
                best2 = 0.5f * ms;
                best.tb_threads = sh[0]; best.tb_rows = sh[1]; best.grid2 = g;
            }
        }
    }
    // three cycles per pass (isothermal batches): the 64 x 16 tiles of the
    // two-cycle table
    float best3 = 1e30f;
    if (e == hipSuccess && two_cycle_ok && !c->batch_thermal && (e = upload_tiles2(c, 16)) == hipSuccess) {
        const int grids[4] = {2 * ncu, 4 * ncu, 8 * ncu, c->ntiles2};
        for (int g : grids) {
            if (g > c->ntiles2) g = c->ntiles2;
            float ms = 0.0f;
            e = time_it([&] { return launch_step3_batch(c->d_doms, c->d_tiles2, c->ntiles2, 0, c->storage,
                                                        c->batch_uniform, g, c->stream); }, ms);
            if (e != hipSuccess) break;
            if (ms / 3.0f < best3) { best3 = ms / 3.0f; best.grid3 = g; }
        }
    }
    // four cycles per pass (isothermal batches): one workgroup per 64 x 26 tile
    float best4 = 1e30f;
    if (e == hipSuccess && two_cycle_ok && !c->batch_thermal && (e = upload_tiles4(c)) == hipSuccess) {
        float ms = 0.0f;
        e = time_it([&] { return launch_step4_batch(c->d_doms, c->d_tiles4, c->ntiles4, 0, c->storage,
                                                    c->batch_uniform, c->stream); }, ms);
        if (e == hipSuccess) {
            best4 = ms / 4.0f;
            best.four = 1;
        }
    }
    best.tblock = (best2 < best1) ? 2 : 1;
    if (best3 < best1 && best3 < best2) {
        best.tblock = 3;
        best.tb_rows = 16;   // the three-cycle kernel walks the 64 x 16 table
    }
    if (best4 < best1 && best4 < best2 && best4 < best3) {
        best.tblock = 4;
        best.tb_rows = 16;   // its three-cycle passes walk the 64 x 16 table
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
}

}  // namespace

extern "C" int lbm_batch_workspace_size(int32_t n, const lbm_desc *descs, size_t *bytes) {
    int rc = validate_batch(n, descs);
    if (rc) return rc;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    *bytes = batch_layout(n, descs).total;
    return LBM_OK;
}

extern "C" int lbm_create_batch(int32_t n, const lbm_desc *descs, const float *const *phis,
                                const float *const *kappas, void *workspace, size_t ws_bytes,
                                void *stream, const char *tune_cache, lbm_ctx **out) {
    int rc = validate_batch(n, descs);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % ALIGN) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    const BatchLayout B = batch_layout(n, descs);
    if (ws_bytes < B.total) return fail(LBM_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, B.total);
    for (int32_t k = 0; k < n; ++k) {
        if (descs[k].medium != LBM_MEDIUM_UNIFORM && (!phis || !phis[k]))
            return fail(LBM_EINVAL, "domain %d: phi plane required", k);
        if (descs[k].medium == LBM_MEDIUM_PHI_KAPPA && (!kappas || !kappas[k]))
            return fail(LBM_EINVAL, "domain %d: kappa plane required", k);
    }
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_EINVAL, "host allocation failed");
    c->stream = (hipStream_t)stream;
    (void)hipGetDevice(&c->device);
    c->batch = true;
    c->storage = descs[0].storage == LBM_FP16_DEV ? ST_F16 : ST_F32;
    c->batch_thermal = descs[0].thermal.enabled != 0;
    c->dom.resize((size_t)n);
    char *base = (char *)workspace;
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < n && e == hipSuccess; ++k) {
        Domain &D = c->dom[(size_t)k];
        const float *phi = phis ? phis[k] : nullptr;
        const float *kap = kappas ? kappas[k] : nullptr;
        rc = setup_domain(D, &descs[k], phi, kap, base + B.off[(size_t)k]);
        if (rc) { delete c; return rc; }
        e = init_domain(D, 0, phi, kap, c->stream);
    }
    c->batch_uniform = true;
    for (const Domain &D : c->dom)
        if (medium_kind(D.dom) != MK_UNIFORM) c->batch_uniform = false;
    c->d_doms = (Dom *)(base + B.off_doms);
    c->d_tiles = (int4 *)(base + B.off_tiles);
    size_t state_bytes = 0;
    for (const Domain &D : c->dom) state_bytes += D.L.f_bytes + D.L.g_bytes;
    c->h_doms.resize(4 * (size_t)n);
    c->d_doms_rec = c->d_doms + 2 * (size_t)n;
    for (int32_t k = 0; k < n; ++k) {
        c->dom[(size_t)k].dom.nt_store = state_bytes >= kCacheBytes ? 1 : 0;
        c->h_doms[2 * (size_t)k] = dom_for(c->dom[(size_t)k], 0);
        c->h_doms[2 * (size_t)k + 1] = dom_for(c->dom[(size_t)k], 1);
        c->h_doms[2 * (size_t)n + 2 * (size_t)k] = dom_rec(c->dom[(size_t)k], 0);
        c->h_doms[2 * (size_t)n + 2 * (size_t)k + 1] = dom_rec(c->dom[(size_t)k], 1);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_doms, c->h_doms.data(), sizeof(Dom) * c->h_doms.size(), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->d_tiles2 = (int4 *)(base + B.off_tiles2);
    c->d_tiles4 = (int4 *)(base + B.off_tiles4);
    Tuned best;
    const uint64_t sig = batch_signature(c);
    if (e == hipSuccess && !cache_lookup(tune_cache, sig, best)) {
        e = autotune(c, best);
        if (e == hipSuccess) cache_store(tune_cache, sig, best);
    }
    if (e == hipSuccess) {
        c->sched = best.s;
        e = upload_tiles(c, best.s);
        c->grid = best.grid > c->ntiles ? c->ntiles : best.grid;
    }
    if (e == hipSuccess) {
        c->tb_threads = best.tb_threads;
        c->tb_rows = best.tb_rows;
        e = upload_tiles2(c, best.tb_rows);
        c->grid2 = best.grid2 > c->ntiles2 ? c->ntiles2 : best.grid2;
        c->grid3 = best.grid3 > c->ntiles2 ? c->ntiles2 : best.grid3;
        c->tblock = best.tblock;
    }
    if (e == hipSuccess && !c->batch_thermal && two_cycle_possible(c)) {
        e = upload_tiles4(c);
        c->four_ok = e == hipSuccess;
    }
    // a tuning-cache entry cannot select a mode this batch does not have
    if (c->batch_thermal && c->tblock > 2) c->tblock = 2;
    if (c->tblock == 4 && !c->four_ok) c->tblock = 3;
    if (c->tblock >= 2 && !two_cycle_possible(c)) c->tblock = 1;
    if (e != hipSuccess) {
        rc = device_fail(nullptr, e, "batch creation");
        delete c;
        return rc;
    }
    c->graph_steps = 32;
    register_live(c);
    *out = c;
    return LBM_OK;
}

namespace {

// The backward pass shared by lbm_backward and lbm_backward_params; theta
// (host, 4 doubles) receives dL/dnu, dL/da_x, dL/da_y, dL/dU_lid when non-NULL.
int backward_impl(lbm_ctx *c, const float *dL_du, float *dL_dphi, float *dL_dkappa, double *theta) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(LBM_ENOTSUP, "the adjoint runs on single-domain contexts");
    Domain &D = c->dom[0];
    const lbm_desc &d = D.desc;
    if (!dL_du) return fail(LBM_EINVAL, "dL_du is required");
    if (!dL_dphi && !theta) return fail(LBM_EINVAL, "dL_dphi is required");
    if (d.ckpt_every <= 0) return fail(LBM_ESTATE, "context was created without recording (ckpt_every = 0)");
    if (on_node_walls(d)) return fail(LBM_ENOTSUP, "adjoint of on-node (extrapolated) walls is not implemented");
    if (d.storage != LBM_FP32_DEV) return fail(LBM_ENOTSUP, "adjoint needs FP32 storage");
    if (dL_dphi && d.medium == LBM_MEDIUM_UNIFORM) return fail(LBM_ENOTSUP, "dL/dphi needs a porosity plane");
    const bool th = d.thermal.enabled != 0;
    // The recomputation's passes record u at every cycle and give the same bits
    // whatever their length; from 2^22 nodes isothermal domains in mode 3 or 4 take
    // four-cycle recording passes (2048^2: backward 256 ms against 274.5 with
    // three-cycle ones).
    const bool rec4 = !th && (c->tblock == 4 || (c->tblock == 3 && (int64_t)d.nx * d.ny >= ((int64_t)1 << 22)));
    if (dL_dkappa && d.medium != LBM_MEDIUM_PHI_KAPPA) return fail(LBM_EINVAL, "dL_dkappa needs LBM_MEDIUM_PHI_KAPPA");
    if (!c->rec_valid) return fail(LBM_ESTATE, "no recorded trajectory leads to the current state");
    const int64_t T = c->t, k = d.ckpt_every;
    if (T > 0 && (T - 1) / k >= D.L.nck)
        return fail(LBM_ESTATE, "t = %lld exceeds the recorded capacity", (long long)T);

    const Layout &L = D.L;
    float *lam[2] = {(float *)(D.base + L.off_lam[0]), (float *)(D.base + L.off_lam[1])};
    float *gphi = (float *)(D.base + L.off_gphi);
    float *gk = d.medium == LBM_MEDIUM_PHI_KAPPA ? (float *)(D.base + L.off_gkappa) : nullptr;
    float *urec = (float *)(D.base + L.off_urec);
    const size_t rstride = 5 * (size_t)L.plane;  // floats per recorded step
    float *lamg[2] = {th ? (float *)(D.base + L.off_lamg[0]) : nullptr, th ? (float *)(D.base + L.off_lamg[1]) : nullptr};
    double *acc = theta ? (double *)(D.base + L.off_theta) : nullptr;
    double *acc_seed = acc ? acc + 4 * adjoint_theta_offset(d.nx, d.ny, 0) : nullptr;
    double *acc_step = acc ? acc + 4 * adjoint_theta_offset(d.nx, d.ny, 1) : nullptr;
    double *acc_step2 = acc ? acc + 4 * adjoint_theta_offset(d.nx, d.ny, 2) : nullptr;
    hipStream_t st = c->stream;

    hipError_t e = hipSuccess;
    if (acc) e = launch_fill_zero(acc, sizeof(double) * 4 * (L.theta_slots + 1), st);
    if (e == hipSuccess)
        e = th ? launch_adjoint_seed_thermal(dom_for(D, c->cur), src_now(T), dL_du, lam[0], lamg[0], gphi, gk, acc_seed, st)
               : launch_adjoint_seed(dom_for(D, c->cur), src_now(T), dL_du, lam[0], gphi, gk, acc_seed, st);
    if (e != hipSuccess) return device_fail(c, e, "adjoint seed");
    int la = 0;  // lam[la] holds a(t + 1)
    if (T > 0) {
        for (int64_t s0 = ((T - 1) / k) * k; s0 >= 0; s0 -= k) {
            const int64_t s1 = (s0 + k < T) ? s0 + k : T;
            // recompute the segment from its checkpoint, recording u(t) (and the stress moments)
            const char *slot = D.base + L.off_ck + (size_t)(s0 / k) * L.ck_slot;
            e = hipMemcpyAsync(D.base + L.off_rf[0], slot, L.f_bytes, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess && th)
                e = hipMemcpyAsync(D.base + L.off_rg[0], slot + L.f_bytes, L.g_bytes, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return device_fail(c, e, "checkpoint restore");
            int p = 0;
            for (int64_t t = s0; t < s1;) {
                Dom dr = D.dom;
                dr.fin = D.base + L.off_rf[p];
                dr.fout = D.base + L.off_rf[p ^ 1];
                dr.urec = urec + (size_t)(t - s0) * rstride;
                dr.rec_stress = theta ? 1 : 0;
                if (th) {
                    dr.gin = (const float *)(D.base + L.off_rg[p]);
                    dr.gout = (float *)(D.base + L.off_rg[p ^ 1]);
                }
                if (rec4 && t > 0 && t + 3 < s1) {
                    // four cycles in one pass, recording at t, t + 1, t + 2 and t + 3
                    e = launch_step4_rec(dr, c->sched.swizzle, dr.urec + rstride, dr.urec + 2 * rstride,
                                         dr.urec + 3 * rstride, st);
                    t += 4;
                } else if (c->tblock >= 3 && t > 0 && t + 2 < s1) {
                    // three cycles in one pass, recording at t, t + 1 and t + 2
                    e = launch_step3(dr, ST_F32, c->sched.swizzle, dr.urec + rstride, dr.urec + 2 * rstride, st);
                    t += 3;
                } else if (c->tblock >= 2 && t > 0 && t + 1 < s1) {
                    // two cycles in one pass, recording at t and t + 1 (with dT when thermal)
                    e = launch_step2(dr, ST_F32, c->sched.swizzle, c->tb_threads, c->tb_rows, dr.urec + rstride, st);
                    t += 2;
                } else {
                    e = launch_step(dr, ST_F32, t == 0 ? SRC_DIRECT : SRC_GATHER, true, c->sched, st);
                    t += 1;
                }
                if (e != hipSuccess) return device_fail(c, e, "recompute step");
                p ^= 1;
            }
            // backward through the segment (two or three steps per pass in the multi-cycle modes)
            for (int64_t t = s1 - 1; t >= s0;) {
                const float *ut = urec + (size_t)(t - s0) * rstride;
                if (th && c->tblock >= 2 && t - 1 >= s0) {
                    e = launch_adjoint_step2_thermal(D.dom, lam[la], lam[la ^ 1], lamg[la], lamg[la ^ 1], ut,
                                                     ut - rstride, gphi, gk, acc_step2, st);
                    t -= 2;
                } else if (th) {
                    e = launch_adjoint_step_thermal(D.dom, lam[la], lam[la ^ 1], lamg[la], lamg[la ^ 1], ut, gphi, gk,
                                                    acc_step, st);
                    t -= 1;
                } else if (c->tblock >= 3 && t - 2 >= s0) {
                    e = launch_adjoint_step3(D.dom, lam[la], lam[la ^ 1], ut, ut - rstride, ut - 2 * rstride, gphi,
                                             gk, acc_step2, st);
                    t -= 3;
                } else if (c->tblock >= 2 && t - 1 >= s0) {
                    e = launch_adjoint_step2(D.dom, lam[la], lam[la ^ 1], ut, ut - rstride, gphi, gk, acc_step2, st);
                    t -= 2;
                } else {
                    e = launch_adjoint_step(D.dom, lam[la], lam[la ^ 1], ut, gphi, gk, acc_step, st);
                    t -= 1;
                }
                if (e != hipSuccess) return device_fail(c, e, "adjoint step");
                la ^= 1;
            }
        }
    }
    if (dL_dphi) e = launch_unpitch(gphi, L.pitch, dL_dphi, d.nx, d.ny, st);
    if (e == hipSuccess && dL_dkappa) e = launch_unpitch(gk, L.pitch, dL_dkappa, d.nx, d.ny, st);
    if (e != hipSuccess) return device_fail(c, e, "gradient copy");
    if (theta) {
        double *res = acc + 4 * (int64_t)L.theta_slots;
        e = launch_theta_final(acc, (int64_t)L.theta_slots, res, st);
        if (e == hipSuccess) e = hipMemcpyAsync(theta, res, sizeof(double) * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(c, e, "parameter gradients");
    }
    return LBM_OK;
}

}  // namespace

extern "C" int lbm_tangent(lbm_ctx *c, const float *dphi, const double *dtheta, float *du) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(LBM_ENOTSUP, "the tangent runs on single-domain contexts");
    Domain &D = c->dom[0];
    const lbm_desc &d = D.desc;
    if (!du) return fail(LBM_EINVAL, "du is required");
    if (d.ckpt_every <= 0) return fail(LBM_ESTATE, "context was created without recording (ckpt_every = 0)");
    if (d.thermal.enabled) return fail(LBM_ENOTSUP, "tangent of the thermal coupling is not implemented");
    if (on_node_walls(d)) return fail(LBM_ENOTSUP, "tangent of on-node (extrapolated) walls is not implemented");
    if (d.storage != LBM_FP32_DEV) return fail(LBM_ENOTSUP, "the tangent needs FP32 storage");
    if (dphi && d.medium == LBM_MEDIUM_UNIFORM) return fail(LBM_ENOTSUP, "a porosity direction needs a porosity plane");
    if (!c->rec_valid) return fail(LBM_ESTATE, "no recorded trajectory leads to the current state");
    const int64_t T = c->t;
    const Layout &L = D.L;
    hipStream_t st = c->stream;
    float *tan[2] = {(float *)(D.base + L.off_lam[0]), (float *)(D.base + L.off_lam[1])};
    float *dphi_p = nullptr;
    hipError_t e = hipSuccess;
    if (dphi) {
        dphi_p = (float *)(D.base + L.off_gphi);
        e = launch_fill_zero(dphi_p, align_up(L.p_bytes, 16), st);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(dphi_p, (size_t)L.pitch * 4, dphi, (size_t)d.nx * 4, (size_t)d.nx * 4,
                                 (size_t)d.ny, hipMemcpyDeviceToDevice, st);
    }
    // f(0) from the first checkpoint; the tangent of f(0) is zero
    if (e == hipSuccess) e = hipMemcpyAsync(D.base + L.off_rf[0], D.base + L.off_ck, L.f_bytes, hipMemcpyDeviceToDevice, st);   // slot 0
    if (e == hipSuccess) e = launch_fill_zero(tan[0], (size_t)L.p_bytes * 8, st);
    if (e != hipSuccess) return device_fail(c, e, "tangent set-up");
    const float dnu = dtheta ? (float)dtheta[0] : 0.0f, dax = dtheta ? (float)dtheta[1] : 0.0f;
    const float day = dtheta ? (float)dtheta[2] : 0.0f, dU = dtheta ? (float)dtheta[3] : 0.0f;
    int p = 0;
    for (int64_t t = 0; t <= T; ++t) {
        Dom ds = D.dom, dtn = D.dom;
        ds.fin = D.base + L.off_rf[p];
        ds.fout = D.base + L.off_rf[p ^ 1];
        dtn.fin = tan[p];
        dtn.fout = tan[p ^ 1];
        dtn.lid6 = dU / 6.0f;
        const Source src = t == 0 ? SRC_DIRECT : SRC_GATHER;
        if (t == T) e = launch_tangent_u(ds, dtn, src, dphi_p, dnu, dax, day, du, st);
        else e = launch_tangent_step(ds, dtn, src, dphi_p, dnu, dax, day, st);
        if (e != hipSuccess) return device_fail(c, e, "tangent step");
        p ^= 1;
    }
    return LBM_OK;
}

extern "C" int lbm_backward(lbm_ctx *c, const float *dL_du, float *dL_dphi, float *dL_dkappa) {
    if (c && !c->batch && !dL_dphi) return fail(LBM_EINVAL, "dL_du and dL_dphi are required");
    return backward_impl(c, dL_du, dL_dphi, dL_dkappa, nullptr);
}

extern "C" int lbm_backward_params(lbm_ctx *c, const float *dL_du, float *dL_dphi, float *dL_dkappa,
                                   double *dL_dtheta) {
    if (!dL_dtheta) return fail(LBM_EINVAL, "dL_dtheta is required");
    return backward_impl(c, dL_du, dL_dphi, dL_dkappa, dL_dtheta);
}
