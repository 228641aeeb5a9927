// Fault injection through the null device (tests/sanitize/null_device.cpp):
// the library's host code, with its kernel launch stubs, runs on a fake HIP
// runtime in host memory, under AddressSanitizer and UndefinedBehaviorSanitizer.
// Checked against the contract of include/lbm.h:
//   * a NaN injected into a population makes lbm_reduce return LBM_EUNSTABLE
//     (single domain and one domain of a batch), and a restart from an
//     lbm_save snapshot clears it;
//   * calls out of order: the adjoint and the tangent without recording,
//     after lbm_load, and past the recorded capacity; a per-node viscosity
//     ratio without its plane; save/load on a batch; a batch's state at
//     t > 0; a snapshot of another configuration;
//   * an injected device error poisons the context (LBM_EDEVICE from then on);
//   * a failed call leaves the time unchanged;
//   * a second lbm_destroy, calls on a destroyed handle and on a handle that
//     was never created are refused without touching memory;
//   * the step is launched (directly and from a replayed graph);
//   * the pass shape switches at 2^23 nodes (isothermal only): four cycles on
//     64 x 26 tiles by default, 64 x 28 tiles when switched to three.
// Built and run by tests/test_sanitize_cpu.py; exits 0 when every call
// returns what the header promises.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lbm.h"

extern "C" {
long null_device_launches(const char *sub);
void null_device_fail_after(int n);
int null_device_poke_state(int i, int x, int y, float v);
}

static int failures = 0;

static void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, lbm_last_error());
        ++failures;
    }
}

// workspace in host memory, which is device memory on the null device
struct Workspace {
    void *p = nullptr;
    size_t bytes = 0;
    explicit Workspace(size_t b) : bytes(b) {
        p = std::aligned_alloc(256, (b + 255) / 256 * 256);
        std::memset(p, 0, b);
    }
    ~Workspace() { std::free(p); }
};

static lbm_desc channel(int nx, int ny) {
    lbm_desc d;
    lbm_desc_defaults(&d);
    d.nx = nx; d.ny = ny; d.nu = 0.1;
    d.bc_x = LBM_PERIODIC; d.bc_y = LBM_WALLS;
    d.phi0 = 0.5; d.kappa0 = 0.01; d.ax = 1e-6;
    return d;
}

static int64_t time_of(const lbm_ctx *c) {
    int64_t t = -1;
    lbm_time(c, &t);
    return t;
}

static void single_domain() {
    lbm_desc d = channel(130, 70);
    size_t bytes = 0;
    expect(lbm_workspace_size(&d, 0, &bytes) == LBM_OK, "workspace size");
    Workspace ws(bytes);
    lbm_ctx *c = nullptr;
    expect(lbm_create(&d, nullptr, nullptr, ws.p, ws.bytes, nullptr, &c) == LBM_OK, "create");
    if (!c) return;
    double m = 0, r = 0;
    expect(lbm_reduce(c, 0, &m, &r) == LBM_OK && std::isfinite(m), "reduce at t = 0");
    const long steps0 = null_device_launches("k_step");
    expect(lbm_step(c, 7) == LBM_OK && time_of(c) == 7, "step 7");
    expect(null_device_launches("k_step") > steps0, "the step kernels were launched");
    expect(lbm_reduce(c, 0, &m, &r) == LBM_OK && std::isfinite(m), "reduce at t = 7");
    size_t sb = 0;
    expect(lbm_state_bytes(c, &sb) == LBM_OK && sb > 64, "state bytes");
    std::vector<unsigned char> snap(sb);
    expect(lbm_save(c, snap.data(), sb) == LBM_OK, "save");

    // a NaN in one population: unstable, no side effect, cleared by a restart
    expect(null_device_poke_state(3, 5, 5, NAN) == 0, "poke a NaN into f_3 at (5, 5)");
    expect(lbm_reduce(c, 0, &m, &r) == LBM_EUNSTABLE, "NaN population gives EUNSTABLE");
    expect(!std::isfinite(m), "mass reported non-finite");
    expect(lbm_reduce_static(c, 0, &m, &r) == LBM_EUNSTABLE, "NaN population gives EUNSTABLE (static scratch)");
    expect(time_of(c) == 7, "time unchanged by the failed reduction");
    expect(lbm_load(c, snap.data(), sb) == LBM_OK, "restart from the snapshot");
    expect(lbm_reduce(c, 0, &m, &r) == LBM_OK && std::isfinite(m), "reduce after the restart");
    expect(lbm_reduce_static(c, 0, &m, &r) == LBM_OK, "reduce through the static scratch");

    // calls out of order or on missing state
    std::vector<float> du(2 * (size_t)d.nx * d.ny, 0.0f), g(3 * (size_t)d.nx * d.ny, 0.0f);
    expect(lbm_backward(c, du.data(), g.data(), nullptr) == LBM_ESTATE, "backward without recording");
    const double dth[4] = {1e-3, 0, 0, 0};
    expect(lbm_tangent(c, nullptr, dth, du.data()) == LBM_ESTATE, "tangent without recording");
    expect(lbm_set_viscosity_ratio(c, 0, g.data()) == LBM_ESTATE, "viscosity ratio without its plane");
    expect(lbm_step(c, -1) == LBM_EINVAL, "negative step count");
    expect(lbm_reduce(c, 1, &m, &r) == LBM_EINVAL, "domain out of range");
    expect(lbm_load(c, snap.data(), sb - 1) == LBM_EINVAL, "snapshot of the wrong size");
    std::vector<unsigned char> bad = snap;
    bad[0] ^= 0xff;
    expect(lbm_load(c, bad.data(), sb) == LBM_EINVAL, "snapshot with a bad magic number");
    expect(time_of(c) == 7, "time unchanged by the refused calls");

    // stepping from a replayed graph
    expect(lbm_set_graph_steps(c, 6) == LBM_OK, "graph steps");
    const long before = null_device_launches("k_step");
    expect(lbm_step(c, 20) == LBM_OK && time_of(c) == 27, "step 20 through graphs");
    expect(null_device_launches("k_step") > before, "graph replays launch the step kernels");

    // an injected device error poisons the context
    null_device_fail_after(0);
    expect(lbm_step(c, 3) == LBM_EDEVICE, "injected launch failure gives EDEVICE");
    null_device_fail_after(-1);
    expect(lbm_step(c, 1) == LBM_EDEVICE, "poisoned context refuses a step");
    expect(lbm_reduce(c, 0, &m, &r) == LBM_EDEVICE, "poisoned context refuses a reduction");
    expect(lbm_save(c, snap.data(), sb) == LBM_EDEVICE, "poisoned context refuses a save");

    // destroy twice, then use the stale handle
    expect(lbm_destroy(c) == LBM_OK, "destroy");
    expect(lbm_destroy(c) == LBM_EINVAL, "second destroy is refused");
    expect(lbm_step(c, 1) == LBM_EINVAL, "step on a destroyed context");
    expect(lbm_time(c, nullptr) == LBM_EINVAL, "time on a destroyed context");
    int32_t a1;
    expect(lbm_schedule(c, &a1, nullptr, nullptr, nullptr) == LBM_EINVAL, "schedule on a destroyed context");
    lbm_ctx *never = reinterpret_cast<lbm_ctx *>(static_cast<uintptr_t>(0x1000));
    expect(lbm_destroy(never) == LBM_EINVAL, "destroy of a handle never created");
    expect(lbm_reduce(never, 0, &m, &r) == LBM_EINVAL, "reduce on a handle never created");
}

static void recording() {
    lbm_desc d = channel(96, 40);
    d.medium = LBM_MEDIUM_PHI_KAPPA;
    d.ckpt_every = 10;
    size_t bytes = 0;
    expect(lbm_workspace_size(&d, 40, &bytes) == LBM_OK, "recorded workspace size");
    Workspace ws(bytes);
    std::vector<float> phi((size_t)d.nx * d.ny, 0.6f), kappa((size_t)d.nx * d.ny, 0.01f);
    lbm_ctx *c = nullptr;
    expect(lbm_create(&d, phi.data(), kappa.data(), ws.p, ws.bytes, nullptr, &c) == LBM_OK, "create recording");
    if (!c) return;
    std::vector<float> du(2 * (size_t)d.nx * d.ny, 0.0f), dphi((size_t)d.nx * d.ny, 0.0f);
    expect(lbm_step(c, 25) == LBM_OK, "recorded step 25");
    const long adj0 = null_device_launches("k_adjoint");
    expect(lbm_backward(c, du.data(), dphi.data(), nullptr) == LBM_OK, "backward at t = 25");
    expect(null_device_launches("k_adjoint") > adj0, "the adjoint kernels were launched");
    const double dth[4] = {1e-3, 0, 0, 0};
    expect(lbm_tangent(c, nullptr, dth, du.data()) == LBM_OK, "tangent at t = 25");
    expect(lbm_step(c, 30) == LBM_OK && time_of(c) == 55, "step past the recorded capacity");
    expect(lbm_backward(c, du.data(), dphi.data(), nullptr) == LBM_ESTATE, "backward past the capacity");
    size_t sb = 0;
    lbm_state_bytes(c, &sb);
    std::vector<unsigned char> snap(sb);
    expect(lbm_save(c, snap.data(), sb) == LBM_OK, "save recording context");
    expect(lbm_load(c, snap.data(), sb) == LBM_OK, "load recording context");
    expect(lbm_backward(c, du.data(), dphi.data(), nullptr) == LBM_ESTATE, "backward after a load");
    expect(lbm_tangent(c, nullptr, dth, du.data()) == LBM_ESTATE, "tangent after a load");
    expect(lbm_destroy(c) == LBM_OK, "destroy recording context");

    // in mode 4 the recorded forward and the recomputation inside lbm_backward
    // take four-cycle passes (never over a checkpoint time or a segment's end)
    Workspace ws4(bytes);
    lbm_ctx *c4 = nullptr;
    expect(lbm_create(&d, phi.data(), kappa.data(), ws4.p, ws4.bytes, nullptr, &c4) == LBM_OK, "create (mode 4)");
    if (!c4) return;
    expect(lbm_set_time_blocking(c4, 4) == LBM_OK, "mode 4 on a recording context");
    const long f4 = null_device_launches("k_step4");
    expect(lbm_step(c4, 25) == LBM_OK && time_of(c4) == 25, "recorded steps in mode 4");
    expect(null_device_launches("k_step4") == f4 + 5, "four-cycle passes 1-5, 5-9, 10-14, 14-18, 20-24 while recording");
    const long b4 = null_device_launches("k_step4_rec");
    expect(lbm_backward(c4, du.data(), dphi.data(), nullptr) == LBM_OK, "backward in mode 4");
    expect(null_device_launches("k_step4_rec") == b4 + 5,
           "recording passes 1-5, 5-9, 10-14, 14-18, 20-24 in the recomputation");
    expect(lbm_destroy(c4) == LBM_OK, "destroy (mode 4)");
}

static void thermal_snapshot_into_isothermal() {
    lbm_desc a = channel(64, 48);
    a.bc_x = LBM_WALLS;
    lbm_desc b = a;
    b.thermal.enabled = 1; b.thermal.tau_T = 0.8; b.thermal.Th = 2.0; b.thermal.Tc = 1.0;
    b.thermal.T0 = 1.5; b.thermal.g_beta = 1e-5;
    size_t ba = 0, bb = 0;
    lbm_workspace_size(&a, 0, &ba);
    lbm_workspace_size(&b, 0, &bb);
    Workspace wa(ba), wb(bb);
    lbm_ctx *ca = nullptr, *cb = nullptr;
    expect(lbm_create(&a, nullptr, nullptr, wa.p, wa.bytes, nullptr, &ca) == LBM_OK, "create isothermal");
    expect(lbm_create(&b, nullptr, nullptr, wb.p, wb.bytes, nullptr, &cb) == LBM_OK, "create thermal");
    if (!ca || !cb) return;
    expect(lbm_step(cb, 5) == LBM_OK, "thermal step");
    double m, r;
    expect(lbm_reduce(cb, 0, &m, &r) == LBM_OK, "thermal reduce");
    size_t sb = 0;
    lbm_state_bytes(cb, &sb);
    std::vector<unsigned char> snap(sb);
    expect(lbm_save(cb, snap.data(), sb) == LBM_OK, "thermal save");
    expect(lbm_load(ca, snap.data(), sb) == LBM_EINVAL, "thermal snapshot into an isothermal context");
    expect(time_of(ca) == 0, "isothermal context unchanged");
    lbm_destroy(ca);
    lbm_destroy(cb);
}

static void batch() {
    std::vector<lbm_desc> ds(3, channel(130, 70));
    ds[1].nx = 33; ds[1].ny = 65;
    ds[2].nx = 70; ds[2].ny = 17; ds[2].bc_x = LBM_WALLS; ds[2].lid_ux = 0.05;
    size_t bytes = 0;
    expect(lbm_batch_workspace_size(3, ds.data(), &bytes) == LBM_OK, "batch workspace size");
    Workspace ws(bytes);
    lbm_ctx *c = nullptr;
    expect(lbm_create_batch(3, ds.data(), nullptr, nullptr, ws.p, ws.bytes, nullptr, nullptr, &c) == LBM_OK,
           "create batch");
    if (!c) return;
    std::vector<float> df(8 * 130 * 70, 0.0f);
    expect(lbm_step(c, 10) == LBM_OK && time_of(c) == 10, "batch step 10");
    double m, r;
    for (int k = 0; k < 3; ++k) expect(lbm_reduce(c, k, &m, &r) == LBM_OK, "batch reduce");
    expect(null_device_poke_state(0, ds[2].nx - 1, ds[2].ny - 1, INFINITY) == 0, "poke an infinity into domain 2");
    expect(lbm_reduce(c, 2, &m, &r) == LBM_EUNSTABLE, "infinite population gives EUNSTABLE in a batch");
    expect(lbm_set_populations(c, 0, df.data(), nullptr) == LBM_ESTATE, "batch state at t > 0");
    size_t sb = 0;
    expect(lbm_state_bytes(c, &sb) == LBM_ENOTSUP, "state bytes of a batch");
    expect(lbm_save(c, df.data(), 64) == LBM_ENOTSUP, "save of a batch");
    expect(lbm_set_schedule(c, 128, 1, 2, 1) == LBM_ENOTSUP, "schedule of a batch");
    expect(lbm_backward(c, df.data(), nullptr, nullptr) == LBM_ENOTSUP, "adjoint of a batch");
    expect(lbm_destroy(c) == LBM_OK, "destroy batch");
    expect(lbm_destroy(c) == LBM_EINVAL, "second destroy of a batch");
}

// The multi-cycle pass shape: from 2^23 nodes isothermal single domains take four
// cycles on 64 x 26 tiles of 768 threads, or, switched to three, 64 x 28 tiles of
// 768 threads; below 2^23 and for thermal domains three cycles on 64 x 16 tiles of
// 512 threads.
static void tile_shapes() {
    struct Shape { int nx, ny, thermal, set3, cycles, threads, rows, grid; };
    const Shape shapes[] = {
        {2896, 2896, 0, 0, 3, 512, 16, 46 * 181},    // 8,386,816 nodes: below 2^23
        {2896, 2897, 0, 0, 4, 768, 26, 46 * 112},    // 8,389,712 nodes: four cycles
        {2896, 2897, 0, 1, 3, 768, 28, 46 * 104},    // switched to three: tall tiles
        {2896, 2897, 1, 0, 3, 512, 16, 46 * 182},    // thermal: 64 x 16
    };
    for (const Shape &sh : shapes) {
        lbm_desc d = channel(sh.nx, sh.ny);
        d.phi0 = 1.0; d.kappa0 = 0.0;
        if (sh.thermal) {
            d.bc_x = LBM_WALLS;
            d.thermal.enabled = 1; d.thermal.tau_T = 0.8; d.thermal.Th = 2.0; d.thermal.Tc = 1.0;
            d.thermal.T0 = 1.5; d.thermal.g_beta = 1e-6;
        }
        size_t bytes = 0;
        expect(lbm_workspace_size(&d, 0, &bytes) == LBM_OK, "workspace size (tile shapes)");
        Workspace ws(bytes);
        lbm_ctx *c = nullptr;
        expect(lbm_create(&d, nullptr, nullptr, ws.p, ws.bytes, nullptr, &c) == LBM_OK, "create (tile shapes)");
        if (!c) continue;
        if (sh.set3) expect(lbm_set_time_blocking(c, 3) == LBM_OK, "switch to three cycles");
        int32_t cyc = 0, thr = 0, rows = 0, grid = 0;
        expect(lbm_time_blocking(c, &cyc, &thr, &rows, &grid) == LBM_OK, "time blocking query");
        expect(cyc == sh.cycles && thr == sh.threads && rows == sh.rows && grid == sh.grid,
               "multi-cycle pass shape at the 2^23-node switch");
        const char *kname = sh.cycles == 4 ? "k_step4" : "k_step3";
        const long before = null_device_launches(kname);
        expect(lbm_step(c, 9) == LBM_OK, "step (tile shapes)");
        expect(null_device_launches(kname) > before, "multi-cycle kernel launched");
        lbm_destroy(c);
    }
    // a small domain switched to three cycles keeps 64 x 16 tiles
    lbm_desc d = channel(200, 130);
    size_t bytes = 0;
    lbm_workspace_size(&d, 0, &bytes);
    Workspace ws(bytes);
    lbm_ctx *c = nullptr;
    expect(lbm_create(&d, nullptr, nullptr, ws.p, ws.bytes, nullptr, &c) == LBM_OK, "create (small)");
    if (!c) return;
    int32_t cyc = 0, thr = 0, rows = 0, grid = 0;
    expect(lbm_set_time_blocking(c, 3) == LBM_OK, "three cycles on a small domain");
    expect(lbm_time_blocking(c, &cyc, &thr, &rows, &grid) == LBM_OK && cyc == 3 && thr == 512 && rows == 16 &&
               grid == 4 * 9, "small domain keeps 64 x 16 tiles");
    // and switched to four cycles takes 64 x 26 tiles
    expect(lbm_set_time_blocking(c, 4) == LBM_OK, "four cycles on a small domain");
    expect(lbm_time_blocking(c, &cyc, &thr, &rows, &grid) == LBM_OK && cyc == 4 && thr == 768 && rows == 26 &&
               grid == 4 * 5, "small domain in mode 4: 64 x 26 tiles");
    const long before = null_device_launches("k_step4");
    expect(lbm_step(c, 9) == LBM_OK, "step in mode 4");
    expect(null_device_launches("k_step4") == before + 2, "two four-cycle passes after the collide-only cycle");
    lbm_destroy(c);
}

int main() {
    tile_shapes();
    single_domain();
    recording();
    thermal_snapshot_into_isothermal();
    batch();
    std::printf("null-device driver: %d failures\n", failures);
    return failures != 0;
}
