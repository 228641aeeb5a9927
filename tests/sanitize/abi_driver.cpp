// Exercises the host side of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU: descriptor
// validation, workspace sizing (single, recorded, batched), the refusal paths
// of lbm_create and lbm_create_batch (bad arguments; device failures on a
// host without a GPU, which must free everything they allocated), calls on
// NULL contexts, status strings and the per-thread error message. Built and
// run by tests/test_sanitize_cpu.py; exits 0 when every call returns the
// status the header promises.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lbm.h"

static int failures = 0;

static void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, lbm_last_error());
        ++failures;
    }
}

static lbm_desc valid_desc() {
    lbm_desc d;
    lbm_desc_defaults(&d);
    d.nx = 130; d.ny = 70; d.nu = 0.1;
    d.bc_x = LBM_PERIODIC; d.bc_y = LBM_WALLS;
    d.phi0 = 0.5; d.kappa0 = 0.01;
    return d;
}

int main() {
    size_t bytes = 0;
    lbm_desc d = valid_desc();
    expect(lbm_workspace_size(&d, 0, &bytes) == LBM_OK && bytes > 0, "valid workspace size");
    const size_t plain = bytes;
    d.ckpt_every = 50;
    expect(lbm_workspace_size(&d, 1000, &bytes) == LBM_OK && bytes > plain, "recorded workspace size");
    expect(lbm_workspace_size(&d, -1, &bytes) == LBM_EINVAL, "negative recording capacity");
    d.thermal.enabled = 1; d.thermal.tau_T = 0.8; d.thermal.Th = 1.0;
    expect(lbm_workspace_size(&d, 1000, &bytes) == LBM_OK, "thermal recorded workspace size");
    d.storage = LBM_FP16_DEV;
    d.ckpt_every = 0;
    expect(lbm_workspace_size(&d, 0, &bytes) == LBM_OK, "FP16 thermal workspace size");

    // every invalid field is refused
    struct Bad { const char *what; void (*mutate)(lbm_desc &); int code; };
    const Bad bad[] = {
        {"nx = 0", [](lbm_desc &x) { x.nx = 0; }, LBM_EINVAL},
        {"ny < 0", [](lbm_desc &x) { x.ny = -4; }, LBM_EINVAL},
        {"2^31 nodes exceeded", [](lbm_desc &x) { x.nx = 65536; x.ny = 65536; }, LBM_EINVAL},
        {"unknown bc", [](lbm_desc &x) { x.bc_x = 7; }, LBM_EINVAL},
        {"walled axis with one node", [](lbm_desc &x) { x.bc_y = LBM_WALLS; x.ny = 1; }, LBM_EINVAL},
        {"on-node axis with two nodes", [](lbm_desc &x) { x.bc_x = LBM_WALLS_NEE; x.bc_y = LBM_PERIODIC; x.nx = 2; }, LBM_EINVAL},
        {"mixed wall kinds", [](lbm_desc &x) { x.bc_x = LBM_WALLS_NEE; }, LBM_ENOTSUP},
        {"lid on periodic y", [](lbm_desc &x) { x.bc_y = LBM_PERIODIC; x.lid_ux = 0.1; }, LBM_EINVAL},
        {"nan lid", [](lbm_desc &x) { x.lid_ux = NAN; }, LBM_EINVAL},
        {"nu = 0", [](lbm_desc &x) { x.nu = 0.0; }, LBM_EINVAL},
        {"infinite nu", [](lbm_desc &x) { x.nu = INFINITY; }, LBM_EINVAL},
        {"J < 0", [](lbm_desc &x) { x.J = -1.0; }, LBM_EINVAL},
        {"s_e = 2", [](lbm_desc &x) { x.s_e = 2.0; }, LBM_EINVAL},
        {"s_q = 0", [](lbm_desc &x) { x.s_q = 0.0; }, LBM_EINVAL},
        {"unknown medium", [](lbm_desc &x) { x.medium = 9; }, LBM_EINVAL},
        {"phi0 = 0", [](lbm_desc &x) { x.phi0 = 0.0; }, LBM_EINVAL},
        {"phi0 > 1", [](lbm_desc &x) { x.phi0 = 1.5; }, LBM_EINVAL},
        {"kappa0 < 0", [](lbm_desc &x) { x.kappa0 = -1.0; }, LBM_EINVAL},
        {"Ergun without dp", [](lbm_desc &x) { x.medium = LBM_MEDIUM_PHI_ERGUN; x.dp = 0.0; }, LBM_EINVAL},
        {"nan F_eps", [](lbm_desc &x) { x.F_eps = NAN; }, LBM_EINVAL},
        {"nan force", [](lbm_desc &x) { x.ax = NAN; }, LBM_EINVAL},
        {"unknown storage", [](lbm_desc &x) { x.storage = 3; }, LBM_EINVAL},
        {"ckpt_every < 0", [](lbm_desc &x) { x.ckpt_every = -1; }, LBM_EINVAL},
        {"j_plane = 2", [](lbm_desc &x) { x.j_plane = 2; }, LBM_EINVAL},
        {"tau_T = 1/2", [](lbm_desc &x) { x.thermal.enabled = 1; x.thermal.tau_T = 0.5; }, LBM_EINVAL},
        {"sigma = 0", [](lbm_desc &x) { x.thermal.enabled = 1; x.thermal.tau_T = 0.8; x.thermal.sigma = 0.0; }, LBM_EINVAL},
        {"nan Th", [](lbm_desc &x) { x.thermal.enabled = 1; x.thermal.tau_T = 0.8; x.thermal.Th = NAN; }, LBM_EINVAL},
    };
    for (const Bad &b : bad) {
        lbm_desc x = valid_desc();
        b.mutate(x);
        expect(lbm_workspace_size(&x, 0, &bytes) == b.code, b.what);
        expect(std::strlen(lbm_last_error()) > 0, "message for a refused descriptor");
    }
    expect(lbm_workspace_size(nullptr, 0, &bytes) == LBM_EINVAL, "NULL descriptor");
    expect(lbm_workspace_size(&d, 0, nullptr) == LBM_EINVAL, "NULL size output");

    // lbm_create refusals before any device work
    d = valid_desc();
    lbm_workspace_size(&d, 0, &bytes);
    lbm_ctx *ctx = nullptr;
    std::vector<unsigned char> host(bytes + 512);
    void *aligned = (void *)(((uintptr_t)host.data() + 255) & ~(uintptr_t)255);
    expect(lbm_create(&d, nullptr, nullptr, nullptr, bytes, nullptr, &ctx) == LBM_EINVAL, "NULL workspace");
    expect(lbm_create(&d, nullptr, nullptr, (char *)aligned + 4, bytes, nullptr, &ctx) == LBM_EINVAL,
           "misaligned workspace");
    expect(lbm_create(&d, nullptr, nullptr, aligned, bytes - 1, nullptr, &ctx) == LBM_EINVAL, "small workspace");
    expect(lbm_create(&d, nullptr, nullptr, aligned, bytes, nullptr, nullptr) == LBM_EINVAL, "NULL out");
    lbm_desc e = d;
    e.medium = LBM_MEDIUM_PHI_ERGUN; e.dp = 1.0;
    expect(lbm_create(&e, nullptr, nullptr, aligned, bytes, nullptr, &ctx) == LBM_EINVAL, "missing phi plane");
    // without a GPU the first device call fails: EDEVICE, nothing left allocated
    const int rc = lbm_create(&d, nullptr, nullptr, aligned, bytes, nullptr, &ctx);
    expect(rc == LBM_EDEVICE || rc == LBM_OK, "create on a host without a GPU");
    if (rc == LBM_OK) lbm_destroy(ctx);

    // batches
    std::vector<lbm_desc> ds(3, valid_desc());
    ds[1].nx = 33; ds[2].ny = 17; ds[2].bc_x = LBM_WALLS; ds[2].lid_ux = 0.05;
    expect(lbm_batch_workspace_size(3, ds.data(), &bytes) == LBM_OK && bytes > 0, "batch workspace size");
    expect(lbm_batch_workspace_size(0, ds.data(), &bytes) == LBM_EINVAL, "empty batch");
    ds[1].storage = LBM_FP16_DEV;
    expect(lbm_batch_workspace_size(3, ds.data(), &bytes) == LBM_EINVAL, "mixed storage");
    ds[1].storage = LBM_FP32_DEV;
    ds[2].ckpt_every = 10;
    expect(lbm_batch_workspace_size(3, ds.data(), &bytes) == LBM_ENOTSUP, "recording batch");
    ds[2].ckpt_every = 0;
    lbm_batch_workspace_size(3, ds.data(), &bytes);
    std::vector<unsigned char> bhost(bytes + 512);
    void *baligned = (void *)(((uintptr_t)bhost.data() + 255) & ~(uintptr_t)255);
    const int brc = lbm_create_batch(3, ds.data(), nullptr, nullptr, baligned, bytes, nullptr, nullptr, &ctx);
    expect(brc == LBM_EDEVICE || brc == LBM_OK, "batch create on a host without a GPU");
    if (brc == LBM_OK) lbm_destroy(ctx);

    // NULL contexts
    int64_t t;
    double m, r;
    size_t sb;
    int32_t a1, a2, a3, a4;
    expect(lbm_step(nullptr, 1) == LBM_EINVAL, "step NULL");
    expect(lbm_time(nullptr, &t) == LBM_EINVAL, "time NULL");
    expect(lbm_macroscopic(nullptr, 0, nullptr, nullptr, nullptr) == LBM_EINVAL, "macroscopic NULL");
    expect(lbm_reduce(nullptr, 0, &m, &r) == LBM_EINVAL, "reduce NULL");
    expect(lbm_reduce_static(nullptr, 0, &m, &r) == LBM_EINVAL, "reduce_static NULL");
    expect(lbm_state_bytes(nullptr, &sb) == LBM_EINVAL, "state_bytes NULL");
    expect(lbm_save(nullptr, host.data(), 64) == LBM_EINVAL, "save NULL");
    expect(lbm_load(nullptr, host.data(), 64) == LBM_EINVAL, "load NULL");
    expect(lbm_schedule(nullptr, &a1, &a2, &a3, &a4) == LBM_EINVAL, "schedule NULL");
    expect(lbm_time_blocking(nullptr, &a1, &a2, &a3, &a4) == LBM_EINVAL, "time_blocking NULL");
    expect(lbm_set_time_blocking(nullptr, 2) == LBM_EINVAL, "set_time_blocking NULL");
    expect(lbm_set_graph_steps(nullptr, 8) == LBM_EINVAL, "set_graph_steps NULL");
    expect(lbm_backward(nullptr, nullptr, nullptr, nullptr) == LBM_EINVAL, "backward NULL");
    expect(lbm_tangent(nullptr, nullptr, nullptr, nullptr) == LBM_EINVAL, "tangent NULL");
    expect(lbm_destroy(nullptr) == LBM_OK, "destroy NULL");
    for (int s = 1; s >= -6; --s) expect(lbm_strerror(s) && std::strlen(lbm_strerror(s)) > 0, "strerror");
    expect(lbm_desc_defaults(nullptr) == LBM_EINVAL, "defaults NULL");
    std::printf("abi sanitizer driver: %d failures\n", failures);
    return failures != 0;
}
