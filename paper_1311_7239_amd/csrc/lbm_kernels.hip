// HIP kernels for gfx950 of the fused D2Q8 porous MRT-LB step (Liu & He,
// arXiv:1311.7239, Eqs. 3, 4, 8-20) and the D2Q5 thermal model (App. B).
//
// One kernel pass per time step does, for every node: gather the eight
// post-collision deviations of the previous step from the neighbours (pull
// streaming, Eq. 15, with periodic wrap or halfway bounce-back), collide in
// moment space (Eq. 14) with the porous equilibrium and drag forcing, and
// store the eight new post-collision deviations into the other buffer.
// Each stored value is read by exactly one neighbour, so the pass moves the
// minimum 2 x 8 populations per node through HBM; there is no reuse for LDS
// to capture and the 8x8 transform is a handful of adds, so the kernel is a
// coalesced streaming kernel, not an MFMA one.
#include <hip/hip_runtime.h>

#include "lbm_launch.h"

namespace mrt {

constexpr int BLOCK = 256;

// ------------------------------------------------------------------ step

// Thermal-coupled acceleration phi*a of one node (Sec. 3.4 buoyancy on top
// of the uniform a), and the rest of the per-node update shared by both
// paths below: collide, then return u.
template <bool THERMAL>
__device__ __forceinline__ void node_update(const Dom &d, const Cell &c, float f[8], float g[5],
                                            float &ux, float &uy, float &n7, float &n8, float &dT) {
    // half of a (the step works on half forces; every product is halved exactly)
    float ayh = d.ayh;
    dT = 0.0f;
    if (THERMAL) {
        dT = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
        ayh = d.ayh + d.gbetah * dT;
    }
    collide_h(f, d, c, c.phi * d.axh, c.phi * ayh, ux, uy, n7, n8);
    if (THERMAL) thermal_collide(g, d, ux, uy);
}

// One 256-thread tile: TWT threads along x, each handling NX consecutive
// nodes in each of ROWS rows (rows TH apart). Tiles that touch no boundary
// take vector loads of whole rows of NX values per plane; edge tiles gather
// node by node with wrap/bounce-back. Both paths run the same per-node
// arithmetic, so every schedule produces the same bits.
template <typename S, bool THERMAL, int SRC, bool REC, int TWT, int NX, int ROWS>
__device__ __forceinline__ void step_tile(const Dom &d, int tx, int ty) {
    constexpr int TH = BLOCK / TWT;
    constexpr int TW = TWT * NX;
    const int lx = threadIdx.x % TWT, ly = threadIdx.x / TWT;
    const int x0 = tx * TW, y0 = ty * TH * ROWS;
    const int xb = x0 + lx * NX;
    const S *__restrict__ fin = (const S *)d.fin;
    S *__restrict__ fout = (S *)d.fout;
    const bool interior = (SRC == SRC_GATHER) && x0 >= 1 && x0 + TW <= d.nx - 1 && y0 >= 1 &&
                          y0 + TH * ROWS <= d.ny - 1;

    if (interior) {
        float f[ROWS][8][NX];
        float g[THERMAL ? ROWS : 1][5][NX];
        float ph[ROWS][NX] = {}, kp[ROWS][NX] = {};
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int64_t o = (int64_t)(y0 + ly + r * TH) * d.pitch + xb;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                load_row<S, NX>(fin + i * d.plane + o - EY[i] * d.pitch - EX[i], f[r][i]);
            if (THERMAL) {
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    load_row<float, NX>(d.gin + j * d.plane + o - TYv[j] * d.pitch - TXv[j],
                                        g[THERMAL ? r : 0][j]);
            }
            if (d.medium != MED_UNIFORM) load_row<float, NX>(d.phi + o, ph[r]);
            if (d.medium == MED_PHI_KAPPA) load_row<float, NX>(d.kappa + o, kp[r]);
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int64_t o = (int64_t)(y0 + ly + r * TH) * d.pitch + xb;
            float ux[NX], uy[NX], n7[NX], n8[NX], dT[NX];
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                float fn[8], gn[5];
#pragma unroll
                for (int i = 0; i < 8; ++i) fn[i] = f[r][i][k];
                if (THERMAL) {
#pragma unroll
                    for (int j = 0; j < 5; ++j) gn[j] = g[THERMAL ? r : 0][j][k];
                }
                Cell c = cell_from(d, ph[r][k], kp[r][k]);
                cell_viscosity(d, c, o + k);
                node_update<THERMAL>(d, c, fn, gn, ux[k], uy[k], n7[k], n8[k], dT[k]);
#pragma unroll
                for (int i = 0; i < 8; ++i) f[r][i][k] = fn[i];
                if (THERMAL) {
#pragma unroll
                    for (int j = 0; j < 5; ++j) g[THERMAL ? r : 0][j][k] = gn[j];
                }
            }
            if (d.nt_store) {
#pragma unroll
                for (int i = 0; i < 8; ++i) store_row_nt<S, NX>(fout + i * d.plane + o, f[r][i]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) store_row<S, NX>(fout + i * d.plane + o, f[r][i]);
            }
            if (THERMAL) {
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    if (d.nt_store) store_row_nt<float, NX>(d.gout + j * d.plane + o, g[THERMAL ? r : 0][j]);
                    else store_row<float, NX>(d.gout + j * d.plane + o, g[THERMAL ? r : 0][j]);
                }
            }
            if (d.uprev) {
                if (d.nt_store) {
                    store_row_nt<float, NX>(d.uprev + o, ux);
                    store_row_nt<float, NX>(d.uprev + d.plane + o, uy);
                } else {
                    store_row<float, NX>(d.uprev + o, ux);
                    store_row<float, NX>(d.uprev + d.plane + o, uy);
                }
            }
            if (REC) {
                store_row<float, NX>(d.urec + o, ux);
                store_row<float, NX>(d.urec + d.plane + o, uy);
                if (d.rec_stress) {
                    store_row<float, NX>(d.urec + 2 * d.plane + o, n7);
                    store_row<float, NX>(d.urec + 3 * d.plane + o, n8);
                }
                if (THERMAL) store_row<float, NX>(d.urec + 4 * d.plane + o, dT);
            }
        }
        return;
    }

    // edge tiles (and the collide-only first cycle): node by node
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + ly + r * TH;
        if (y >= d.ny) continue;
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const int x = xb + k;
            if (x >= d.nx) continue;
            float fn[8], gn[5];
            if (SRC == SRC_DIRECT) {
                load_own<S>(d, fin, x, y, fn);
                if (THERMAL) load_own_thermal(d, d.gin, x, y, gn);
            } else {
                gather_general<S>(d, fin, x, y, fn);
                if (THERMAL) gather_thermal(d, d.gin, x, y, false, gn);
                nee_fixup<S, THERMAL>(d, fin, x, y, fn, gn);
            }
            const int64_t o = (int64_t)y * d.pitch + x;
            const Cell c = load_cell(d, o);
            float ux, uy, n7, n8, dT;
            node_update<THERMAL>(d, c, fn, gn, ux, uy, n7, n8, dT);
#pragma unroll
            for (int i = 0; i < 8; ++i) Store<S>::st(fout + i * d.plane + o, fn[i]);
            if (THERMAL) {
#pragma unroll
                for (int j = 0; j < 5; ++j) d.gout[j * d.plane + o] = gn[j];
            }
            if (d.uprev) {
                d.uprev[o] = ux;
                d.uprev[d.plane + o] = uy;
            }
            if (REC) {
                d.urec[o] = ux;
                d.urec[d.plane + o] = uy;
                if (d.rec_stress) {
                    d.urec[2 * d.plane + o] = n7;
                    d.urec[3 * d.plane + o] = n8;
                }
                if (THERMAL) d.urec[4 * d.plane + o] = dT;
            }
        }
    }
}

template <typename S, bool THERMAL, int SRC, bool REC, int TWT, int NX, int ROWS>
__global__ __launch_bounds__(BLOCK) void k_step(Dom d, int tiles_x, int swz) {
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    step_tile<S, THERMAL, SRC, REC, TWT, NX, ROWS>(d, b % tiles_x, b / tiles_x);
}

// Persistent batched step: block b walks a contiguous run of the tile table
// (tiles of one domain row stay on one XCD and in order), so the grid size is
// a free tuning parameter independent of the number of tiles.
template <typename S, bool THERMAL, int TWT, int NX, int ROWS>
__global__ __launch_bounds__(BLOCK) void k_step_batch(const Dom *__restrict__ doms,
                                                      const int4 *__restrict__ tiles,
                                                      int ntiles, int parity) {
    const int64_t nb = gridDim.x;
    const int t0 = (int)((int64_t)blockIdx.x * ntiles / nb);
    const int t1 = (int)(((int64_t)blockIdx.x + 1) * ntiles / nb);
    for (int t = t0; t < t1; ++t) {
        const int4 tl = tiles[t];
        const Dom d = doms[2 * tl.x + parity];
        step_tile<S, THERMAL, SRC_GATHER, false, TWT, NX, ROWS>(d, tl.y, tl.z);
    }
}

void tile_counts(const Schedule &s, int nx, int ny, int *tiles_x, int *tiles_y) {
    const int th = BLOCK / s.tile_w;
    const int tw = s.tile_w * s.vec;
    *tiles_x = (nx + tw - 1) / tw;
    *tiles_y = (ny + th * s.rows - 1) / (th * s.rows);
}

// The schedules compiled into the library: (threads along x, nodes per
// thread along x, rows per thread).
#define MRT_SCHEDULES(X) \
    X(256, 1, 1) X(256, 1, 2) X(128, 1, 1) X(128, 1, 2) X(64, 1, 2) X(64, 1, 4) \
    X(128, 2, 1) X(64, 2, 2) X(64, 4, 1) X(32, 4, 2) X(64, 4, 2) X(16, 4, 4)

bool schedule_supported(const Schedule &s) {
#define MRT_SUP(T, V, R) if (s.tile_w == T && s.vec == V && s.rows == R) return true;
    MRT_SCHEDULES(MRT_SUP)
#undef MRT_SUP
    return false;
}

template <typename S, bool THERMAL, int SRC, bool REC>
static hipError_t launch_step_t(const Dom &d, const Schedule &s, hipStream_t st) {
    int tx, ty;
    tile_counts(s, d.nx, d.ny, &tx, &ty);
    const dim3 grid((unsigned)(tx * ty)), block(BLOCK);
#define MRT_LAUNCH(T, V, R)                                                                  \
    if (s.tile_w == T && s.vec == V && s.rows == R) {                                        \
        hipLaunchKernelGGL((k_step<S, THERMAL, SRC, REC, T, V, R>), grid, block, 0, st, d, tx, \
                           s.swizzle);                                                       \
        return hipGetLastError();                                                            \
    }
    MRT_SCHEDULES(MRT_LAUNCH)
#undef MRT_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_step(const Dom &d, int storage, Source src, bool rec, const Schedule &s,
                       hipStream_t st) {
    // the collide-only first cycle always runs with the plain schedule
    static const Schedule flat{256, 1, 1, 0};
    const bool th = d.thermal != 0;
    if (rec && storage != ST_F32) return hipErrorInvalidValue;
    if (src == SRC_DIRECT) {
        if (storage == ST_F32) {
            if (th) return rec ? launch_step_t<float, true, SRC_DIRECT, true>(d, flat, st)
                               : launch_step_t<float, true, SRC_DIRECT, false>(d, flat, st);
            return rec ? launch_step_t<float, false, SRC_DIRECT, true>(d, flat, st)
                       : launch_step_t<float, false, SRC_DIRECT, false>(d, flat, st);
        }
        if (th) return launch_step_t<_Float16, true, SRC_DIRECT, false>(d, flat, st);
        return launch_step_t<_Float16, false, SRC_DIRECT, false>(d, flat, st);
    }
    if (storage == ST_F32) {
        if (th) return rec ? launch_step_t<float, true, SRC_GATHER, true>(d, s, st)
                           : launch_step_t<float, true, SRC_GATHER, false>(d, s, st);
        return rec ? launch_step_t<float, false, SRC_GATHER, true>(d, s, st)
                   : launch_step_t<float, false, SRC_GATHER, false>(d, s, st);
    }
    if (th) return launch_step_t<_Float16, true, SRC_GATHER, false>(d, s, st);
    return launch_step_t<_Float16, false, SRC_GATHER, false>(d, s, st);
}

template <typename S, bool THERMAL, int SRC, bool REC>
static const void *step_fn_t(const Schedule &s) {
#define MRT_FN(T, V, R) \
    if (s.tile_w == T && s.vec == V && s.rows == R) return (const void *)&k_step<S, THERMAL, SRC, REC, T, V, R>;
    MRT_SCHEDULES(MRT_FN)
#undef MRT_FN
    return nullptr;
}

const void *step_kernel_fn(int storage, bool thermal, const Schedule &s) {
    if (storage == ST_F32)
        return thermal ? step_fn_t<float, true, SRC_GATHER, false>(s) : step_fn_t<float, false, SRC_GATHER, false>(s);
    return thermal ? step_fn_t<_Float16, true, SRC_GATHER, false>(s) : step_fn_t<_Float16, false, SRC_GATHER, false>(s);
}

template <typename S, bool THERMAL>
static const void *batch_fn_t(const Schedule &s) {
#define MRT_BFN(T, V, R) \
    if (s.tile_w == T && s.vec == V && s.rows == R) return (const void *)&k_step_batch<S, THERMAL, T, V, R>;
    MRT_SCHEDULES(MRT_BFN)
#undef MRT_BFN
    return nullptr;
}

const void *batch_kernel_fn(int storage, bool thermal, const Schedule &s) {
    if (storage == ST_F32) return thermal ? batch_fn_t<float, true>(s) : batch_fn_t<float, false>(s);
    return thermal ? batch_fn_t<_Float16, true>(s) : batch_fn_t<_Float16, false>(s);
}

template <typename S, bool THERMAL>
static hipError_t launch_batch_t(const Dom *doms, const int4 *tiles, int ntiles, int parity,
                                 const Schedule &s, int grid, hipStream_t st) {
    const dim3 g((unsigned)grid), b(BLOCK);
#define MRT_BLAUNCH(T, V, R)                                                                       \
    if (s.tile_w == T && s.vec == V && s.rows == R) {                                              \
        hipLaunchKernelGGL((k_step_batch<S, THERMAL, T, V, R>), g, b, 0, st, doms, tiles, ntiles, parity); \
        return hipGetLastError();                                                                  \
    }
    MRT_SCHEDULES(MRT_BLAUNCH)
#undef MRT_BLAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_step_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity,
                             int storage, bool thermal, const Schedule &s, int grid, hipStream_t st) {
    if (grid <= 0 || ntiles <= 0) return hipErrorInvalidValue;
    if (storage == ST_F32)
        return thermal ? launch_batch_t<float, true>(doms, tiles, ntiles, parity, s, grid, st)
                       : launch_batch_t<float, false>(doms, tiles, ntiles, parity, s, grid, st);
    return thermal ? launch_batch_t<_Float16, true>(doms, tiles, ntiles, parity, s, grid, st)
                   : launch_batch_t<_Float16, false>(doms, tiles, ntiles, parity, s, grid, st);
}

// Recorded u (and stress moments) of the multi-cycle passes.
// The records go through buffer stores: a recorded step spans at most five
// planes, below 4 GiB whenever multi-cycle passes run. They are read back only
// by the adjoint sweep after the whole segment, so they are streamed past the
// caches (non-temporal), which keeps the recomputation's own state there
// (2048^2 recomputation with the adjoint sweep: 6% less time).
__device__ __forceinline__ void record_node(const Dom &d, BufRes rec, uint32_t o4, float ux, float uy, float n7,
                                            float n8) {
    const uint32_t pb4 = (uint32_t)(d.plane * 4);
    BufIO<float>::st_nt(rec, o4, 0u, ux);
    BufIO<float>::st_nt(rec, o4, pb4, uy);
    if (d.rec_stress) {
        BufIO<float>::st_nt(rec, o4, 2 * pb4, n7);
        BufIO<float>::st_nt(rec, o4, 3 * pb4, n8);
    }
}

// One node's record held back until the next node's loads have been issued
// (with THERMAL also dT, plane 4).
template <bool THERMAL>
struct Pending {
    uint32_t o4 = 0u;
    float ux = 0.0f, uy = 0.0f, n7 = 0.0f, n8 = 0.0f, dT = 0.0f;
    bool on = false;
    __device__ __forceinline__ void hold(uint32_t o, float a, float b, float c, float e, float t) {
        o4 = o; ux = a; uy = b; n7 = c; n8 = e; dT = t; on = true;
    }
    __device__ __forceinline__ void flush(const Dom &d, BufRes rec) {
        if (on) {
            record_node(d, rec, o4, ux, uy, n7, n8);
            if (THERMAL) BufIO<float>::st_nt(rec, o4, (uint32_t)(4 * d.plane * 4), dT);
        }
        on = false;
    }
};

// u of a pass's last collision (the velocity one cycle before the state the
// pass leaves) into the two planes d.uprev, for the steady residual. Only the
// last pass of an lbm_step call records it; the planes are below 4 GiB
// whenever multi-cycle passes run.
__device__ __forceinline__ void store_uprev(const Dom &d, uint32_t o4, float ux, float uy) {
    const BufRes r = buf_res(d.uprev, (uint32_t)(2 * d.plane * 4));
    if (d.nt_store) {
        BufIO<float>::st_nt(r, o4, 0u, ux);
        BufIO<float>::st_nt(r, o4, (uint32_t)(d.plane * 4), uy);
    } else {
        BufIO<float>::st(r, o4, 0u, ux);
        BufIO<float>::st(r, o4, (uint32_t)(d.plane * 4), uy);
    }
}

// ------------------------------------------------- two steps per pass

// Temporal blocking: one launch advances t -> t + 2 with a single HBM pass.
// A workgroup owns a TW x TH output tile. Phase A gathers f(t) (from the
// post-collision state s_t in HBM) and collides on the tile plus a one-node
// ring, keeping s_{t+1} in LDS; phase B gathers f(t+1) from LDS (periodic
// neighbours are in the ring, walls bounce back), collides, and stores
// s_{t+2}. Per output node the pass reads (TW+2)(TH+2)/(TW TH) populations and
// writes one, instead of reading and writing one per step. Every node runs
// the same per-node code as the one-step kernel, and FP16 storage rounds the
// intermediate state exactly as a store/reload would, so the result is
// bitwise that of two one-step launches. With THERMAL the D2Q5 field takes the
// same path: phase A keeps g beside f in LDS (ldsg, five planes), phase B
// gathers it with bounce-back and anti-bounce-back across the walls.
//
// Work items: thread (wave w, lane l) owns row r = w + NW k of the
// (TW + 2) x (TH + 2) frame, column 1 + l, in both phases (phase B visits
// rows 1 .. TH), so its node's porosity is loaded and its drag coefficients
// computed once, in phase A. Each wave covers one whole TW = 64 row; the two
// ring columns go to the waves without a row at the last iteration.
template <typename S, int TW, int TH, int NT, bool REC, int MK, bool THERMAL>
__device__ __forceinline__ void step2_tile(const Dom &d, int x0, int y0, float *urec_next,
                                           float (&lds)[8][TH + 2][TW + 2], float *ldsg) {
    constexpr int EW = TW + 2, EH = TH + 2;
    constexpr int ES = (int)sizeof(S);
    constexpr int NW = NT / 64;                 // waves per workgroup
    constexpr int NK = (EH + NW - 1) / NW;      // frame rows per thread
    constexpr int WR = EH - NW * (NK - 1);      // first wave without a row at k = NK - 1
    constexpr int RA = 2 * EH;                  // ring items of phase A
    static_assert(TW == 64 && NT % 64 == 0, "one tile row per wave");
    static_assert((NW - WR) * 64 >= RA, "ring items fit the free waves");
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    // the state buffers are below 4 GiB (the host keeps larger domains on the
    // one-cycle kernel), so every byte offset fits the buffer instructions
    const uint32_t fbytes = (uint32_t)(8 * d.plane * ES);
    const BufRes rin = buf_res(d.fin, fbytes), rout = buf_res(d.fout, fbytes);
    // recorded planes: u (2), the stress moments (2, with rec_stress), dT (plane 4, thermal)
    const uint32_t rbytes = REC ? (uint32_t)((THERMAL ? 5 : (d.rec_stress ? 4 : 2)) * d.plane * 4) : 0u;
    // D2Q5 buffers (FP32, five planes, also below 4 GiB)
    const uint32_t gbytes = THERMAL ? (uint32_t)(5 * d.plane * 4) : 0u;
    const BufRes rgin = buf_res(THERMAL ? d.gin : nullptr, gbytes), rgout = buf_res(THERMAL ? d.gout : nullptr, gbytes);
    const MediumSrc<MK> med(d);
    // every source of phase A inside the domain, no wrap needed
    const bool interior = x0 >= 2 && x0 + TW + 2 <= d.nx && y0 >= 2 && y0 + TH + 2 <= d.ny;
    Cell ck[NK];   // the cell of this thread's frame node k (rows only, not ring items)

    // item k of phase A: the thread's frame row, or at k = NK - 1 a ring item
    auto a_item = [&](int k, int &ex, int &ey) -> bool {
        ey = w + NW * k;
        ex = 1 + lane;
        if (k < NK - 1 || ey < EH) return true;
        const int ri = (w - WR) * 64 + lane;
        if (ri >= RA) return false;
        ey = ri >> 1;
        ex = (ri & 1) ? EW - 1 : 0;
        return true;
    };

    // phase A: s_{t+1} on the extended tile (and u(t) on the tile when recording)
    auto finish_a = [&](int k, float (&f)[8], float (&g)[5], const CellRaw &raw, int ex, int ey, int64_t o) {
        const Cell c = med.cell(d, raw);
        ck[k] = c;
        float ux, uy, n7, n8, dT;
        node_update<THERMAL>(d, c, f, g, ux, uy, n7, n8, dT);
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[i][ey][ex] = (float)(S)f[i];
        if (THERMAL) {
#pragma unroll
            for (int j = 0; j < 5; ++j) ldsg[(j * EH + ey) * EW + ex] = g[j];
        }
        if (REC && ex >= 1 && ex <= TW && ey >= 1 && ey <= TH && x0 - 1 + ex < d.nx &&
            y0 - 1 + ey < d.ny) {
            const BufRes rr = buf_res(d.urec, rbytes);
            record_node(d, rr, (uint32_t)(o * 4), ux, uy, n7, n8);
            if (THERMAL) BufIO<float>::st_nt(rr, (uint32_t)(o * 4), (uint32_t)(4 * d.plane * 4), dT);
        }
    };
    if (interior) {
        // link i pulls from (gx - e_ix, gy - e_iy): the lane's offset of (gx - 1, gy - 1)
        // plus a uniform, non-negative per-link offset. Software pipelined: the next
        // item's loads are issued before this one collides.
        auto fetch = [&](int k, float (&f)[8], float (&g)[5], CellRaw &r, int &ex, int &ey) -> bool {
            if (!a_item(k, ex, ey)) return false;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            const uint32_t vo = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * ES);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                f[i] = BufIO<S>::ld(rin, vo, (uint32_t)((i * d.plane + (1 - EY[i]) * d.pitch + (1 - EX[i])) * ES));
            if (THERMAL) {
                const uint32_t vg = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * 4);
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    g[j] = BufIO<float>::ld(rgin, vg, (uint32_t)((j * d.plane + (1 - TYv[j]) * d.pitch + (1 - TXv[j])) * 4));
            }
            r = med.load((uint32_t)((gy * d.pitch + gx) * 4));
            return true;
        };
        float fn[8], gn[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        CellRaw rn{0.0f, 0.0f, 0.0f};
        int exn = 0, eyn = 0;
        bool vn = fetch(0, fn, gn, rn, exn, eyn);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            float f[8], g[5];
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = fn[i];
#pragma unroll
            for (int j = 0; j < 5; ++j) g[j] = gn[j];
            const CellRaw r = rn;
            const int ex = exn, ey = eyn;
            const bool v = vn;
            if (k + 1 < NK) vn = fetch(k + 1, fn, gn, rn, exn, eyn);
            if (v) finish_a(k, f, g, r, ex, ey, (int64_t)(y0 - 1 + ey) * d.pitch + (x0 - 1 + ex));
        }
    } else {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            int ex, ey;
            if (!a_item(k, ex, ey)) continue;
            int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            if (gx < 0 || gx >= d.nx) {
                if (d.bc_x != BC_PERIODIC) continue;
                gx = ((gx % d.nx) + d.nx) % d.nx;
            }
            if (gy < 0 || gy >= d.ny) {
                if (d.bc_y != BC_PERIODIC) continue;
                gy = ((gy % d.ny) + d.ny) % d.ny;
            }
            float f[8], g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            gather_general_buf<S>(d, rin, gx, gy, f);
            if (THERMAL) gather_thermal_buf(d, rgin, gx, gy, g);
            const int64_t o = (int64_t)gy * d.pitch + gx;
            finish_a(k, f, g, med.load((uint32_t)(o * 4)), ex, ey, o);
        }
    }
    lds_barrier();

    // phase B: s_{t+2} on the tile (and u(t+1) when recording)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int ly = w + NW * k - 1, lx = lane;
        const int gx = x0 + lx, gy = y0 + ly;
        if (ly < 0 || ly >= TH || gx >= d.nx || gy >= d.ny) continue;
        float f[8];
        const float *flat = &lds[0][0][0];
        if (interior) {
            // every source is the neighbour's value: one base, constant offsets
            const int base = (ly + 1) * EW + lx + 1;
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = flat[base + i * EH * EW - EY[i] * EW - EX[i]];
        } else {
            // one LDS read per link at a selected index (the neighbour's value, or the
            // node's own opposite value across a wall); written as an index select
            // rather than two guarded reads, a form the compiler got wrong here
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                bool out = false, top = false;
                const int sx = gx - EX[i], sy = gy - EY[i];
                if (EX[i] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) out = true;
                if (EY[i] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) {
                    out = true;
                    top = (sy >= d.ny);
                }
                const int src = out ? (OPP[i] * EH + ly + 1) * EW + lx + 1
                                    : (i * EH + ly + 1 - EY[i]) * EW + lx + 1 - EX[i];
                const float v = flat[src];
                f[i] = top ? v + (float)EX[i] * d.lid6 : v;
            }
        }
        float g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (THERMAL) {
            // the D2Q5 links: the neighbour's value, or across a wall the node's own
            // opposite value (bounce-back on y walls, anti-bounce-back on x walls),
            // again as one read at a selected index
            g[0] = ldsg[(ly + 1) * EW + lx + 1];
#pragma unroll
            for (int j = 1; j < 5; ++j) {
                int kind = 0;
                if (!interior) {
                    const int sx = gx - TXv[j], sy = gy - TYv[j];
                    if (TXv[j] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) kind = (sx < 0) ? 2 : 3;
                    if (TYv[j] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) kind = 1;
                }
                const int src = kind == 0 ? (j * EH + ly + 1 - TYv[j]) * EW + lx + 1 - TXv[j]
                                          : (TOPP[j] * EH + ly + 1) * EW + lx + 1;
                const float v = ldsg[src];
                g[j] = (kind <= 1) ? v : ((kind == 2) ? d.abbh - v : d.abbc - v);
            }
        }
        const int64_t o = (int64_t)gy * d.pitch + gx;
        float ux, uy, n7, n8, dT;
        node_update<THERMAL>(d, ck[k], f, g, ux, uy, n7, n8, dT);
        const uint32_t vo = (uint32_t)(o * ES);
        if (d.nt_store) {
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<S>::st_nt(rout, vo, (uint32_t)(i * d.plane * ES), f[i]);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<S>::st(rout, vo, (uint32_t)(i * d.plane * ES), f[i]);
        }
        if (THERMAL) {
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                if (d.nt_store) BufIO<float>::st_nt(rgout, (uint32_t)(o * 4), (uint32_t)(j * d.plane * 4), g[j]);
                else BufIO<float>::st(rgout, (uint32_t)(o * 4), (uint32_t)(j * d.plane * 4), g[j]);
            }
        }
        if (d.uprev) store_uprev(d, (uint32_t)(o * 4), ux, uy);
        if (REC) {
            const BufRes rr = buf_res(urec_next, rbytes);
            record_node(d, rr, (uint32_t)(o * 4), ux, uy, n7, n8);
            if (THERMAL) BufIO<float>::st_nt(rr, (uint32_t)(o * 4), (uint32_t)(4 * d.plane * 4), dT);
        }
    }
}


template <typename S, int TW, int TH, int NT, bool REC, int MK, bool THERMAL>
__global__ __launch_bounds__(NT) void k_step2(Dom d, int tiles_x, int swz, float *urec_next) {
    __shared__ float lds[8][TH + 2][TW + 2];
    __shared__ float ldsg[THERMAL ? 5 * (TH + 2) * (TW + 2) : 1];
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    step2_tile<S, TW, TH, NT, REC, MK, THERMAL>(d, (b % tiles_x) * TW, (b / tiles_x) * TH, urec_next, lds, ldsg);
}

// Batched two-cycle pass over a table of 64 x TH tiles: with ONE each workgroup
// takes one tile (grid == ntiles), else workgroup b walks a contiguous run.
template <typename S, int TW, int TH, int NT, int MK, bool THERMAL, bool ONE>
__global__ __launch_bounds__(NT) void k_step2_batch(const Dom *__restrict__ doms,
                                                    const int4 *__restrict__ tiles, int ntiles,
                                                    int parity) {
    __shared__ float lds[8][TH + 2][TW + 2];
    __shared__ float ldsg[THERMAL ? 5 * (TH + 2) * (TW + 2) : 1];
    if (ONE) {
        // one workgroup per tile (grid == ntiles): no loop state stays live
        const int4 tl = tiles[blockIdx.x];
        const Dom d = doms[2 * tl.x + parity];
        step2_tile<S, TW, TH, NT, false, MK, THERMAL>(d, tl.y * TW, tl.z * TH, nullptr, lds, ldsg);
        return;
    }
    const int64_t nb = gridDim.x;
    const int t0 = (int)((int64_t)blockIdx.x * ntiles / nb);
    const int t1 = (int)(((int64_t)blockIdx.x + 1) * ntiles / nb);
    for (int t = t0; t < t1; ++t) {
        const int4 tl = tiles[t];
        const Dom d = doms[2 * tl.x + parity];
        step2_tile<S, TW, TH, NT, false, MK, THERMAL>(d, tl.y * TW, tl.z * TH, nullptr, lds, ldsg);
        lds_barrier();   // the next tile's phase A rewrites the LDS
    }
}

constexpr int STEP2_TW = 64;

// Compiled two-cycle tiles: (threads per workgroup, tile rows); tiles are 64 wide.
#define MRT_STEP2_SHAPES(X) X(256, 16) X(512, 16) X(256, 8) X(512, 8)

bool step2_shape_supported(int threads, int rows) {
#define MRT_S2SUP(N, H) if (threads == N && rows == H) return true;
    MRT_STEP2_SHAPES(MRT_S2SUP)
#undef MRT_S2SUP
    return false;
}

void step2_tiles(int nx, int ny, int rows, int *tiles_x, int *tiles_y) {
    *tiles_x = (nx + STEP2_TW - 1) / STEP2_TW;
    *tiles_y = (ny + rows - 1) / rows;
}

// ------------------------------------------------ three steps per pass

// One LDS gather of a node whose own values sit at (cx, cy) of a W x H tile
// layout (plane stride W H): the neighbour's post-collision value per link,
// or across a wall the node's own opposite value plus the lid term. With
// `interior` every source is a neighbour (constant offsets).
template <int W, int H>
__device__ __forceinline__ void lds_gather(const Dom &d, const float *flat, bool interior, int gx, int gy,
                                           int cx, int cy, float f[8]) {
    if (interior) {
        const int base = cy * W + cx;
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = flat[base + i * W * H - EY[i] * W - EX[i]];
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        bool out = false, top = false;
        const int sx = gx - EX[i], sy = gy - EY[i];
        if (EX[i] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) out = true;
        if (EY[i] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) {
            out = true;
            top = (sy >= d.ny);
        }
        const int src = out ? (OPP[i] * H + cy) * W + cx : (i * H + cy - EY[i]) * W + cx - EX[i];
        const float v = flat[src];
        f[i] = top ? v + (float)EX[i] * d.lid6 : v;
    }
}

// The D2Q5 links of node (gx, gy) from an LDS layout [5][H][W] at position
// (cx, cy): the neighbour's value, or across a wall the node's own opposite
// link (bounce-back on y walls, anti-bounce-back on x walls), as one read at a
// selected index.
template <int W, int H>
__device__ __forceinline__ void lds_gather_thermal(const Dom &d, const float *flat, bool interior, int gx, int gy,
                                                   int cx, int cy, float g[5]) {
    g[0] = flat[cy * W + cx];
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        int kind = 0;
        if (!interior) {
            const int sx = gx - TXv[j], sy = gy - TYv[j];
            if (TXv[j] != 0 && (sx < 0 || sx >= d.nx) && d.bc_x != BC_PERIODIC) kind = (sx < 0) ? 2 : 3;
            if (TYv[j] != 0 && (sy < 0 || sy >= d.ny) && d.bc_y != BC_PERIODIC) kind = 1;
        }
        const int src = kind == 0 ? (j * H + cy - TYv[j]) * W + cx - TXv[j] : (TOPP[j] * H + cy) * W + cx;
        const float v = flat[src];
        g[j] = (kind <= 1) ? v : ((kind == 2) ? d.abbh - v : d.abbc - v);
    }
}


// Temporal blocking over three cycles: a workgroup owns a TW x TH tile. Phase A
// gathers f(t) from HBM on the tile plus a two-node ring and collides into LDS;
// phase B gathers f(t+1) from LDS on the tile plus a one-node ring, collides and
// keeps the results in registers; after a barrier they replace phase A's values
// in the same LDS (a smaller layout), and phase C gathers f(t+2), collides and
// stores f+(t+2). Same per-node function and FP16 rounding of every
// intermediate as three one-cycle passes, so the result is bitwise theirs.
//
// Work items: thread (wave w, lane l) owns row r = w + NW k of the
// (TW + 4) x (TH + 4) frame of phase A, column 2 + l, for k = 0 .. NK - 1, in
// every phase: phase A visits all frame rows, phase B rows 1 .. TH + 2 and
// phase C rows 2 .. TH + 1, so a thread meets the same node in each phase. The
// node's porosity is loaded and its drag coefficients computed once, in phase
// A, and kept in registers for B and C. Each wave covers one whole TW = 64
// row (aligned, coalesced loads, stride-1 LDS access); the ring columns (4 of
// phase A, 2 of phase B) go to the waves without a row at the last iteration.
// With REC (FP32 recomputation for the adjoint) u and, with rec_stress, the
// stress moments of the tile nodes are recorded at t (d.urec), t + 1 (urec1)
// and t + 2 (urec2).
template <typename S, int TW, int TH, int NT, bool REC, int MK, bool THERMAL>
__device__ __forceinline__ void step3_tile(const Dom &d, int x0, int y0, float *urec1, float *urec2, float *lds,
                                           float *ldsg) {
    constexpr int AW = TW + 4, AH = TH + 4;
    constexpr int BW = TW + 2, BH = TH + 2, BN = BW * BH;
    constexpr int ES = (int)sizeof(S);
    constexpr int NW = NT / 64;                 // waves per workgroup
    constexpr int NK = (AH + NW - 1) / NW;      // frame rows per thread
    constexpr int WR = AH - NW * (NK - 1);      // first wave without a row at k = NK - 1
    constexpr int RA = 4 * AH, RB = 2 * BH;     // ring items of phases A and B
    static_assert(TW == 64 && NT % 64 == 0, "one tile row per wave");
    static_assert((NW - WR) * 64 >= RA && (NW - WR) * 64 >= RB, "ring items fit the free waves");
    static_assert(WR >= BH + 1 - NW * (NK - 1) && WR >= TH + 2 - NW * (NK - 1), "free waves have no B or C row");
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const uint32_t fbytes = (uint32_t)(8 * d.plane * ES);
    const BufRes rin = buf_res(d.fin, fbytes), rout = buf_res(d.fout, fbytes);
    const MediumSrc<MK> med(d);
    const bool interior = x0 >= 3 && x0 + TW + 3 <= d.nx && y0 >= 3 && y0 + TH + 3 <= d.ny;
    // resources of the three recorded steps, each built where its phase starts
    const uint32_t rbytes = REC ? (uint32_t)((THERMAL ? 5 : (d.rec_stress ? 4 : 2)) * d.plane * 4) : 0u;
    // D2Q5 buffers (FP32, five planes, below 4 GiB)
    const uint32_t gbytes = THERMAL ? (uint32_t)(5 * d.plane * 4) : 0u;
    const BufRes rgin = buf_res(THERMAL ? d.gin : nullptr, gbytes), rgout = buf_res(THERMAL ? d.gout : nullptr, gbytes);

    // CDNA's vector-memory counter retires loads and stores in order, so a wait
    // for a load also waits for every store issued before it. Each phase
    // therefore issues its global loads before the stores that belong to the
    // previous node: records are held one node (Pending).
    Pending<THERMAL> pend;
    Cell ck[NK];   // the cell of this thread's frame node k (rows only, not ring items)

    // item k of phase A: the thread's frame row, or at k = NK - 1 a ring item
    auto a_item = [&](int k, int &ca, int &ra) -> bool {
        ra = w + NW * k;
        ca = 2 + lane;
        if (k < NK - 1 || ra < AH) return true;
        const int ri = (w - WR) * 64 + lane;
        if (ri >= RA) return false;
        ra = ri >> 2;
        const int c = ri & 3;
        ca = c < 2 ? c : TW + c;
        return true;
    };

    // phase A: s_{t+1} on the tile + 2 ring
    const BufRes rr0 = buf_res(REC ? d.urec : nullptr, rbytes);
    auto finish_a = [&](int k, float (&f)[8], float (&g)[5], const CellRaw &raw, int ca, int ra, int64_t o) {
        if (REC) pend.flush(d, rr0);
        const Cell c = med.cell(d, raw);
        ck[k] = c;
        float ux, uy, n7, n8, dT;
        node_update<THERMAL>(d, c, f, g, ux, uy, n7, n8, dT);
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[(i * AH + ra) * AW + ca] = (float)(S)f[i];
        if (THERMAL) {
#pragma unroll
            for (int j = 0; j < 5; ++j) ldsg[(j * AH + ra) * AW + ca] = g[j];
        }
        if (REC && ca >= 2 && ca < TW + 2 && ra >= 2 && ra < TH + 2 && x0 - 2 + ca < d.nx && y0 - 2 + ra < d.ny)
            pend.hold((uint32_t)(o * 4), ux, uy, n7, n8, dT);
    };
    if (interior) {
        // software pipelined: the next item's loads are issued before this one collides
        auto fetch = [&](int k, float (&f)[8], float (&g)[5], CellRaw &r, int &ca, int &ra) -> bool {
            if (!a_item(k, ca, ra)) return false;
            const int gx = x0 - 2 + ca, gy = y0 - 2 + ra;
            const uint32_t vo = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * ES);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                f[i] = BufIO<S>::ld(rin, vo, (uint32_t)((i * d.plane + (1 - EY[i]) * d.pitch + (1 - EX[i])) * ES));
            if (THERMAL) {
                const uint32_t vg = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * 4);
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    g[j] = BufIO<float>::ld(rgin, vg, (uint32_t)((j * d.plane + (1 - TYv[j]) * d.pitch + (1 - TXv[j])) * 4));
            }
            r = med.load((uint32_t)((gy * d.pitch + gx) * 4));
            return true;
        };
        float fn[8], gn[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        CellRaw rn{0.0f, 0.0f, 0.0f};
        int can = 0, ran = 0;
        bool vn = fetch(0, fn, gn, rn, can, ran);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            float f[8], g[5];
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = fn[i];
#pragma unroll
            for (int j = 0; j < 5; ++j) g[j] = gn[j];
            const CellRaw r = rn;
            const int ca = can, ra = ran;
            const bool v = vn;
            if (k + 1 < NK) vn = fetch(k + 1, fn, gn, rn, can, ran);
            if (v) finish_a(k, f, g, r, ca, ra, (int64_t)(y0 - 2 + ra) * d.pitch + (x0 - 2 + ca));
        }
    } else {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            int ca, ra;
            if (!a_item(k, ca, ra)) continue;
            int gx = x0 - 2 + ca, gy = y0 - 2 + ra;
            if (!wrap_node(d, gx, gy)) continue;
            float f[8], g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            gather_general_buf<S>(d, rin, gx, gy, f);
            if (THERMAL) gather_thermal_buf(d, rgin, gx, gy, g);
            const int64_t o = (int64_t)gy * d.pitch + gx;
            // a wrapped ring node is recorded by the tile that owns it
            finish_a(k, f, g, med.load((uint32_t)(o * 4)), ca, ra, o);
        }
    }
    if (REC) pend.flush(d, rr0);
    lds_barrier();

    // phase B: s_{t+2} on the tile + 1 ring, kept in registers
    const BufRes rr1 = buf_res(urec1, rbytes);
    float fb[NK][8], gb[NK][THERMAL ? 5 : 1];
    int slot[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        slot[k] = -1;
        const int rb = w + NW * k - 1;
        int bx = 1 + lane, by = rb;
        const bool row = rb >= 0 && rb < BH;
        if (!row) {
            const int ri = (w - WR) * 64 + lane;
            if (k != NK - 1 || w < WR || ri >= RB) continue;
            by = ri >> 1;
            bx = (ri & 1) ? BW - 1 : 0;
        }
        int gx = x0 - 1 + bx, gy = y0 - 1 + by;
        if (!interior && !wrap_node(d, gx, gy)) continue;
        const int64_t o = (int64_t)gy * d.pitch + gx;
        Cell c;
        if (row) {
            c = ck[k];
        } else {
            c = med.cell(d, med.load((uint32_t)(o * 4)));
        }
        lds_gather<AW, AH>(d, lds, interior, gx, gy, bx + 1, by + 1, fb[k]);
        float g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (THERMAL) lds_gather_thermal<AW, AH>(d, ldsg, interior, gx, gy, bx + 1, by + 1, g);
        float ux, uy, n7, n8, dT;
        node_update<THERMAL>(d, c, fb[k], g, ux, uy, n7, n8, dT);
        if (THERMAL) {
#pragma unroll
            for (int j = 0; j < 5; ++j) gb[k][THERMAL ? j : 0] = g[j];
        }
        // phase B loads nothing from HBM on tile rows, so its records are stored
        // at once rather than held behind the next node's loads
        if (REC && bx >= 1 && bx <= TW && by >= 1 && by <= TH && x0 - 1 + bx < d.nx && y0 - 1 + by < d.ny) {
            record_node(d, rr1, (uint32_t)(o * 4), ux, uy, n7, n8);
            if (THERMAL) BufIO<float>::st_nt(rr1, (uint32_t)(o * 4), (uint32_t)(4 * d.plane * 4), dT);
        }
        slot[k] = by * BW + bx;
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        if (slot[k] < 0) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[i * BN + slot[k]] = (float)(S)fb[k][i];
        if (THERMAL) {
#pragma unroll
            for (int j = 0; j < 5; ++j) ldsg[j * BN + slot[k]] = gb[k][THERMAL ? j : 0];
        }
    }
    lds_barrier();

    // phase C: s_{t+3} on the tile, to HBM
    const BufRes rr2 = buf_res(urec2, rbytes);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int rc = w + NW * k - 2;
        const int gx = x0 + lane, gy = y0 + rc;
        if (rc < 0 || rc >= TH || gx >= d.nx || gy >= d.ny) continue;
        float f[8], g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        lds_gather<BW, BH>(d, lds, interior, gx, gy, lane + 1, rc + 1, f);
        if (THERMAL) lds_gather_thermal<BW, BH>(d, ldsg, interior, gx, gy, lane + 1, rc + 1, g);
        const int64_t o = (int64_t)gy * d.pitch + gx;
        float ux, uy, n7, n8, dT;
        node_update<THERMAL>(d, ck[k], f, g, ux, uy, n7, n8, dT);
        const uint32_t vo = (uint32_t)(o * ES);
        // one branch for the whole store sequence (per-store branches split the stream)
        if (d.nt_store) {
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<S>::st_nt(rout, vo, (uint32_t)(i * d.plane * ES), f[i]);
            if (THERMAL) {
#pragma unroll
                for (int j = 0; j < 5; ++j) BufIO<float>::st_nt(rgout, (uint32_t)(o * 4), (uint32_t)(j * d.plane * 4), g[j]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<S>::st(rout, vo, (uint32_t)(i * d.plane * ES), f[i]);
            if (THERMAL) {
#pragma unroll
                for (int j = 0; j < 5; ++j) BufIO<float>::st(rgout, (uint32_t)(o * 4), (uint32_t)(j * d.plane * 4), g[j]);
            }
        }
        if (d.uprev) store_uprev(d, (uint32_t)(o * 4), ux, uy);
        if (REC) {
            record_node(d, rr2, (uint32_t)(o * 4), ux, uy, n7, n8);
            if (THERMAL) BufIO<float>::st_nt(rr2, (uint32_t)(o * 4), (uint32_t)(4 * d.plane * 4), dT);
        }
    }
}

// The isothermal recording pass is held to 80 VGPRs, six waves per SIMD: three
// 512-thread workgroups per CU instead of two (a two-dword spill).
template <typename S, int TW, int TH, int NT, bool REC, int MK, bool THERMAL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(REC && !THERMAL ? 6 : 1))) void k_step3(
    Dom d, int tiles_x, int swz, float *urec1, float *urec2) {
    __shared__ float lds[8 * (TH + 4) * (TW + 4)];
    __shared__ float ldsg[THERMAL ? 5 * (TH + 4) * (TW + 4) : 1];
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    step3_tile<S, TW, TH, NT, REC, MK, THERMAL>(d, (b % tiles_x) * TW, (b / tiles_x) * TH, urec1, urec2, lds, ldsg);
}

// Batched three-cycle pass over a table of TW x TH tiles (isothermal domains;
// MK_BRANCHED for any medium, MK_UNIFORM when every domain is uniform); ONE as
// for the two-cycle pass.
template <typename S, int TW, int TH, int NT, int MK, bool ONE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(ONE ? 6 : 4))) void k_step3_batch(const Dom *__restrict__ doms, const int4 *__restrict__ tiles,
                                                    int ntiles, int parity) {
    __shared__ float lds[8 * (TH + 4) * (TW + 4)];
    if (ONE) {
        // one workgroup per tile (grid == ntiles): without the loop's state the
        // kernel stays within its registers (the loop variant spills)
        const int4 tl = tiles[blockIdx.x];
        const Dom d = doms[2 * tl.x + parity];
        step3_tile<S, TW, TH, NT, false, MK, false>(d, tl.y * TW, tl.z * TH, nullptr, nullptr, lds, nullptr);
        return;
    }
    const int64_t nb = gridDim.x;
    const int t0 = (int)((int64_t)blockIdx.x * ntiles / nb);
    const int t1 = (int)(((int64_t)blockIdx.x + 1) * ntiles / nb);
    for (int t = t0; t < t1; ++t) {
        const int4 tl = tiles[t];
        const Dom d = doms[2 * tl.x + parity];
        step3_tile<S, TW, TH, NT, false, MK, false>(d, tl.y * TW, tl.z * TH, nullptr, nullptr, lds, nullptr);
        lds_barrier();   // the next tile's phase A rewrites the LDS
    }
}

// Batched passes and single domains below 2^23 nodes: 64 x 16 tiles, 512 threads.
constexpr int STEP3_TW = 64, STEP3_TH = 16, STEP3_NT = 512;
// Single isothermal domains of 2^23 nodes or more: 64 x 28 tiles with 768
// threads (12 waves: 8 with three frame rows, 4 with two plus the ring
// columns), two workgroups and 24 waves per CU. The ring recomputation falls
// from 3572 collisions per 3072 updates (1.163) to 5948 per 5376 (1.106).
// Measured (log-normal channel, FP32, ms per step): 8192^2 0.326 against
// 0.342, 4096^2 0.0830 against 0.0873, but 2048^2 0.0246 against 0.0236 and
// 1024^2 0.0080 against 0.0077, where fewer, larger workgroups lose more to
// the tail of the grid than they save. At 8192^2, 64 x 18 tiles with 512
// threads took 1.01 ms per launch and 64 x 24 with 640 threads 1.41 ms
// (ten waves leave room for one workgroup per CU), against 0.967 here.
// Thermal domains (13 LDS planes) and the recording pass (80 VGPRs) keep
// 64 x 16: at 768 threads either would leave one workgroup per CU. Single
// isothermal domains of 2^23 nodes or more take four cycles per pass by
// default (k_step4 below); these tiles serve them when switched to three.
constexpr int STEP3_TH_TALL = 28, STEP3_NT_TALL = 768;

static bool step3_tall(const Dom &d, bool rec) {
    return !d.thermal && !rec && (int64_t)d.nx * d.ny >= ((int64_t)1 << 23);
}

void step3_tiles(const Dom &d, bool rec, int *tiles_x, int *tiles_y) {
    const int th = step3_tall(d, rec) ? STEP3_TH_TALL : STEP3_TH;
    *tiles_x = (d.nx + STEP3_TW - 1) / STEP3_TW;
    *tiles_y = (d.ny + th - 1) / th;
}

int step3_single_threads(const Dom &d, bool rec) { return step3_tall(d, rec) ? STEP3_NT_TALL : STEP3_NT; }

int step3_single_rows(const Dom &d, bool rec) { return step3_tall(d, rec) ? STEP3_TH_TALL : STEP3_TH; }

template <int MK, bool TH>
static const void *step3_fn_t(int storage, bool rec, bool tall) {
    if (rec) return storage == ST_F32 ? (const void *)&k_step3<float, STEP3_TW, STEP3_TH, STEP3_NT, true, MK, TH> : nullptr;
    if constexpr (!TH) {
        if (tall)
            return storage == ST_F32
                       ? (const void *)&k_step3<float, STEP3_TW, STEP3_TH_TALL, STEP3_NT_TALL, false, MK, false>
                       : (const void *)&k_step3<_Float16, STEP3_TW, STEP3_TH_TALL, STEP3_NT_TALL, false, MK, false>;
    }
    return storage == ST_F32 ? (const void *)&k_step3<float, STEP3_TW, STEP3_TH, STEP3_NT, false, MK, TH>
                             : (const void *)&k_step3<_Float16, STEP3_TW, STEP3_TH, STEP3_NT, false, MK, TH>;
}

template <bool TH>
static const void *step3_fn_th(const Dom &d, int storage, bool rec) {
    const bool tall = step3_tall(d, rec);
    switch (medium_kind(d)) {
    case MK_ERGUN: return step3_fn_t<MK_ERGUN, TH>(storage, rec, tall);
    case MK_UNIFORM: return step3_fn_t<MK_UNIFORM, TH>(storage, rec, tall);
    default: return step3_fn_t<MK_ANY, TH>(storage, rec, tall);
    }
}

const void *step3_kernel_fn(const Dom &d, int storage, bool rec) {
    return d.thermal ? step3_fn_th<true>(d, storage, rec) : step3_fn_th<false>(d, storage, rec);
}

template <int MK, bool ONE>
static const void *step3_batch_fn_mk(int storage) {
    return storage == ST_F32 ? (const void *)&k_step3_batch<float, STEP3_TW, STEP3_TH, STEP3_NT, MK, ONE>
                             : (const void *)&k_step3_batch<_Float16, STEP3_TW, STEP3_TH, STEP3_NT, MK, ONE>;
}

const void *step3_batch_kernel_fn(int storage, bool uniform, bool one) {
    if (one) return uniform ? step3_batch_fn_mk<MK_UNIFORM, true>(storage) : step3_batch_fn_mk<MK_BRANCHED, true>(storage);
    return uniform ? step3_batch_fn_mk<MK_UNIFORM, false>(storage) : step3_batch_fn_mk<MK_BRANCHED, false>(storage);
}

int step3_threads() { return STEP3_NT; }

hipError_t launch_step3_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity, int storage, bool uniform,
                              int grid, hipStream_t st) {
    if (grid <= 0 || ntiles <= 0) return hipErrorInvalidValue;
    if (grid > ntiles) grid = ntiles;   // workgroups beyond the last tile would idle
    const void *fn = step3_batch_kernel_fn(storage, uniform, grid == ntiles);
    void *args[4] = {&doms, &tiles, &ntiles, &parity};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(STEP3_NT), args, 0, st);
}

hipError_t launch_step3(const Dom &d, int storage, int swizzle, float *urec1, float *urec2, hipStream_t st) {
    const bool rec = urec1 != nullptr;
    const void *fn = step3_kernel_fn(d, storage, rec);
    if (!fn || (rec && (!d.urec || !urec2))) return hipErrorInvalidValue;
    int tx, ty;
    step3_tiles(d, rec, &tx, &ty);
    Dom dd = d;
    int swz = swizzle;
    void *args[5] = {&dd, &tx, &swz, &urec1, &urec2};
    return hipLaunchKernel(fn, dim3((unsigned)(tx * ty)), dim3((unsigned)step3_single_threads(d, rec)), args, 0, st);
}

// ------------------------------------------------- four cycles per pass

// Temporal blocking over four cycles, for isothermal domains (single, batched,
// and the recording pass of the adjoint's recomputation): the three-cycle pass
// with one more LDS phase. A workgroup owns a
// TW x TH tile. Phase A gathers f(t) from HBM on the tile plus a three-node
// ring and collides into LDS; phase B gathers f(t+1) from LDS on the tile plus
// a two-node ring and phase C f(t+2) on the tile plus a one-node ring, each
// keeping its results in registers until a barrier lets them replace the
// previous layout in the same LDS (each layout smaller than the one before);
// phase D gathers f(t+3), collides and stores f+(t+3). Same per-node function
// and FP16 rounding of every intermediate as four one-cycle passes, so the
// result is bitwise theirs.
//
// Thread (wave w, lane l) owns row r = w + NW k of the (TW + 6) x (TH + 6)
// frame of phase A, column 3 + l, in every phase (phase B visits frame rows
// 1 .. TH + 4, C rows 2 .. TH + 3, D rows 3 .. TH + 2), so its cell is
// computed once; the ring columns (6 of phase A, 4 of B, 2 of C) go to the
// waves without a row at the last iteration. With REC (FP32 recomputation for
// the adjoint) u and, with rec_stress, the stress moments of the tile nodes are
// recorded at t (d.urec), t + 1, t + 2 and t + 3 (urec1 .. urec3).
template <typename S, int TW, int TH, int NT, bool REC, int MK>
__device__ __forceinline__ void step4_tile(const Dom &d, int x0, int y0, float *urec1, float *urec2, float *urec3,
                                           float *lds) {
    constexpr int AW = TW + 6, AH = TH + 6;
    constexpr int BW = TW + 4, BH = TH + 4, BN = BW * BH;
    constexpr int CW = TW + 2, CH = TH + 2, CN = CW * CH;
    constexpr int ES = (int)sizeof(S);
    constexpr int NW = NT / 64;                 // waves per workgroup
    constexpr int NK = (AH + NW - 1) / NW;      // frame rows per thread
    constexpr int WR = AH - NW * (NK - 1);      // first wave without a row at k = NK - 1
    constexpr int RA = 6 * AH, RB = 4 * BH, RC = 2 * CH;   // ring items of phases A, B, C
    static_assert(TW == 64 && NT % 64 == 0, "one tile row per wave");
    static_assert((NW - WR) * 64 >= RA && RA >= RB && RB >= RC, "ring items fit the free waves");
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const uint32_t fbytes = (uint32_t)(8 * d.plane * ES);
    const BufRes rin = buf_res(d.fin, fbytes), rout = buf_res(d.fout, fbytes);
    const MediumSrc<MK> med(d);
    // every gather of every phase reads inside the domain, at constant offsets
    const bool interior = x0 >= 4 && x0 + TW + 4 <= d.nx && y0 >= 4 && y0 + TH + 4 <= d.ny;
    Cell ck[NK];   // the cell of this thread's frame node k (rows only, not ring items)
    float g[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // no D2Q5 field
    float ux, uy, n7, n8, dT;
    // the recorded planes of one step (u, and with rec_stress the stress moments)
    const uint32_t rbytes = REC ? (uint32_t)((d.rec_stress ? 4 : 2) * d.plane * 4) : 0u;
    // phase A's records are held one node, so that its loads go out before them
    Pending<false> pend;

    // item k of phase A: the thread's frame row, or at k = NK - 1 a ring item
    auto a_item = [&](int k, int &ca, int &ra) -> bool {
        ra = w + NW * k;
        ca = 3 + lane;
        if (k < NK - 1 || ra < AH) return true;
        const int ri = (w - WR) * 64 + lane;
        if (ri >= RA) return false;
        ra = ri / 6;
        const int c = ri - 6 * ra;
        ca = c < 3 ? c : TW + c;
        return true;
    };

    // phase A: s_{t+1} on the tile + 3 ring
    const BufRes rr0 = buf_res(REC ? d.urec : nullptr, rbytes);
    auto finish_a = [&](int k, float (&f)[8], const CellRaw &raw, int ca, int ra, int64_t o) {
        if (REC) pend.flush(d, rr0);
        const Cell c = med.cell(d, raw);
        ck[k] = c;
        node_update<false>(d, c, f, g, ux, uy, n7, n8, dT);
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[(i * AH + ra) * AW + ca] = (float)(S)f[i];
        if (REC && ca >= 3 && ca < TW + 3 && ra >= 3 && ra < TH + 3 && x0 - 3 + ca < d.nx && y0 - 3 + ra < d.ny)
            pend.hold((uint32_t)(o * 4), ux, uy, n7, n8, dT);
    };
    if (interior) {
        // software pipelined: the next item's loads are issued before this one collides
        auto fetch = [&](int k, float (&f)[8], CellRaw &r, int &ca, int &ra) -> bool {
            if (!a_item(k, ca, ra)) return false;
            const int gx = x0 - 3 + ca, gy = y0 - 3 + ra;
            const uint32_t vo = (uint32_t)(((gy - 1) * d.pitch + (gx - 1)) * ES);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                f[i] = BufIO<S>::ld(rin, vo, (uint32_t)((i * d.plane + (1 - EY[i]) * d.pitch + (1 - EX[i])) * ES));
            r = med.load((uint32_t)((gy * d.pitch + gx) * 4));
            return true;
        };
        float fn[8];
        CellRaw rn{0.0f, 0.0f, 0.0f};
        int can = 0, ran = 0;
        bool vn = fetch(0, fn, rn, can, ran);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            float f[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = fn[i];
            const CellRaw r = rn;
            const int ca = can, ra = ran;
            const bool v = vn;
            if (k + 1 < NK) vn = fetch(k + 1, fn, rn, can, ran);
            if (v) finish_a(k, f, r, ca, ra, (int64_t)(y0 - 3 + ra) * d.pitch + (x0 - 3 + ca));
        }
    } else {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            int ca, ra;
            if (!a_item(k, ca, ra)) continue;
            int gx = x0 - 3 + ca, gy = y0 - 3 + ra;
            if (!wrap_node(d, gx, gy)) continue;
            float f[8];
            gather_general_buf<S>(d, rin, gx, gy, f);
            // a wrapped ring node is recorded by the tile that owns it
            const int64_t o = (int64_t)gy * d.pitch + gx;
            finish_a(k, f, med.load((uint32_t)(o * 4)), ca, ra, o);
        }
    }
    if (REC) pend.flush(d, rr0);
    lds_barrier();

    float fr[NK][8];
    int slot[NK];

    // phase B: s_{t+2} on the tile + 2 ring, kept in registers (no HBM loads on tile
    // rows, so the records are stored at once)
    const BufRes rr1 = buf_res(urec1, rbytes);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        slot[k] = -1;
        const int rb = w + NW * k - 1;
        int bx = 2 + lane, by = rb;
        const bool row = rb >= 0 && rb < BH;
        if (!row) {
            const int ri = (w - WR) * 64 + lane;
            if (k != NK - 1 || w < WR || ri >= RB) continue;
            by = ri >> 2;
            const int c = ri & 3;
            bx = c < 2 ? c : TW + c;
        }
        int gx = x0 - 2 + bx, gy = y0 - 2 + by;
        if (!interior && !wrap_node(d, gx, gy)) continue;
        const int64_t o = (int64_t)gy * d.pitch + gx;
        const Cell c = row ? ck[k] : med.cell(d, med.load((uint32_t)(o * 4)));
        lds_gather<AW, AH>(d, lds, interior, gx, gy, bx + 1, by + 1, fr[k]);
        node_update<false>(d, c, fr[k], g, ux, uy, n7, n8, dT);
        if (REC && bx >= 2 && bx < TW + 2 && by >= 2 && by < TH + 2 && x0 - 2 + bx < d.nx && y0 - 2 + by < d.ny)
            record_node(d, rr1, (uint32_t)(o * 4), ux, uy, n7, n8);
        slot[k] = by * BW + bx;
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        if (slot[k] < 0) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[i * BN + slot[k]] = (float)(S)fr[k][i];
    }
    lds_barrier();

    // phase C: s_{t+3} on the tile + 1 ring, kept in registers
    const BufRes rr2 = buf_res(urec2, rbytes);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        slot[k] = -1;
        const int rc = w + NW * k - 2;
        int cx = 1 + lane, cy = rc;
        const bool row = rc >= 0 && rc < CH;
        if (!row) {
            const int ri = (w - WR) * 64 + lane;
            if (k != NK - 1 || w < WR || ri >= RC) continue;
            cy = ri >> 1;
            cx = (ri & 1) ? CW - 1 : 0;
        }
        int gx = x0 - 1 + cx, gy = y0 - 1 + cy;
        if (!interior && !wrap_node(d, gx, gy)) continue;
        const int64_t o = (int64_t)gy * d.pitch + gx;
        const Cell c = row ? ck[k] : med.cell(d, med.load((uint32_t)(o * 4)));
        lds_gather<BW, BH>(d, lds, interior, gx, gy, cx + 1, cy + 1, fr[k]);
        node_update<false>(d, c, fr[k], g, ux, uy, n7, n8, dT);
        if (REC && cx >= 1 && cx < TW + 1 && cy >= 1 && cy < TH + 1 && x0 - 1 + cx < d.nx && y0 - 1 + cy < d.ny)
            record_node(d, rr2, (uint32_t)(o * 4), ux, uy, n7, n8);
        slot[k] = cy * CW + cx;
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        if (slot[k] < 0) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i) lds[i * CN + slot[k]] = (float)(S)fr[k][i];
    }
    lds_barrier();

    // phase D: s_{t+4} on the tile, to HBM
    const BufRes rr3 = buf_res(urec3, rbytes);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int rd = w + NW * k - 3;
        const int gx = x0 + lane, gy = y0 + rd;
        if (rd < 0 || rd >= TH || gx >= d.nx || gy >= d.ny) continue;
        float f[8];
        lds_gather<CW, CH>(d, lds, interior, gx, gy, lane + 1, rd + 1, f);
        node_update<false>(d, ck[k], f, g, ux, uy, n7, n8, dT);
        const int64_t o = (int64_t)gy * d.pitch + gx;
        const uint32_t vo = (uint32_t)(o * ES);
        // one branch for the whole store sequence (per-store branches split the stream)
        if (d.nt_store) {
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<S>::st_nt(rout, vo, (uint32_t)(i * d.plane * ES), f[i]);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) BufIO<S>::st(rout, vo, (uint32_t)(i * d.plane * ES), f[i]);
        }
        if (d.uprev) store_uprev(d, (uint32_t)(o * 4), ux, uy);
        if (REC) record_node(d, rr3, (uint32_t)(o * 4), ux, uy, n7, n8);
    }
}

template <typename S, int TW, int TH, int NT, int MK>
__global__ __launch_bounds__(NT) void k_step4(Dom d, int tiles_x, int swz) {
    __shared__ float lds[8 * (TH + 6) * (TW + 6)];
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    step4_tile<S, TW, TH, NT, false, MK>(d, (b % tiles_x) * TW, (b / tiles_x) * TH, nullptr, nullptr, nullptr, lds);
}

// The recording pass of the adjoint's recomputation (FP32), held to 80 VGPRs:
// six waves per SIMD, two workgroups per CU.
template <int TW, int TH, int NT, int MK>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6))) void k_step4_rec(
    Dom d, int tiles_x, int swz, float *urec1, float *urec2, float *urec3) {
    __shared__ float lds[8 * (TH + 6) * (TW + 6)];
    int b = blockIdx.x;
    if (swz) b = xcd_swizzle(b, gridDim.x);
    step4_tile<float, TW, TH, NT, true, MK>(d, (b % tiles_x) * TW, (b / tiles_x) * TH, urec1, urec2, urec3, lds);
}

// 64 x 26 tiles with 768 threads (12 waves: 8 with three frame rows, 4 with
// two plus the ring columns): 72 KB of LDS, two workgroups per CU. Per
// workgroup 2240 + 2040 + 1848 + 1664 collisions for 6656 updates (1.171, against
// 1.106 for three cycles on 64 x 28), and phase A reads a 70 x 32 frame per
// 64 x 26 tile for four cycles instead of a 68 x 32 frame per 64 x 28 for three.
constexpr int STEP4_TW = 64, STEP4_TH = 26, STEP4_NT = 768;

void step4_tiles(const Dom &d, int *tiles_x, int *tiles_y) {
    *tiles_x = (d.nx + STEP4_TW - 1) / STEP4_TW;
    *tiles_y = (d.ny + STEP4_TH - 1) / STEP4_TH;
}

int step4_threads() { return STEP4_NT; }

int step4_rows() { return STEP4_TH; }

// Batched four-cycle pass over a table of 64 x 26 tiles (isothermal domains;
// MK_BRANCHED for any medium, MK_UNIFORM when every domain is uniform), one
// workgroup per tile. (Workgroups walking runs of tiles, as the three-cycle
// batch offers, spill 42-44 VGPRs at two workgroups per CU and are not built.)
template <typename S, int MK>
__global__ __launch_bounds__(STEP4_NT) __attribute__((amdgpu_waves_per_eu(6))) void k_step4_batch(
    const Dom *__restrict__ doms, const int4 *__restrict__ tiles, int parity) {
    __shared__ float lds[8 * (STEP4_TH + 6) * (STEP4_TW + 6)];
    const int4 tl = tiles[blockIdx.x];
    const Dom d = doms[2 * tl.x + parity];
    step4_tile<S, STEP4_TW, STEP4_TH, STEP4_NT, false, MK>(d, tl.y * STEP4_TW, tl.z * STEP4_TH, nullptr, nullptr,
                                                          nullptr, lds);
}

template <int MK>
static const void *step4_batch_fn_mk(int storage) {
    return storage == ST_F32 ? (const void *)&k_step4_batch<float, MK> : (const void *)&k_step4_batch<_Float16, MK>;
}

const void *step4_batch_kernel_fn(int storage, bool uniform) {
    return uniform ? step4_batch_fn_mk<MK_UNIFORM>(storage) : step4_batch_fn_mk<MK_BRANCHED>(storage);
}

hipError_t launch_step4_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity, int storage, bool uniform,
                              hipStream_t st) {
    if (ntiles <= 0) return hipErrorInvalidValue;
    const void *fn = step4_batch_kernel_fn(storage, uniform);
    void *args[3] = {&doms, &tiles, &parity};
    return hipLaunchKernel(fn, dim3((unsigned)ntiles), dim3(STEP4_NT), args, 0, st);
}

template <int MK>
static const void *step4_fn_t(int storage) {
    return storage == ST_F32 ? (const void *)&k_step4<float, STEP4_TW, STEP4_TH, STEP4_NT, MK>
                             : (const void *)&k_step4<_Float16, STEP4_TW, STEP4_TH, STEP4_NT, MK>;
}

const void *step4_kernel_fn(const Dom &d, int storage) {
    if (d.thermal) return nullptr;
    switch (medium_kind(d)) {
    case MK_ERGUN: return step4_fn_t<MK_ERGUN>(storage);
    case MK_UNIFORM: return step4_fn_t<MK_UNIFORM>(storage);
    default: return step4_fn_t<MK_ANY>(storage);
    }
}

hipError_t launch_step4(const Dom &d, int storage, int swizzle, hipStream_t st) {
    const void *fn = step4_kernel_fn(d, storage);
    if (!fn) return hipErrorInvalidValue;
    int tx, ty;
    step4_tiles(d, &tx, &ty);
    Dom dd = d;
    int swz = swizzle;
    void *args[3] = {&dd, &tx, &swz};
    return hipLaunchKernel(fn, dim3((unsigned)(tx * ty)), dim3((unsigned)STEP4_NT), args, 0, st);
}

hipError_t launch_step4_rec(const Dom &d, int swizzle, float *urec1, float *urec2, float *urec3, hipStream_t st) {
    if (d.thermal || !d.urec || !urec1 || !urec2 || !urec3) return hipErrorInvalidValue;
    const void *fn;
    switch (medium_kind(d)) {
    case MK_ERGUN: fn = (const void *)&k_step4_rec<STEP4_TW, STEP4_TH, STEP4_NT, MK_ERGUN>; break;
    case MK_UNIFORM: fn = (const void *)&k_step4_rec<STEP4_TW, STEP4_TH, STEP4_NT, MK_UNIFORM>; break;
    default: fn = (const void *)&k_step4_rec<STEP4_TW, STEP4_TH, STEP4_NT, MK_ANY>; break;
    }
    int tx, ty;
    step4_tiles(d, &tx, &ty);
    Dom dd = d;
    int swz = swizzle;
    void *args[6] = {&dd, &tx, &swz, &urec1, &urec2, &urec3};
    return hipLaunchKernel(fn, dim3((unsigned)(tx * ty)), dim3((unsigned)STEP4_NT), args, 0, st);
}

template <typename S, bool REC, int MK, bool THERMAL>
static const void *step2_fn_t(int threads, int rows) {
#define MRT_S2FN(N, H) if (threads == N && rows == H) return (const void *)&k_step2<S, STEP2_TW, H, N, REC, MK, THERMAL>;
    MRT_STEP2_SHAPES(MRT_S2FN)
#undef MRT_S2FN
    return nullptr;
}

template <typename S, int MK, bool THERMAL, bool ONE>
static const void *step2_batch_fn_t(int threads, int rows) {
#define MRT_S2BFN(N, H) if (threads == N && rows == H) return (const void *)&k_step2_batch<S, STEP2_TW, H, N, MK, THERMAL, ONE>;
    MRT_STEP2_SHAPES(MRT_S2BFN)
#undef MRT_S2BFN
    return nullptr;
}

template <int MK, bool ONE>
static const void *step2_batch_fn_mk(int storage, bool thermal, int threads, int rows) {
    if (thermal)
        return storage == ST_F32 ? step2_batch_fn_t<float, MK, true, ONE>(threads, rows)
                                 : step2_batch_fn_t<_Float16, MK, true, ONE>(threads, rows);
    return storage == ST_F32 ? step2_batch_fn_t<float, MK, false, ONE>(threads, rows)
                             : step2_batch_fn_t<_Float16, MK, false, ONE>(threads, rows);
}

const void *step2_batch_kernel_fn(int storage, bool thermal, bool uniform, bool one, int threads, int rows) {
    if (one)
        return uniform ? step2_batch_fn_mk<MK_UNIFORM, true>(storage, thermal, threads, rows)
                       : step2_batch_fn_mk<MK_BRANCHED, true>(storage, thermal, threads, rows);
    return uniform ? step2_batch_fn_mk<MK_UNIFORM, false>(storage, thermal, threads, rows)
                   : step2_batch_fn_mk<MK_BRANCHED, false>(storage, thermal, threads, rows);
}

hipError_t launch_step2_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity, int storage,
                              bool thermal, bool uniform, int threads, int rows, int grid, hipStream_t st) {
    if (grid <= 0 || ntiles <= 0) return hipErrorInvalidValue;
    if (grid > ntiles) grid = ntiles;   // workgroups beyond the last tile would idle
    const void *fn = step2_batch_kernel_fn(storage, thermal, uniform, grid == ntiles, threads, rows);
    if (!fn) return hipErrorInvalidValue;
    void *args[4] = {&doms, &tiles, &ntiles, &parity};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3((unsigned)threads), args, 0, st);
}

template <int MK>
static const void *step2_fn_mk(int storage, int threads, int rows, bool rec, bool thermal) {
    if (thermal) {
        if (rec) return storage == ST_F32 ? step2_fn_t<float, true, MK, true>(threads, rows) : nullptr;
        return storage == ST_F32 ? step2_fn_t<float, false, MK, true>(threads, rows)
                                 : step2_fn_t<_Float16, false, MK, true>(threads, rows);
    }
    if (storage == ST_F32)
        return rec ? step2_fn_t<float, true, MK, false>(threads, rows) : step2_fn_t<float, false, MK, false>(threads, rows);
    return rec ? nullptr : step2_fn_t<_Float16, false, MK, false>(threads, rows);
}

const void *step2_kernel_fn(const Dom &d, int storage, int threads, int rows, bool rec) {
    const bool th = d.thermal != 0;
    switch (medium_kind(d)) {
    case MK_ERGUN: return step2_fn_mk<MK_ERGUN>(storage, threads, rows, rec, th);
    case MK_UNIFORM: return step2_fn_mk<MK_UNIFORM>(storage, threads, rows, rec, th);
    default: return step2_fn_mk<MK_BRANCHED>(storage, threads, rows, rec, th);
    }
}

hipError_t launch_step2(const Dom &d, int storage, int swizzle, int threads, int rows,
                        float *urec_next, hipStream_t st) {
    const bool rec = urec_next != nullptr;
    const void *fn = step2_kernel_fn(d, storage, threads, rows, rec);
    if (!fn || (rec && !d.urec)) return hipErrorInvalidValue;
    int tx, ty;
    step2_tiles(d.nx, d.ny, rows, &tx, &ty);
    Dom dd = d;
    int swz = swizzle;
    void *args[4] = {&dd, &tx, &swz, &urec_next};
    return hipLaunchKernel(fn, dim3((unsigned)(tx * ty)), dim3((unsigned)threads), args, 0, st);
}

// --------------------------------------------------------- node readers

// f(t) (and g(t)) of node (x, y) from a state buffer in the given layout.
template <typename S, bool THERMAL>
__device__ __forceinline__ void read_state(const Dom &d, int src, int x, int y, float f[8],
                                           float g[5]) {
    if (src == SRC_DIRECT) {
        load_own<S>(d, (const S *)d.fin, x, y, f);
        if (THERMAL) load_own_thermal(d, d.gin, x, y, g);
    } else {
        gather_general<S>(d, (const S *)d.fin, x, y, f);
        if (THERMAL) gather_thermal(d, d.gin, x, y, false, g);
        nee_fixup<S, THERMAL>(d, (const S *)d.fin, x, y, f, g);
    }
}

// f(t) of a node one link or more from every edge of a gather-layout state
// below 4 GiB: pulled at constant per-link offsets through a buffer resource
// (no wrap, wall or extrapolation can reach it).
template <typename S>
__device__ __forceinline__ void gather_inner(const Dom &d, const BufRes &r, int x, int y, float f[8]) {
    constexpr int ES = (int)sizeof(S);
    const uint32_t vo = (uint32_t)(((y - 1) * d.pitch + (x - 1)) * ES);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        f[i] = BufIO<S>::ld(r, vo, (uint32_t)((i * d.plane + (1 - EY[i]) * d.pitch + (1 - EX[i])) * ES));
}

// whether an output kernel may take gather_inner for a state: the pull layout of
// an isothermal domain whose population buffer is below 4 GiB
template <typename S, bool THERMAL>
__device__ __forceinline__ bool inner_gather_ok(const Dom &d, int src) {
    return !THERMAL && src == SRC_GATHER && (uint64_t)8 * (uint64_t)d.plane * sizeof(S) < ((uint64_t)1 << 32);
}

// velocity of node (x, y) at the state's time, as the step computes it
template <bool THERMAL>
__device__ __forceinline__ void state_velocity_c(const Dom &d, const Cell &c, const float f[8],
                                                 const float g[5], float &ux, float &uy,
                                                 float &m1, float &dT) {
    float ayh = d.ayh;
    dT = 0.0f;
    if (THERMAL) {
        dT = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
        ayh = d.ayh + d.gbetah * dT;
    }
    node_velocity_h(f, c, c.phi * d.axh, c.phi * ayh, ux, uy, m1);
}

template <bool THERMAL>
__device__ __forceinline__ void state_velocity(const Dom &d, int64_t o, const float f[8],
                                               const float g[5], float &ux, float &uy,
                                               float &m1, float &dT) {
    state_velocity_c<THERMAL>(d, load_cell(d, o), f, g, ux, uy, m1, dT);
}

// A workgroup covers BLOCK consecutive nodes of row y; blocks one node or more
// from every edge gather through gather_inner.
template <typename S, bool THERMAL>
__global__ __launch_bounds__(BLOCK) void k_macro(Dom d, int src, float Pi0, float *p, float *ux,
                                                 float *uy, float *T) {
    const int xb = blockIdx.x * BLOCK, x = xb + threadIdx.x, y = blockIdx.y;
    const bool ok = inner_gather_ok<S, THERMAL>(d, src);
    const BufRes rin = buf_res(d.fin, ok ? (uint32_t)(8 * d.plane * (int64_t)sizeof(S)) : 0u);
    float f[8], g[5];
    if (ok && y >= 1 && y <= d.ny - 2 && xb >= 1 && xb + BLOCK <= d.nx - 1) {
        gather_inner<S>(d, rin, x, y, f);
    } else {
        if (x >= d.nx) return;
        read_state<S, THERMAL>(d, src, x, y, f, g);
    }
    const int64_t o = (int64_t)y * d.pitch + x;
    const Cell c = load_cell(d, o);
    float u, v, m1, dT;
    state_velocity_c<THERMAL>(d, c, f, g, u, v, m1, dT);
    const int64_t q = (int64_t)y * d.nx + x;
    if (ux) ux[q] = u;
    if (uy) uy[q] = v;
    if (p) {
        // Eq. (20): phi p = (3/5)(m1 - (2/3)|u|^2/phi), m1 = (5/3) Pi0 + dm1
        const float Pi = Pi0 + (mulc(m1, MRT_C3_5) - mulc((u * u + v * v) * c.inv_phi, MRT_C2_5));
        p[q] = Pi * c.inv_phi;
    }
    if (T) T[q] = d.T0 + dT;
}

template <typename S, bool THERMAL>
static hipError_t macro_t(const Dom &d, Source src, float Pi0, float *p, float *ux, float *uy,
                          float *T, hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + BLOCK - 1) / BLOCK), (unsigned)d.ny);
    hipLaunchKernelGGL((k_macro<S, THERMAL>), grid, dim3(BLOCK), 0, st, d, (int)src, Pi0, p, ux,
                       uy, T);
    return hipGetLastError();
}

hipError_t launch_macroscopic(const Dom &d, int storage, Source src, float Pi0, float *p,
                              float *ux, float *uy, float *T, hipStream_t st) {
    const bool th = d.thermal != 0;
    if (storage == ST_F32)
        return th ? macro_t<float, true>(d, src, Pi0, p, ux, uy, T, st)
                  : macro_t<float, false>(d, src, Pi0, p, ux, uy, T, st);
    return th ? macro_t<_Float16, true>(d, src, Pi0, p, ux, uy, T, st)
              : macro_t<_Float16, false>(d, src, Pi0, p, ux, uy, T, st);
}

template <typename S, bool THERMAL>
__global__ __launch_bounds__(BLOCK) void k_get_pop(Dom d, int src, float *df, float *dg) {
    const int x = blockIdx.x * BLOCK + threadIdx.x, y = blockIdx.y;
    if (x >= d.nx) return;
    float f[8], g[5];
    read_state<S, THERMAL>(d, src, x, y, f, g);
    const int64_t n = (int64_t)d.nx * d.ny, q = (int64_t)y * d.nx + x;
#pragma unroll
    for (int i = 0; i < 8; ++i) df[i * n + q] = f[i];
    if (THERMAL && dg) {
#pragma unroll
        for (int j = 0; j < 5; ++j) dg[j * n + q] = g[j];
    }
}

template <typename S>
__global__ __launch_bounds__(BLOCK) void k_set_pop(Dom d, const float *df, const float *dg) {
    const int x = blockIdx.x * BLOCK + threadIdx.x, y = blockIdx.y;
    if (x >= d.nx) return;
    const int64_t n = (int64_t)d.nx * d.ny, q = (int64_t)y * d.nx + x;
    const int64_t o = (int64_t)y * d.pitch + x;
    S *fo = (S *)d.fout;
#pragma unroll
    for (int i = 0; i < 8; ++i) Store<S>::st(fo + i * d.plane + o, df[i * n + q]);
    if (d.thermal) {
#pragma unroll
        for (int j = 0; j < 5; ++j) d.gout[j * d.plane + o] = dg ? dg[j * n + q] : 0.0f;
    }
}

hipError_t launch_get_populations(const Dom &d, int storage, Source src, float *df,
                                  float *dg, hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + BLOCK - 1) / BLOCK), (unsigned)d.ny);
    const bool th = d.thermal != 0;
    if (storage == ST_F32) {
        if (th) hipLaunchKernelGGL((k_get_pop<float, true>), grid, dim3(BLOCK), 0, st, d, (int)src, df, dg);
        else hipLaunchKernelGGL((k_get_pop<float, false>), grid, dim3(BLOCK), 0, st, d, (int)src, df, dg);
    } else {
        if (th) hipLaunchKernelGGL((k_get_pop<_Float16, true>), grid, dim3(BLOCK), 0, st, d, (int)src, df, dg);
        else hipLaunchKernelGGL((k_get_pop<_Float16, false>), grid, dim3(BLOCK), 0, st, d, (int)src, df, dg);
    }
    return hipGetLastError();
}

hipError_t launch_set_populations(const Dom &d, int storage, const float *df, const float *dg,
                                  hipStream_t st) {
    const dim3 grid((unsigned)((d.nx + BLOCK - 1) / BLOCK), (unsigned)d.ny);
    if (storage == ST_F32) hipLaunchKernelGGL((k_set_pop<float>), grid, dim3(BLOCK), 0, st, d, df, dg);
    else hipLaunchKernelGGL((k_set_pop<_Float16>), grid, dim3(BLOCK), 0, st, d, df, dg);
    return hipGetLastError();
}

__global__ __launch_bounds__(BLOCK) void k_fill_zero(uint4 *p, size_t n16) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * BLOCK)
        p[i] = z;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)p & 15) || (bytes & 15)) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + BLOCK - 1) / BLOCK;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(BLOCK), 0, st, (uint4 *)p, n16);
    return hipGetLastError();
}

// Per-node s_nu = 1 / (1/2 + 3 J nu) (Eq. 21, cs^2 = 1/3) from a [ny][nx]
// plane of viscosity ratios J (or the constant J0 where J is NULL), in double
// and rounded once, so a plane of constant J holds the uniform rate exactly.
// With `bad` set the kernel only checks: any J that is not finite and > 0
// stores 1 there (every such thread stores the same value), and out is untouched.
__global__ __launch_bounds__(BLOCK) void k_snu_plane(const float *J, double J0, double nu,
                                                     float *out, int pitch, int nx, int *bad) {
    const int x = blockIdx.x * BLOCK + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const double j = J ? (double)J[(int64_t)y * nx + x] : J0;
    if (bad) {
        if (!(j > 0.0 && j <= 3.4e38)) *bad = 1;
        return;
    }
    const double tau = 0.5 + 3.0 * j * nu;
    out[(int64_t)y * pitch + x] = (float)(1.0 / tau);
}

hipError_t launch_snu_plane(const float *J, double J0, double nu, float *out, int pitch, int nx,
                            int ny, int *bad, hipStream_t st) {
    const dim3 grid((unsigned)((nx + BLOCK - 1) / BLOCK), (unsigned)ny);
    hipLaunchKernelGGL(k_snu_plane, grid, dim3(BLOCK), 0, st, J, J0, nu, out, pitch, nx, bad);
    return hipGetLastError();
}

__global__ __launch_bounds__(BLOCK) void k_unpitch(const float *src, int pitch, float *dst,
                                                   int nx, int ny) {
    const int x = blockIdx.x * BLOCK + threadIdx.x, y = blockIdx.y;
    if (x < nx) dst[(int64_t)y * nx + x] = src[(int64_t)y * pitch + x];
}

hipError_t launch_unpitch(const float *src, int pitch, float *dst, int nx, int ny,
                          hipStream_t st) {
    const dim3 grid((unsigned)((nx + BLOCK - 1) / BLOCK), (unsigned)ny);
    hipLaunchKernelGGL(k_unpitch, grid, dim3(BLOCK), 0, st, src, pitch, dst, nx, ny);
    return hipGetLastError();
}

// ------------------------------------------------------------ reductions

// Fixed-order block reduction of three doubles (wavefront butterfly, then
// the four wavefront results in order). Bitwise reproducible for a given
// assignment of values to threads.
__device__ __forceinline__ void block_sum3(double v[3], double *out) {
    __shared__ double sh[BLOCK / 64][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double a = v[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
        v[k] = a;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[w][0] = v[0]; sh[w][1] = v[1]; sh[w][2] = v[2];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int j = 0; j < BLOCK / 64; ++j) s += sh[j][k];
            out[k] = s;
        }
    }
}

int reduce_blocks(int nx, int ny) {
    const int64_t n = (int64_t)nx * ny;
    int64_t b = (n + BLOCK - 1) / BLOCK;
    if (b > 4096) b = 4096;
    return (int)b;
}

template <typename S, bool THERMAL>
__global__ __launch_bounds__(BLOCK) void k_reduce(Dom cur, int src_cur, const float *uprev,
                                                  double *partials) {
    // at most 2^31 nodes, so node numbers and the stride stay below 2^32
    const uint32_t n = (uint32_t)cur.nx * (uint32_t)cur.ny, nx = (uint32_t)cur.nx;
    double acc[3] = {0.0, 0.0, 0.0};
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK) {
        const int x = (int)(k % nx), y = (int)(k / nx);
        const int64_t o = (int64_t)y * cur.pitch + x;
        float f[8], g[5];
        read_state<S, THERMAL>(cur, src_cur, x, y, f, g);
        float ux, uy, m1, dT;
        state_velocity<THERMAL>(cur, o, f, g, ux, uy, m1, dT);
        acc[0] += (double)m1;
        acc[2] += (double)ux * ux + (double)uy * uy;
        if (uprev) {
            // u(t - 1) as the last collision of the previous pass computed it
            const float px = uprev[o], py = uprev[cur.plane + o];
            const double dx = (double)ux - px, dy = (double)uy - py;
            acc[1] += dx * dx + dy * dy;
        }
    }
    block_sum3(acc, partials + 3 * blockIdx.x);
}

__global__ __launch_bounds__(BLOCK) void k_reduce_final(const double *partials, int nb,
                                                        double *result) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < nb; j += BLOCK) {
        acc[0] += partials[3 * j + 0];
        acc[1] += partials[3 * j + 1];
        acc[2] += partials[3 * j + 2];
    }
    block_sum3(acc, result);
}

hipError_t launch_reduce(const Dom &cur, Source src_cur, const float *uprev, int storage, double *partials,
                         double *result, hipStream_t st) {
    const int nb = reduce_blocks(cur.nx, cur.ny);
    const bool th = cur.thermal != 0;
    if (storage == ST_F32) {
        if (th) hipLaunchKernelGGL((k_reduce<float, true>), dim3(nb), dim3(BLOCK), 0, st, cur, (int)src_cur, uprev, partials);
        else hipLaunchKernelGGL((k_reduce<float, false>), dim3(nb), dim3(BLOCK), 0, st, cur, (int)src_cur, uprev, partials);
    } else {
        if (th) hipLaunchKernelGGL((k_reduce<_Float16, true>), dim3(nb), dim3(BLOCK), 0, st, cur, (int)src_cur, uprev, partials);
        else hipLaunchKernelGGL((k_reduce<_Float16, false>), dim3(nb), dim3(BLOCK), 0, st, cur, (int)src_cur, uprev, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, st, partials, nb, result);
    return hipGetLastError();
}

}  // namespace mrt
