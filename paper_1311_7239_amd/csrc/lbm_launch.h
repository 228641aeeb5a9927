// Host-side launch interface between the C ABI (lbm_abi.cpp) and the HIP
// kernels (lbm_kernels.hip). Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace mrt {

enum Storage { ST_F32 = 0, ST_F16 = 1 };

// How a kernel obtains f(t) from a state buffer: by pulling from the
// neighbours (the buffer holds post-collision f+(t-1)), or directly (the
// buffer holds f(0) itself, which is the layout at t = 0).
enum Source { SRC_GATHER = 0, SRC_DIRECT = 1, SRC_NONE = 2 };

struct Schedule {
    int tile_w;  // threads of a 256-thread block along x
    int vec;     // consecutive nodes per thread along x (1, 2 or 4)
    int rows;    // rows per thread
    int swizzle; // map consecutive tiles onto the same XCD
};

// Number of 256-thread tiles covering the domain with a schedule.
void tile_counts(const Schedule &s, int nx, int ny, int *tiles_x, int *tiles_y);
bool schedule_supported(const Schedule &s);

// One collide-and-stream cycle of one domain: reads d.fin (and d.gin),
// writes d.fout (and d.gout); records u(t) into d.urec when rec.
hipError_t launch_step(const Dom &d, int storage, Source src, bool rec, const Schedule &s,
                       hipStream_t st);

// Two cycles in one pass (temporal blocking): reads s_t from d.fin, writes
// s_{t+2} to d.fout; isothermal, gather layout only. With urec_next non-null
// (FP32 only) it also records u(t) into d.urec and u(t+1) into urec_next.
// Tiles are 64 wide and `rows` tall, run by `threads` threads. Kernel entry
// arguments: (Dom, int tiles_x, int swizzle, float *urec_next).
hipError_t launch_step2(const Dom &d, int storage, int swizzle, int threads, int rows,
                        float *urec_next, hipStream_t st);
bool step2_shape_supported(int threads, int rows);
void step2_tiles(int nx, int ny, int rows, int *tiles_x, int *tiles_y);
const void *step2_kernel_fn(const Dom &d, int storage, int threads, int rows, bool rec);
// Three collide-stream cycles in one HBM pass (64-wide tiles; step3_tiles and
// step3_single_threads give the grid and the workgroup size; kernel arguments
// (Dom, int tiles_x, int swizzle, float *urec1, float *urec2)).
// With urec1/urec2 (FP32 only) the pass records at t (d.urec), t + 1, t + 2.
hipError_t launch_step3(const Dom &d, int storage, int swizzle, float *urec1, float *urec2, hipStream_t st);
// grid and workgroup size of launch_step3 for a domain, with or without recording
void step3_tiles(const Dom &d, bool rec, int *tiles_x, int *tiles_y);
int step3_single_threads(const Dom &d, bool rec);
int step3_single_rows(const Dom &d, bool rec);
const void *step3_kernel_fn(const Dom &d, int storage, bool rec);
// Four collide-stream cycles in one HBM pass (single isothermal domains, no
// recording; 64 x 26 tiles, step4_threads() threads; kernel arguments
// (Dom, tiles_x, swizzle)). step4_kernel_fn is null for a thermal domain.
hipError_t launch_step4(const Dom &d, int storage, int swizzle, hipStream_t st);
void step4_tiles(const Dom &d, int *tiles_x, int *tiles_y);
int step4_threads();
int step4_rows();
const void *step4_kernel_fn(const Dom &d, int storage);
// the four-cycle pass recording u (and with d.rec_stress the stress moments) at
// t (d.urec), t + 1, t + 2, t + 3 (FP32 isothermal domains; same grid)
hipError_t launch_step4_rec(const Dom &d, int swizzle, float *urec1, float *urec2, float *urec3, hipStream_t st);
// batched four-cycle pass over a table of 64 x 26 tiles (isothermal domains),
// one workgroup per tile (a grid of ntiles; kernel arguments (doms, tiles,
// parity)); uniform as for the three-cycle batch
const void *step4_batch_kernel_fn(int storage, bool uniform);
hipError_t launch_step4_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity, int storage, bool uniform,
                              hipStream_t st);
// batched three-cycle pass over a table of 64 x 16 tiles (isothermal domains);
// uniform: every domain has a uniform medium and one s_nu (medium_kind MK_UNIFORM),
// so the kernel loads no medium planes; one: one workgroup per tile (a grid of
// exactly ntiles), else workgroups walk runs of tiles. The launchers clamp the
// grid to ntiles and pick one = (grid == ntiles).
const void *step3_batch_kernel_fn(int storage, bool uniform, bool one);
int step3_threads();
hipError_t launch_step3_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity, int storage, bool uniform,
                              int grid, hipStream_t st);
// Batched two-cycle pass over a table of 64 x rows tiles (domain, tx, ty, 0);
// entry arguments (const Dom*, const int4*, int ntiles, int parity); uniform as above.
hipError_t launch_step2_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity, int storage,
                              bool thermal, bool uniform, int threads, int rows, int grid, hipStream_t st);
const void *step2_batch_kernel_fn(int storage, bool thermal, bool uniform, bool one, int threads, int rows);

// Persistent batched step over a tile table: doms[2*k + parity] describes
// domain k with its buffers for this parity; tiles[j] = (domain, tx, ty, 0).
// thermal: every domain of the table carries the D2Q5 field (or none does).
hipError_t launch_step_batch(const Dom *doms, const int4 *tiles, int ntiles, int parity,
                             int storage, bool thermal, const Schedule &s, int grid, hipStream_t st);

// Kernel entry points for building HIP graphs by hand (gather-layout step of
// one domain: arguments (Dom, int tiles_x, int swizzle); batched step:
// arguments (const Dom*, const int4*, int ntiles, int parity)).
const void *step_kernel_fn(int storage, bool thermal, const Schedule &s);
const void *batch_kernel_fn(int storage, bool thermal, const Schedule &s);

hipError_t launch_macroscopic(const Dom &d, int storage, Source src, float Pi0, float *p,
                              float *ux, float *uy, float *T, hipStream_t st);
hipError_t launch_get_populations(const Dom &d, int storage, Source src, float *df,
                                  float *dg, hipStream_t st);
hipError_t launch_set_populations(const Dom &d, int storage, const float *df,
                                  const float *dg, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);

// FP64 reductions: partial sums (sum dm1, sum |u - u_prev|^2, sum |u|^2) per
// block, then one fixed-order pass into result[3]. u_prev comes from the two
// planes uprev ([ny][pitch] u_x then u_y, recorded by the last pass); with
// uprev NULL the second sum is 0.
int reduce_blocks(int nx, int ny);
hipError_t launch_reduce(const Dom &cur, Source src_cur, const float *uprev, int storage, double *partials,
                         double *result, hipStream_t st);

// Discrete adjoint pieces (FP32 storage, isothermal). acc (may be NULL):
// per-workgroup FP64 slots of 4 (nu, a_x, a_y, U_lid) to which each launch
// adds its share of the parameter gradients; with acc, the u record carries
// the stress moments in planes 2 and 3.
// Seed: lam(T) = (du/df)^T dL/du and g_phi = (du/dphi)^T dL/du at time T.
hipError_t launch_adjoint_seed(const Dom &d, Source src, const float *dLdu, float *lam,
                               float *gphi, float *gkappa, double *acc, hipStream_t st);
// One backward step: lam_out = J(t)^T G^T lam_in, g += (dC/dphi)^T G^T lam_in,
// using u(t) from urec.
hipError_t launch_adjoint_step(const Dom &d, const float *lam_in, float *lam_out,
                               const float *u_t, float *gphi, float *gkappa, double *acc, hipStream_t st);
// Two backward steps per pass: lam_out = a(t-1) from lam_in = a(t+1), using
// u(t) and u(t-1).
hipError_t launch_adjoint_step2(const Dom &d, const float *lam_in, float *lam_out, const float *u_t,
                                const float *u_tm1, float *gphi, float *gkappa, double *acc, hipStream_t st);
hipError_t launch_adjoint_step2_thermal(const Dom &d, const float *lam_in, float *lam_out, const float *lamg_in,
                                        float *lamg_out, const float *u_t, const float *u_tm1, float *gphi,
                                        float *gkappa, double *acc, hipStream_t st);
hipError_t launch_adjoint_step3(const Dom &d, const float *lam_in, float *lam_out, const float *u_t,
                                const float *u_tm1, const float *u_tm2, float *gphi, float *gkappa, double *acc,
                                hipStream_t st);
// The coupled D2Q8 + D2Q5 adjoint (one step per pass): lamg holds the
// adjoint of the thermal populations (5 planes); u_t carries dT in plane 4.
hipError_t launch_adjoint_seed_thermal(const Dom &d, Source src, const float *dLdu, float *lam, float *lamg,
                                       float *gphi, float *gkappa, double *acc, hipStream_t st);
hipError_t launch_adjoint_step_thermal(const Dom &d, const float *lam_in, float *lam_out, const float *lamg_in,
                                       float *lamg_out, const float *u_t, float *gphi, float *gkappa, double *acc,
                                       hipStream_t st);
// Slots of 4 doubles the three adjoint kernels use for a domain (seed, step,
// two-step regions, in that order) and the first slot of each region.
int64_t adjoint_theta_slots(int nx, int ny);
int64_t adjoint_theta_offset(int nx, int ny, int which);
// Tangent-linear (forward mode): one cycle of the state (d) and its tangent
// (dt: the tangent buffers, lid6 = dU/6), and the tangent of u at the
// state's time into du [2][ny][nx].
hipError_t launch_tangent_step(const Dom &d, const Dom &dt, Source src, const float *dphi, float dnu,
                               float dax, float day, hipStream_t st);
hipError_t launch_tangent_u(const Dom &d, const Dom &dt, Source src, const float *dphi, float dnu, float dax,
                            float day, float *du, hipStream_t st);
// out[0..3] = the sum of n slots, in a fixed order.
hipError_t launch_theta_final(const double *slots, int64_t n, double *out, hipStream_t st);
hipError_t launch_snu_plane(const float *J, double J0, double nu, float *out, int pitch, int nx,
                            int ny, int *bad, hipStream_t st);
hipError_t launch_unpitch(const float *src, int pitch, float *dst, int nx, int ny,
                          hipStream_t st);

}  // namespace mrt
