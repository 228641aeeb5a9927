/*
 * mrtlbm: C ABI of the GPU (gfx950) implementation of the D2Q8 porous
 * multiple-relaxation-time lattice Boltzmann scheme of Liu & He,
 * "Multiple-relaxation-time lattice Boltzmann modeling of incompressible
 * flows in porous media" (arXiv:1311.7239), with the D2Q5 MRT thermal model
 * of its Appendix B.
 *
 * Model (Sec. 2): generalized Brinkman-Forchheimer-extended Darcy flow,
 * Eqs. (1)-(3); D2Q8 velocities (Eq. 7), moment transform M (Eq. 10),
 * porosity-dependent equilibrium moments (Eqs. 11-12), relaxation
 * diag(1, s_e, 1, s_q, 1, s_q, s_nu, s_nu) (Eq. 13) with s_nu = 1/tau and
 * tau = 1/2 + 3 J nu (Eq. 21), moment-space forcing (Eq. 16) carrying the
 * Darcy and Forchheimer drag of Eq. (3), explicit velocity (Eqs. 18-19),
 * pressure (Eq. 20), collision (Eq. 14) and streaming (Eq. 15).
 * Units: lattice units, delta_x = delta_t = c = 1, rho0 = 1.
 *
 * Conventions shared by every entry point:
 *   - Grids are row-major [y][x] with x fastest; node (x, y) is the cell
 *     centre (x + 1/2, y + 1/2). Walls sit half a link outside the edge
 *     nodes (x = 0 and x = nx, y = 0 and y = ny).
 *   - Every array argument is DEVICE memory unless marked "host". The
 *     library never allocates device memory: the caller passes a workspace
 *     of at least the size lbm_workspace_size() reports, keeps it alive and
 *     unshared while the context exists, and owns every output buffer.
 *   - Work is enqueued asynchronously on the HIP stream given at creation.
 *     Only lbm_reduce, lbm_save and lbm_load synchronise that stream.
 *   - Time t counts completed collide-and-stream cycles; "the state at t"
 *     is the pre-collision populations f(t) of Eq. (15).
 *   - Populations are stored as deviations from the rest state
 *     f_ref_i = 3 w_i Pi0 (Eq. 22 at u = 0 with phi p = Pi0), w = 1/9 on
 *     axis links and 1/36 on diagonal links; thermal populations as
 *     deviations from w_T T0 with w_T = (4 + varpi)/20 (App. B, varpi = 0).
 *   - Every function returns LBM_OK (0) or a negative status; a failed call
 *     has no side effect unless it returns LBM_EDEVICE, after which the
 *     context is poisoned. No function prints, aborts or throws.
 *   - A context is not thread-safe. Handles are checked against the set of
 *     live contexts (see lbm_destroy).
 */
#ifndef MRTLBM_LBM_H
#define MRTLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument or descriptor             */
#define LBM_ESTATE (-2)    /* call not valid in the context's state      */
#define LBM_EDEVICE (-3)   /* a HIP call failed; the context is poisoned */
#define LBM_EUNSTABLE (-4) /* non-finite mass or residual                */
#define LBM_ENOTSUP (-5)   /* combination not supported                  */

/* boundary kinds per axis */
#define LBM_PERIODIC 0
#define LBM_WALLS 1 /* halfway bounce-back; top wall y = ny moves at lid_ux */
/* On-node walls with non-equilibrium extrapolation, the paper's default wall
 * treatment (Sec. 3, its Ref. [40]): the first and last node of the axis lie
 * on the walls (so a side L holds L + 1 nodes) and every population of a
 * wall node is rebuilt each step as f^eq(phi p of the inner neighbour B,
 * wall velocity) + f(B) - f^eq(state of B), f^eq from Eq. (22); the top row
 * moves at lid_ux except at on-node x walls. Thermal: x walls are Dirichlet
 * (Th at x = 0, Tc at x = nx - 1), y walls adiabatic (T of B). Needs >= 3
 * nodes on the axis; the other axis is periodic or on-node (mixing with
 * LBM_WALLS gives ENOTSUP). Such contexts advance one cycle per pass and
 * have no adjoint or tangent (ENOTSUP). */
#define LBM_WALLS_NEE 2

/* population storage */
#define LBM_FP32_DEV 0 /* IEEE binary32 deviations                      */
#define LBM_FP16_DEV 1 /* IEEE binary16 deviations, round-to-nearest-even */

/* porous medium description */
#define LBM_MEDIUM_UNIFORM 0   /* phi0, kappa0 everywhere                    */
#define LBM_MEDIUM_PHI_ERGUN 1 /* phi plane; K from Eq. (4) with diameter dp */
#define LBM_MEDIUM_PHI_KAPPA 2 /* phi plane and kappa = 1/K plane            */

typedef struct {
    int32_t enabled; /* 0: isothermal flow                                   */
    double tau_T;    /* zeta_1 = zeta_2 = 1/tau_T (Eq. B.7)                   */
    double sigma;    /* thermal capacity ratio (Eq. B.1)                      */
    double zeta3, zeta4; /* 1.1 in the paper (Sec. 3.4)                       */
    double Th, Tc;   /* Dirichlet temperatures of walls x = 0 and x = nx     */
    double T0;       /* reference temperature of a = g beta (T - T0) j        */
    double g_beta;   /* g * beta (Sec. 3.4)                                   */
} lbm_thermal;

typedef struct {
    int32_t nx, ny;   /* nodes, >= 1 each (>= 2 along a walled axis)          */
    int32_t bc_x;     /* LBM_PERIODIC, LBM_WALLS (walls at x = 0, x = nx) or   */
                      /* LBM_WALLS_NEE (walls on the nodes x = 0, x = nx - 1)  */
    int32_t bc_y;     /* likewise along y                                      */
    double lid_ux;    /* x-velocity of the top wall (needs walls in y)         */
    double nu;        /* fluid viscosity nu > 0; tau = 1/2 + 3 J nu (Eq. 21)   */
    double J;         /* viscosity ratio nu_e/nu > 0 (Eq. 5)                   */
    double s_e, s_q;  /* s_2 and s_4 = s_6 of Eq. (13): 1.1 and 1.2 (Sec. 3)   */
    int32_t medium;   /* LBM_MEDIUM_*                                          */
    double phi0;      /* uniform porosity, 0 < phi0 <= 1                       */
    double kappa0;    /* uniform 1/K >= 0 (0 = free fluid)                     */
    double dp;        /* particle diameter of Eq. (4) (MEDIUM_PHI_ERGUN)       */
    double F_eps;     /* >= 0: constant F_phi; < 0: F_phi from Eq. (4) per cell */
    double ax, ay;    /* uniform external acceleration a (Eq. 3)               */
    double Pi0;       /* rest value of phi*p; reference of the storage         */
    int32_t storage;  /* LBM_FP32_DEV or LBM_FP16_DEV                          */
    int32_t ckpt_every; /* 0: no recording; k > 0: record for lbm_backward   */
    int32_t j_plane;  /* 1: per-node viscosity ratio (lbm_set_viscosity_ratio) */
    lbm_thermal thermal;
} lbm_desc;

typedef struct lbm_ctx lbm_ctx; /* opaque, host memory owned by the library */

/* Fills *d with the paper's constants (J = 1, s_e = 1.1, s_q = 1.2,
 * zeta3 = zeta4 = 1.1, sigma = 1, Pi0 = 1, F_eps = -1, storage FP32) and
 * zeros elsewhere. d: host. */
int lbm_desc_defaults(lbm_desc *d);

/* Bytes of device workspace lbm_create needs for this descriptor.
 * max_steps_recorded: largest step count a recorded forward pass will run
 * (ignored unless d->ckpt_every > 0). d, bytes: host. */
int lbm_workspace_size(const lbm_desc *d, int64_t max_steps_recorded, size_t *bytes);

/* Creates a context holding the rest state f(0) = f_ref (t = 0) and, with
 * thermal enabled, g(0) at T = T0. phi / kappa: device [ny][nx] float planes
 * for the MEDIUM_PHI_* modes (NULL otherwise), read on `stream` before this
 * call's work completes, so the caller keeps them alive until the stream
 * passes this point. workspace: device, >= ws_bytes >= lbm_workspace_size(),
 * 256-byte aligned. stream: a hipStream_t (NULL = the null stream).
 * Errors: EINVAL for any invalid descriptor field (nx or ny < 1, a walled
 * axis with fewer than 2 nodes, nu or J <= 0, phi0 outside (0, 1],
 * kappa0 < 0, dp <= 0 with MEDIUM_PHI_ERGUN, s_e or s_q outside (0, 2),
 * tau_T <= 1/2, missing plane, lid on a periodic y axis, too small or
 * misaligned workspace). */
int lbm_create(const lbm_desc *d, const float *phi, const float *kappa, void *workspace,
               size_t ws_bytes, void *stream, lbm_ctx **out);

/* Ragged batch: n independent domains stepped together by one launch per
 * pass (a tile table maps workgroups to (domain, tile); a workgroup takes one
 * tile or walks a run of tiles, by the tuned grid size), replayed
 * from a HIP graph of graph_steps launches (default 32). descs, phis,
 * kappas: host arrays of n entries (phis[k]/kappas[k] device planes or
 * NULL). All domains must share the storage and be all thermal or all
 * isothermal (else ENOTSUP); ckpt_every > 0 gives ENOTSUP. The tile
 * schedule and persistent grid size are chosen by timing every compiled
 * candidate on the stream (autotuning, which synchronises the stream): the
 * one-cycle shapes and grids, and, for batches with bounce-back walls, the
 * two-cycle (temporal blocking) shapes and grids and, when isothermal, the
 * three-cycle grids, keeping the fastest mode, unless tune_cache (host path,
 * may be NULL) already holds a
 * choice for the same batch signature (sizes, boundaries, media, storage,
 * thermal, device); a new choice is appended there as a text line.
 * Results are bitwise identical to stepping each domain alone. The
 * per-domain calls (lbm_macroscopic, lbm_get_populations, lbm_reduce) take
 * the domain index. */
int lbm_batch_workspace_size(int32_t n, const lbm_desc *descs, size_t *bytes);
int lbm_create_batch(int32_t n, const lbm_desc *descs, const float *const *phis,
                     const float *const *kappas, void *workspace, size_t ws_bytes,
                     void *stream, const char *tune_cache, lbm_ctx **out);

/* Per-node viscosity ratio J = nu_e/nu of one domain (Eq. 5): each node
 * relaxes its stress moments at s_7 = s_8 = 1/(1/2 + 3 J nu) (Eqs. 13, 21),
 * as in the partially porous channel of Sec. 3.2, where the porous layer has
 * its own J and the free fluid J = 1. J: device [ny][nx] float plane, read on
 * the context's stream and copied (as rates) into the workspace before this
 * call returns; the caller keeps ownership. The domain must have been
 * created with j_plane = 1 (its plane then starts at the descriptor's J
 * everywhere); works for single contexts and batch domains. Synchronises the
 * stream. Errors: ESTATE without a plane, or once a recorded forward pass
 * (ckpt_every > 0) has left t = 0; EINVAL for NULL or any J that is not
 * finite and > 0 (the previous plane is kept). */
int lbm_set_viscosity_ratio(lbm_ctx *c, int32_t domain, const float *J);

/* Advances every domain by n >= 0 collide-and-stream cycles (Eqs. 14-15). */
int lbm_step(lbm_ctx *c, int64_t n);

/* Current time t (host). */
int lbm_time(const lbm_ctx *c, int64_t *t);

/* Macroscopic fields at the current time (Eqs. 18-20, B.5) of one domain:
 * p [ny][nx] (may be NULL), u [2][ny][nx] (u_x plane then u_y; may be NULL),
 * T [ny][nx] (may be NULL; EINVAL if non-NULL without thermal). */
int lbm_macroscopic(lbm_ctx *c, int32_t domain, float *p, float *u, float *T);

/* Population deviations f_i(t) - f_ref_i of one domain as float
 * [8][ny][nx] (paper order f_1..f_8), and thermal g_j(t) - w_T T0 as
 * [5][ny][nx] (g may be NULL). */
int lbm_get_populations(lbm_ctx *c, int32_t domain, float *df, float *dg);

/* Replaces the state with f(0) = f_ref + df (and g(0) = w_T T0 + dg) and
 * sets t = 0; df [8][ny][nx], dg [5][ny][nx] or NULL (keeps g at T0).
 * Values are rounded to the storage type. Clears any recording. A batch
 * domain takes a new state only while the batch is at t = 0 (else ESTATE). */
int lbm_set_populations(lbm_ctx *c, int32_t domain, const float *df, const float *dg);

/* FP64 reductions of one domain at the current time, computed on the GPU
 * with a fixed-order two-pass tree (bitwise reproducible): total mass
 * sum_x sum_i f_i(t), and the steady residual
 * ||u(t) - u(t-1)||_2 / ||u(t)||_2 (NaN at t = 0), with u(t-1) as the last
 * pass of the last lbm_step call computed it (any pass length gives the same
 * bits). Synchronises the stream.
 * mass, residual: host, either may be NULL. EUNSTABLE if either is not
 * finite (values are still written). */
int lbm_reduce(lbm_ctx *c, int32_t domain, double *mass, double *residual);

/* lbm_reduce for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, bit for bit, with the partial sums in a static
 * device array of the library (3 x 4096 + 4 doubles, 96 KiB, one copy per
 * GPU, held until the process ends) instead of the context's workspace. Calls
 * no allocating routine; the array's address is looked up once per device on
 * the first call there, with the context's device (the one current at
 * creation) made current for that lookup. Every call on one GPU shares that
 * array: calls that overlap on one GPU (from several host threads or streams)
 * race; calls from one thread do not overlap, since each synchronises its
 * stream. EINVAL if the domain needed more than 4096 workgroups of partial
 * sums (never for nx*ny <= 2^31); EDEVICE if the lookup fails. */
int lbm_reduce_static(lbm_ctx *c, int32_t domain, double *mass, double *residual);

/* Discrete adjoint of the recorded forward pass (hand-written, checkpointed
 * recomputation every ckpt_every steps). The loss L must depend on the state
 * only through u(T) at the current time T: dL_du is device [2][ny][nx]
 * (u_x plane then u_y; zeros where L does not look). Writes dL/dphi
 * [ny][nx] (device) and, for MEDIUM_PHI_KAPPA, dL/dkappa (device, may be
 * NULL). In MEDIUM_PHI_ERGUN, kappa and F_phi follow phi through Eq. (4).
 * With the thermal model the adjoint runs through the coupling (the
 * buoyancy of Sec. 3.4 and the D2Q5 equilibrium's dependence on u, App. B;
 * checkpoints then hold g too), one step per pass. ESTATE if the context was
 * not created with ckpt_every > 0, if the state was replaced since t = 0, or
 * if T exceeds the recorded capacity; ENOTSUP for on-node walls, FP16
 * storage, batches or MEDIUM_UNIFORM. The forward state is left at T. */
int lbm_backward(lbm_ctx *c, const float *dL_du, float *dL_dphi, float *dL_dkappa);

/* As lbm_backward, and also the gradient of L with respect to the scalar
 * parameters of the recorded pass: dL_dtheta (host, 4 doubles) receives
 * dL/dnu (nu enters the linear drag of Eq. 3 and s_nu of Eqs. 13 and 21, J
 * held fixed), dL/da_x and dL/da_y (the uniform acceleration of Eq. 3) and
 * dL/dlid_ux (the moving-wall term of the bounce-back lid), each summed over
 * every node and step in a fixed order in FP64 (bitwise reproducible).
 * dL_dphi may be NULL (then MEDIUM_UNIFORM is allowed); dL_dkappa as for
 * lbm_backward. The recomputation records two more FP32 planes per step (the
 * non-equilibrium stress moments). Synchronises the stream. Errors as for
 * lbm_backward; EINVAL if dL_dtheta is NULL. */
int lbm_backward_params(lbm_ctx *c, const float *dL_du, float *dL_dphi, float *dL_dkappa,
                        double *dL_dtheta);

/* Tangent-linear (forward-mode) model of the recorded pass: reruns it from
 * f(0) (the first checkpoint) to the current time T together with the
 * derivative of the state along a direction of the inputs, and writes
 * du = (d u(T) / d eps) at eps = 0 for phi + eps dphi and
 * (nu, a_x, a_y, lid_ux) + eps dtheta, as device [2][ny][nx] (u_x plane then
 * u_y). dphi: device [ny][nx] or NULL (no porosity change); dtheta: host 4
 * doubles or NULL. The forward state is left at T; the checkpointed
 * recording is required as for lbm_backward (ESTATE otherwise), and thermal,
 * on-node walls, FP16 storage and batches give ENOTSUP. For any loss
 * L(u(T)), <dL/du, du> equals <dL/dphi, dphi> + <dL/dtheta, dtheta> from
 * lbm_backward_params up to rounding. */
int lbm_tangent(lbm_ctx *c, const float *dphi, const double *dtheta, float *du);

/* Snapshot of one context's state (host memory, synchronous): a 64-byte
 * header (format tag, a hash of every descriptor field that gives the state
 * its meaning, the thermal block included, t, and the payload size), then
 * f(t) (and g(t)) in the storage type and the two u(t-1) planes of the
 * residual. lbm_state_bytes gives the size; lbm_load takes a snapshot of a
 * context with the same descriptor (else EINVAL, nothing changed) and clears
 * any recording. */
int lbm_state_bytes(const lbm_ctx *c, size_t *bytes);
int lbm_save(lbm_ctx *c, void *host_buf, size_t bytes);
int lbm_load(lbm_ctx *c, const void *host_buf, size_t bytes);

/* Destroys the context (NULL is accepted). The workspace is not touched.
 * The library keeps the set of live contexts: a handle that was already
 * destroyed, or never returned by lbm_create / lbm_create_batch, gets
 * LBM_EINVAL here and from every other entry point, without its memory
 * being read, so a second lbm_destroy is harmless. (Once the allocator has
 * reused the address for a newer context, a stale handle names that one.) */
int lbm_destroy(lbm_ctx *c);

/* Static text for a status code, and the thread-local message of the last
 * failed call on this thread ("" if none). */
const char *lbm_strerror(int status);
const char *lbm_last_error(void);

/* Information on the launch the library uses for the step of this context:
 * threads along x per 256-thread block, nodes per thread along x, rows per
 * thread and grid size (host outputs, each may be NULL). */
int lbm_schedule(const lbm_ctx *c, int32_t *tile_w, int32_t *vec, int32_t *rows, int32_t *grid);

/* Selects the launch shape of the step kernel of a single-domain context:
 * tile_w threads along x per 256-thread block, vec consecutive nodes per
 * thread along x, rows per thread, swizzle 0/1 (contiguous tiles per XCD).
 * Compiled shapes (tile_w, vec, rows): (256,1,1) (256,1,2) (128,1,1)
 * (128,1,2) (64,1,2) (64,1,4) (128,2,1) (64,2,2) (64,4,1) (32,4,2) (64,4,2)
 * (16,4,4). Every shape computes bitwise-identical results; only speed
 * differs. EINVAL for another shape, ENOTSUP on a batch (its schedule is
 * autotuned). */
int lbm_set_schedule(lbm_ctx *c, int32_t tile_w, int32_t vec, int32_t rows, int32_t swizzle);

/* Cycles per HBM pass of a context with bounce-back walls: 1,
 * 2 (temporal blocking: one launch gathers, collides on its tile plus a
 * one-node ring kept in LDS, then collides again, so each population crosses
 * HBM about once per two cycles), 3 (a two-node ring, three collisions per
 * launch) or 4 (a three-node ring, four collisions per launch; single
 * isothermal domains only). Results are bitwise identical in every mode.
 * Multi-cycle passes are skipped for t = 0; while recording for lbm_backward
 * no pass steps over a checkpoint time. Shorter passes fill in where fewer
 * cycles remain. The last pass of each lbm_step call also writes the
 * velocity of its last collision, u(t-1) of the final time t, into two FP32
 * planes of the workspace (8 bytes per node), which lbm_reduce's residual
 * reads. The recomputation inside
 * lbm_backward uses passes of the same length (recording u at every cycle;
 * four-cycle passes also in mode 3 for isothermal domains of at least 2^22
 * nodes, where they are faster) and its adjoint sweep two or three steps per
 * pass in modes 2, 3 and 4 (two for thermal runs). The D2Q5 field of a thermal domain rides
 * in LDS beside the populations. Default for single domains that allow it: 4
 * for isothermal domains of at least 2^23 nodes, 3 for isothermal domains of
 * at least 2^20 nodes and thermal domains of at least 2^22, 2 for
 * smaller ones (with 8-row tiles below 2^20 nodes and for thermal domains), 1
 * for the others; for batches, the
 * autotuner's choice among 1, 2, 3 and 4 (isothermal batches; mode 4 runs one
 * workgroup per 64 x 26 tile from a table of its own; a batch switched to 3 or
 * 4 walks 64 x 16 tiles in its three- and two-cycle passes; switching uploads
 * that tile table and synchronises the stream). ENOTSUP for on-node walls,
 * population or thermal buffers of 4 GiB or more, mode 3 on thermal batches,
 * mode 4 on thermal domains and thermal batches, a mode a batch has no tuned schedule
 * for; EINVAL for another value. */
int lbm_set_time_blocking(lbm_ctx *c, int32_t cycles_per_pass);

/* Current cycles per pass, and the workgroup size, tile rows (tiles are 64
 * nodes wide) and grid size of the multi-cycle pass it runs: the four-cycle
 * kernel in mode 4 (768 threads, 26 rows; for a batch the grid is its number
 * of 64 x 26 tiles), the three-cycle kernel in mode 3
 * (single isothermal domains of 2^23 nodes or more: 768 threads, 28 rows;
 * other domains and batches: 512 threads, 16 rows), else the two-cycle
 * kernel's
 * (host outputs, each may be NULL). */
int lbm_time_blocking(const lbm_ctx *c, int32_t *cycles_per_pass, int32_t *threads, int32_t *rows,
                      int32_t *grid);

/* Workgroup shape of the two-cycle kernel: threads in {256, 512} and tile
 * rows in {8, 16} (tiles are 64 nodes wide). Results do not depend on it.
 * Default 512 threads, 16 rows (8 rows for thermal domains and for domains
 * below 2^20 nodes). ENOTSUP on batches (autotuned). */
int lbm_set_two_cycle_tile(lbm_ctx *c, int32_t threads, int32_t rows);

/* Number of steps lbm_step replays from one hand-built HIP graph of kernel
 * nodes (up to 4096, rounded down to a whole number of passes; 0 launches
 * every step separately).
 * Defaults: 0 for single domains, 32 for batches. Graphs are not used while
 * a trajectory is recorded for lbm_backward. Results do not depend on it. */
int lbm_set_graph_steps(lbm_ctx *c, int32_t steps);

#ifdef __cplusplus
}
#endif
#endif
