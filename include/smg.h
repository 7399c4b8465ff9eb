/*
 * smg.h -- C-ABI of the MI355X stochastic multigrid sampler/solver.
 *
 * The library draws Gaussian fields x ~ N(0, kT A^-1), where A = -L is the discrete
 * Laplacian L = DG on a uniform cell-centred grid (paper: Sec. "Spatially Adaptive
 * Discretizations", uniform-mesh case), periodic in x and y, with no-slip walls on the
 * faces z = 0 and z = nz*h (Sec. 2: steady Stokes with u = 0 on the boundary), and it
 * solves A u = f.  Sampling is the paper's stochastic multigrid method (Sec. "Stochastic
 * Multigrid Methods", Alg. 3 V-cycle; Sec. "Stochastic Iterative Methods", stochastic
 * Gauss-Seidel with J = C - R C R^T): the covariance -L^-1 of the driving field xi of
 * eq. g_gen_xi, scaled by kT.  The solve is the same cycle with the noise switched off
 * (stationary mean (I - R)^-1 s = A^-1 f).
 *
 * Conventions for every entry point:
 *  - Return value: SMG_OK (0) or a negative SMG_E* code; smg_last_error() then returns a
 *    message for the calling thread.  No entry point aborts the process.
 *  - Device memory: every device byte (workspace, chain state, inputs, outputs) belongs
 *    to the caller.  The library never allocates or frees device memory.  Device pointers
 *    must be 256-byte aligned.
 *  - Streams: work is enqueued on the caller's hipStream_t, passed as void*.  Calls are
 *    asynchronous except smg_solve (which synchronises the stream to test convergence)
 *    and smg_bind_workspace (which synchronises after uploading its tables).
 *    A hierarchy holds per-call state in its workspace: calls on one hierarchy must not
 *    overlap (one stream at a time).  Different hierarchies are independent.
 *  - Field layout: C-contiguous [ncomp][nz][ny][nx], x fastest, IEEE float64 unless
 *    stated.  Components are independent scalar fields with the same operator.
 *  - Noise: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed, with counter
 *    (site pair, level | slot<<4 | colour<<12 | comp<<16 | kind<<24, cycle lo, cycle hi);
 *    a result depends only on (seed, cycle indices, parameters), never on launch shape,
 *    batching or stream.
 */
#ifndef SMG_H
#define SMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SMG_OK = 0,
  SMG_EINVAL = -1,      /* invalid argument, shape or parameter */
  SMG_ENOMEM = -2,      /* workspace too small / request over budget */
  SMG_ENOTCONV = -3,    /* solve did not reach rtol within max_cycles */
  SMG_ENONFINITE = -4,  /* NaN or Inf in an input or residual */
  SMG_EHIP = -5,        /* a HIP runtime call failed */
  SMG_ESTATE = -6       /* hierarchy used before smg_bind_workspace */
};

enum { SMG_COARSEST_CHOLESKY = 0, SMG_COARSEST_SMOOTH = 1 };
enum { SMG_FP64 = 0, SMG_FP32_REFINED = 1 };
enum { SMG_OUT_F64 = 0, SMG_OUT_F32 = 1 };

/* Boundary condition of one axis (Sec. 2: the fluid is periodic along the walls and satisfies
 * u = 0 on the no-slip walls; Sec. "Spatially Adaptive Discretizations": the discrete operator
 * takes the boundary through ghost cells).
 *   SMG_BC_DEFAULT         the problem's own condition on that axis: periodic on x and y,
 *                          no-slip walls on the z faces (so a zero-initialised descriptor
 *                          describes the wall-bounded problem).
 *   SMG_BC_PERIODIC        periodic axis.
 *   SMG_BC_DIRICHLET_FACE  homogeneous Dirichlet (no-slip) walls on the two cell faces that
 *                          bound the axis, through an antisymmetric ghost cell (u_ghost =
 *                          -u_wall-cell), so the wall-layer diagonal is 7/h^2.
 * Implemented combination: x and y periodic, z Dirichlet-face (the wall-bounded channel);
 * any other combination is rejected with SMG_EINVAL (a fully periodic grid has the singular
 * constant mode, so it has no Gaussian law with covariance A^-1). */
enum { SMG_BC_DEFAULT = 0, SMG_BC_PERIODIC = 1, SMG_BC_DIRICHLET_FACE = 2 };

/* Grid: nx, ny even (red-black periodicity), nz >= 1, ncomp in [1, 255], h > 0, kT >= 0;
 * bc_x, bc_y, bc_z one of SMG_BC_* per axis (see above). */
typedef struct {
  int32_t nx, ny, nz, ncomp;
  double h;
  double kT;
  int32_t bc_x, bc_y, bc_z;
} smg_grid_desc;

/* Cycle parameters (Alg. 3 V(nu1, nu2); the paper leaves depth and coarsest handling open).
 *   levels        number of levels (0 = automatic: coarsen while a level has more than
 *                 coarsest_max unknowns and can be smoothed).
 *   nu1, nu2      pre/post sweeps per level (each sweep visits every colour once).
 *   coarsest_max  automatic-depth threshold (1..4096); the dense coarsest factor itself is
 *                 limited to 4096 unknowns whatever the depth.
 *   coarsest_mode SMG_COARSEST_CHOLESKY: exact draw A_c^-1 b + sqrt(kT) L_c^-T n;
 *                 SMG_COARSEST_SMOOTH: nu1 + nu2 sweeps only (the literal Alg. 3 step 2).
 *   precision     SMG_FP64 (all FP64) or SMG_FP32_REFINED (FP32 sweeps and transfers inside
 *                 an FP64 correction loop, Alg. 1; FP64 residual and coarsest).
 *   stride        cycles per emitted sample (>= 1).
 *   burn_in       cycles run before the first emitted sample of each smg_sample_field call.
 */
typedef struct {
  int32_t levels;
  int32_t nu1, nu2;
  int32_t coarsest_max;
  int32_t coarsest_mode;
  int32_t precision;
  int32_t stride;
  int32_t burn_in;
} smg_cycle_params;

/* Filled by smg_hierarchy_info. */
typedef struct {
  size_t workspace_bytes;   /* device bytes smg_bind_workspace needs */
  size_t state_bytes;       /* bytes of one chain state: ncomp*nx*ny*nz float64 */
  int32_t n_levels;
  int32_t dims[16][3];      /* (nx, ny, nz) per level, finest first */
  int32_t coarsest_unknowns;
} smg_info;

typedef struct {
  int32_t cycles;           /* V-cycles performed */
  double relres;            /* max over components of ||f - A u||_2 / ||f||_2 */
  double last_ratio;        /* max over components of ||r_k|| / ||r_{k-1}|| for the last cycle
                               (0 when fewer than two cycles ran): the cycle's contraction */
} smg_solve_info;

typedef struct smg_hierarchy smg_hierarchy;

/* Plans the level hierarchy and builds, on the host, the Galerkin coarse operators
 * A^(l) = P^T A^(l-1) P (Sec. "Stochastic Multigrid Methods", variational property) from
 * 1D recurrences, the 2x2x2 block factors of every Galerkin level and the dense Cholesky
 * factor of the coarsest level.  *out receives a host object owned by the caller (free it
 * with smg_destroy_hierarchy).  No device work.  Errors: SMG_EINVAL for unsupported
 * shapes (nx or ny odd, levels not reachable, coarsest above 4096 unknowns) or boundary
 * conditions other than periodic x, y and Dirichlet-face z. */
int smg_create_hierarchy(const smg_grid_desc* desc, const smg_cycle_params* params,
                         smg_hierarchy** out);

/* Sizes and level dimensions of a created hierarchy. */
int smg_hierarchy_info(const smg_hierarchy* h, smg_info* info);

/* Binds caller-owned device memory of at least workspace_bytes (256-byte aligned) on the
 * current device and uploads the operator tables and factors into it on `stream`, then
 * synchronises the stream.  The memory must stay valid until the hierarchy is destroyed
 * or re-bound.  Errors: SMG_EINVAL (null/misaligned), SMG_ENOMEM (too small), SMG_EHIP. */
int smg_bind_workspace(smg_hierarchy* h, void* dev_ptr, size_t bytes, void* stream);

/* Runs the stochastic chain: burn_in + n*stride V-cycles with b = 0 (target N(0, kT A^-1),
 * eq. J_eq_C_R), cycle indices first_cycle, first_cycle+1, ...  `state` (device, in/out,
 * state_bytes, float64 [ncomp][nz][ny][nx]) holds the chain's current field: read at the
 * start, written at the end; zero it for a chain from the zero start.  After the k-th
 * group of `stride` cycles the field is written to out[k-1] (device, [n][ncomp][nz][ny][nx],
 * float64 or float32 per out_dtype); out may be NULL when n == 0.  Resuming with the
 * returned state and first_cycle advanced by the cycles run continues the same chain
 * bit for bit.  Asynchronous on `stream`.  Errors: SMG_EINVAL, SMG_ESTATE, SMG_EHIP. */
int smg_sample_field(smg_hierarchy* h, int64_t n, uint64_t seed, uint64_t first_cycle,
                     void* state, void* out, int32_t out_dtype, void* stream);

/* Solves A u = f (f, u device float64 [ncomp][nz][ny][nx]) by repeated noise-free
 * V-cycles from u = 0 until ||f - A u||_2 <= rtol ||f||_2 for every component or
 * max_cycles cycles ran.  Synchronises `stream` after each cycle to read the residual
 * norms; *info (host) is filled.  Errors: SMG_ENOTCONV (u holds the last iterate),
 * SMG_ENONFINITE (f or a residual not finite), SMG_EINVAL, SMG_ESTATE, SMG_EHIP. */
int smg_solve(smg_hierarchy* h, const void* f, void* u, double rtol, int32_t max_cycles,
              void* stream, smg_solve_info* info);

/* ---- Observables of the chain (Sec. "Stochastic Iterative Methods": the lag-k correlation of
 * the emitted samples decides how many cycles separate effectively independent draws). ----
 * A mode is a triple (a, b, m) naming the real eigenvector phi = e_a(x) e_b(y) w_m(z) of A:
 * e_a is the a-th real periodic vector on n points (a = 0: 1/sqrt(n); a = 2j-1 and a = 2j,
 * 1 <= j < n/2: sqrt(2/n) cos(2 pi j i/n) and sqrt(2/n) sin(2 pi j i/n); a = n-1:
 * (-1)^i/sqrt(n)); w_m (m = 1..nz) is sin(pi m (z + 1/2)/nz) normalised.  Its eigenvalue is
 * (4/h^2)(sin^2(pi j_a/nx) + sin^2(pi j_b/ny) + sin^2(pi m/(2 nz))). */
#define SMG_MAX_MODES 32

/* smg_lowest_modes: the k (<= SMG_MAX_MODES, <= nx*ny*nz) modes with the smallest
 * eigenvalues on an nx x ny x nz grid (nx, ny even), ascending; ties broken by m, then b,
 * then a, eigenvalues compared after rounding to multiples of 2^-30/h^2.  modes: host
 * int32 [k][3] (a, b, m).  Host only.  Errors: SMG_EINVAL. */
int smg_lowest_modes(int32_t nx, int32_t ny, int32_t nz, int32_t k, int32_t* modes);

/* smg_sample_stats: smg_sample_field with FP64 statistics of every emitted sample, taken in
 * the same pass that writes it.  For emitted sample i and component c:
 *   obs[i][c][q] = <phi_q, x_c>  (q < n_modes),  obs[i][c][n_modes] = 1/2 x_c^T A x_c
 *   (obs: device float64 [n][ncomp][n_modes + 1], 8-byte aligned; NULL = none);
 *   moments[0][c][cell] += x_c[cell], moments[1][c][cell] += x_c[cell]^2
 *   (moments: device float64 [2][ncomp][nz][ny][nx], accumulated over calls -- the caller
 *   zeroes it; NULL = none).
 * out may be NULL (statistics only).  modes: host int32 [n_modes][3], 0 <= n_modes <=
 * SMG_MAX_MODES (read during the call).  Sums run in a fixed order, so results do not
 * depend on timing.  Asynchronous, except that a new mode list is uploaded synchronously.
 * Errors: as smg_sample_field, SMG_EINVAL for a mode outside the grid. */
int smg_sample_stats(smg_hierarchy* h, int64_t n, uint64_t seed, uint64_t first_cycle,
                     void* state, void* out, int32_t out_dtype, const int32_t* modes,
                     int32_t n_modes, void* obs, void* moments, void* stream);

/* ---- Batched chains: many independent instances of one grid in every launch. ----
 * A hierarchy of ncomp components can carry nchains independent chains of comps_per_chain
 * components each (nchains * comps_per_chain <= ncomp; only those first components are
 * processed).  Chain c is keyed by its own seed and first cycle and draws exactly the noise
 * that smg_sample_field on a hierarchy of comps_per_chain components draws for that seed and
 * cycle (its components are numbered from 0 in the noise counters), so every result is bit
 * for bit that of the chain run alone; each launch covers all chains at once. */

/* smg_sample_batch: like smg_sample_stats for nchains chains.  seeds and first_cycles: host
 * uint64 [nchains] (first_cycles NULL = all 0), copied into the hierarchy's chain table in
 * stream order; seeds == NULL reuses the table as the previous batched call left it.  Every
 * call advances the table by the cycles it ran, so a repeated call -- or a replay of a
 * captured graph of the call -- continues every chain.  state, out, obs, moments cover the
 * nchains*comps_per_chain processed components ([..][nchains*comps_per_chain][..] layouts).
 * Errors: as smg_sample_stats; SMG_ESTATE when seeds == NULL and no table of this shape
 * was written; at most 255 chains. */
int smg_sample_batch(smg_hierarchy* h, int32_t nchains, int32_t comps_per_chain,
                     const uint64_t* seeds, const uint64_t* first_cycles, int64_t n, void* state,
                     void* out, int32_t out_dtype, const int32_t* modes, int32_t n_modes,
                     void* obs, void* moments, void* stream);

/* smg_solve_batch: solves A u = f for every chain (f, u: [nchains*comps_per_chain][N]).
 * All chains cycle together; a chain's u is written at the cycle its components all reach
 * rtol, so it equals the solve of that chain alone.  infos: host [nchains].  Returns
 * SMG_ENOTCONV if any chain missed rtol within max_cycles (its u is the last iterate). */
int smg_solve_batch(smg_hierarchy* h, int32_t nchains, int32_t comps_per_chain, const void* f,
                    void* u, double rtol, int32_t max_cycles, void* stream,
                    smg_solve_info* infos);

/* ---- Allocation-free sampling (for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). ----
 * smg_sample_field_static: smg_sample_field on a hierarchy whose workspace is the library's own
 * device array of SMG_STATIC_SCRATCH_BYTES (one copy per device, held until the process ends)
 * instead of caller-bound memory; smg_bind_workspace is not needed.  It calls no hipMalloc,
 * hipFree or allocating library routine.  state and out are the caller's, as for
 * smg_sample_field, and results are the same bit for bit.  Every call on a device shares that
 * device's array, which keeps the last call's contents: the tables of a hierarchy are uploaded
 * (and the stream synchronised) when another hierarchy used the array last; calls that overlap
 * on one device (different streams or threads with work in flight) race on the array and must
 * be serialised by the caller.  A hierarchy bound with smg_bind_workspace keeps that binding
 * for its other calls.  Errors: SMG_ENOMEM when the hierarchy's workspace_bytes exceeds
 * SMG_STATIC_SCRATCH_BYTES; otherwise as smg_sample_field. */
#define SMG_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
int smg_sample_field_static(smg_hierarchy* h, int64_t n, uint64_t seed, uint64_t first_cycle,
                            void* state, void* out, int32_t out_dtype, void* stream);

/* ---- Uneven instances in one call (a workload of many grids of different sizes). ----
 * smg_batch_run runs a list of operations on distinct bound hierarchies (each hierarchy at most
 * once), all on `stream`:
 *   SMG_OP_SAMPLE: smg_sample_field (nchains == 0: one chain of all components keyed by seed,
 *     first_cycle) or smg_sample_batch without statistics (nchains >= 1: seeds/first_cycles
 *     host [nchains], seeds NULL = continue the table); state, out, out_dtype, n as there
 *     (out NULL: the cycles run without writing samples).
 *   SMG_OP_SOLVE: smg_solve (nchains == 0) or smg_solve_batch (nchains >= 1) of f into u to
 *     rtol within max_cycles; infos (host, [max(nchains, 1)], or NULL) filled.
 * Sampling items run first, cycle by cycle in step (cycle k of every item before cycle k + 1 of
 * any); then the solve items cycle in step until each has converged or run out of cycles.  In
 * every cycle the levels that each hierarchy runs in its LDS-resident bottom launch (the levels
 * of at most 4096 cells and the coarsest draw: Sec. "Stochastic Multigrid Methods", Alg. 3,
 * below the tiled levels) are run for all items in as few launches as possible (one per sweep
 * precision and noise setting, up to 16 hierarchies and 256 components each), instead of one
 * latency-bound launch per hierarchy.  With SMG_OPT_STREAM_GROUPS above 1 on any sampling
 * item's hierarchy (the largest setting counts), the sampling cycles run in that many staggered
 * groups as in smg_sample_batch, group g taking its share of every item's components, on the
 * side streams of the first sampling item's hierarchy.  Every item's result is bit for bit that
 * of its own call alone.  Without solve items the call is asynchronous (and can be captured in
 * a graph); solve
 * items synchronise the stream once per cycle for all of them.  status receives each item's
 * return code; the function returns SMG_OK or the first failing item's code (SMG_EINVAL for a
 * repeated hierarchy or unknown op, before any work). */
enum { SMG_OP_SAMPLE = 0, SMG_OP_SOLVE = 1 };
typedef struct {
  smg_hierarchy* h;
  int32_t op;
  int32_t nchains, comps_per_chain;
  int32_t out_dtype;
  int64_t n;
  uint64_t seed, first_cycle;
  const uint64_t* seeds;
  const uint64_t* first_cycles;
  void* state;
  void* out;
  const void* f;
  void* u;
  double rtol;
  int32_t max_cycles;
  smg_solve_info* infos;
  int32_t status;
} smg_batch_item;
int smg_batch_run(smg_batch_item* items, int32_t n_items, void* stream);

/* Frees the host object.  Never touches the caller's device memory. */
void smg_destroy_hierarchy(smg_hierarchy* h);

/* Message for the last failing call on this thread ("" if none). */
const char* smg_last_error(void);

/* ---- Component entry points (used by the parity tests; same kernels as the cycle). ----
 * All fields natural layout float64 [ncomp][nz_l][ny_l][nx_l] on the device.
 *
 * smg_debug_smooth: one stochastic Gauss-Seidel sweep pass of one colour on level l
 *   (l = 0: red-black point heat bath, colour 0..1; l >= 1: 2x2x2 block heat bath,
 *   colour 0..7) in place on x with right-hand side b (NULL = 0 on level 0), noise
 *   counters (seed, cycle, slot); noise off when with_noise == 0.
 * smg_debug_restrict_residual: b_{l+1} = P^T (b_l - A_l x_l)  (b_l NULL = 0 on level 0).
 * smg_debug_prolong_add: x_l += P e_{l+1}.
 * smg_debug_coarsest: x_c = A_c^-1 b_c (+ sqrt(kT) L_c^-T n when with_noise) on the
 *   coarsest level. */
int smg_debug_smooth(smg_hierarchy* h, int32_t level, int32_t colour, void* x, const void* b,
                     uint64_t seed, uint64_t cycle, int32_t slot, int32_t with_noise,
                     void* stream);
int smg_debug_restrict_residual(smg_hierarchy* h, int32_t level, const void* x, const void* b,
                                void* b_coarse, void* stream);
int smg_debug_prolong_add(smg_hierarchy* h, int32_t level, void* x, const void* e_coarse,
                          void* stream);
int smg_debug_coarsest(smg_hierarchy* h, void* x, const void* b, uint64_t seed, uint64_t cycle,
                       int32_t with_noise, void* stream);

/* smg_debug_host_table: copies a host-built table of level l into out (host memory of
 *   `count` doubles; no device work, callable without a workspace).
 *   which = 0: Galerkin row coefficients [nz_l][125], index (dz+2)*25 + (dy+2)*5 + (dx+2);
 *   which = 1: block factors [nz_l/2][3][64] (A_BB^-1, L_BB^-T, A_BB, row-major);
 *   which = 2: coarsest A_c^-1 [n_c][n_c];  which = 3: coarsest L_c^-1 [n_c][n_c].
 *   Returns SMG_EINVAL if the table does not exist or count is wrong. */
int smg_debug_host_table(const smg_hierarchy* h, int32_t level, int32_t which, double* out,
                         size_t count);

/* smg_set_option: execution switches that never change results.
 *   SMG_OPT_BOTTOM_KERNEL (default 1): run the levels with at most 4096 cells (and the
 *   coarsest draw) in one LDS-resident launch per cycle; 0 = one launch per colour pass.
 *   SMG_OPT_BLOCK_TILE (default SMG_TILE_AUTO): see below.
 *   SMG_OPT_TIMED_KERNEL (default SMG_TIMED_FINE_PASS): the kernel class that
 *   smg_kernel_timing brackets with events: the level-0 colour pass, the level-1 block
 *   colour passes (one or two colours per launch, see SMG_OPT_BLOCK_PAIRS), or the
 *   LDS-resident bottom launch. */
enum {
  SMG_OPT_BOTTOM_KERNEL = 1,
  SMG_OPT_TIMED_KERNEL = 2,
  SMG_OPT_BLOCK_TILE = 3,
  SMG_OPT_BLOCK_PAIRS = 4,
  SMG_OPT_STREAM_GROUPS = 5
};
/* SMG_OPT_STREAM_GROUPS (default 1, at most 2): smg_sample_field, smg_sample_stats and
 * smg_sample_batch split the components they run into this many contiguous groups (at most
 * one component per group; group i takes components [i nc / G, (i+1) nc / G)) and run each
 * group's cycles and emissions on a side stream of its own, which the hierarchy creates on
 * first use (G streams together, so that the runtime spreads them over its hardware queues; on
 * the current device, at the default priority, destroyed with the hierarchy); the caller's
 * stream only forks and joins.  Group i starts each cycle once
 * group i - 1 has finished that cycle's down-leg, so the groups run staggered: the
 * latency-bound launches of one (the LDS-resident bottom, the small levels) overlap the
 * bandwidth-bound ones of another.  The side streams wait for the caller's stream at the start
 * of the call and the caller's stream waits for them before the call's last work (the state
 * export), so the call stays ordered on the caller's stream.  Every output is bit-identical to
 * the one-stream run.  smg_batch_run groups its sampling items likewise (see there).  One
 * stream while kernel timing is on, in smg_sample_field_static, and in the other entry
 * points.  At most 2: a process gets four hardware queues, shared by all its streams, and two
 * groups on one queue run one after the other behind the stagger's waits (3 groups were never
 * faster than 2 and once 55 % slower, 4 groups 27 % slower).  A grouped call can be captured in a
 * graph (the side streams join the capture through
 * the fork event), but its replay measured slower than that of a one-stream capture: set 1
 * before capturing. */
/* SMG_OPT_BLOCK_PAIRS (default 1): run the eight block colours of a sweep on a Galerkin level
 * as four launches of two colours each (colours c and c ^ 1 differ only in the parity of bx,
 * so one work-group owning whole x-rows draws both in turn from one staged tile); levels wider
 * than 128 cells in x use one launch per colour.  0 = one launch per colour everywhere. */
/* SMG_OPT_BLOCK_TILE: blocks per work-group (x by y) of the Galerkin-level block passes;
 * SMG_TILE_AUTO (default) takes the largest of 8x4, 4x4, 4x2 that gives at least 512
 * work-groups for the pass. */
enum { SMG_TILE_AUTO = 0, SMG_TILE_4X4 = 1, SMG_TILE_4X2 = 2, SMG_TILE_8X4 = 3 };
enum { SMG_TIMED_FINE_PASS = 0, SMG_TIMED_LEVEL1_BLOCK_PASS = 1, SMG_TIMED_BOTTOM = 2 };
int smg_set_option(smg_hierarchy* h, int32_t option, int64_t value);

/* ---- Kernel timing (measurement support). ----
 * When enabled, the library records HIP events on the caller's stream around every run of
 * back-to-back launches of the kernel class chosen by SMG_OPT_TIMED_KERNEL (the colour
 * passes of one sweep, or one bottom launch) and accumulates their elapsed times (read after
 * the stream is idle).  *count receives the number of launches inside the bracketed runs,
 * *total_ms the sum of the runs' elapsed times; both are reset by smg_kernel_timing(h, 1). */
int smg_kernel_timing(smg_hierarchy* h, int32_t enable);
int smg_kernel_timing_read(smg_hierarchy* h, int64_t* count, double* total_ms);


/* ==== Spatially adaptive composite grid: the FAC sampler and solver ====================
 * Mesh (Sec. "Spatially Adaptive Discretizations"): a base grid nx x ny x nz of width h,
 * periodic in x and y, no-slip walls at z = 0 and z = nz*h, with one box of base cells
 * [box[0], box[1]) x [box[2], box[3]) x [box[4], box[5]) refined by two.  Neighbouring cells
 * differ by at most one level.  Operator L = D G (eq. def_L): same-level face gradients
 * (eq. def_discr_grad0); on a coarse-fine face the gradient of the mean of the four fine cells
 * on the coarse face minus the coarse value over 3/4 h, shared by those four cells, with the
 * coarse face value their mean (eqs. def_discr_grad .. def_discr_grad_last, read in 3D);
 * walls by the antisymmetric ghost.  S = diag(volume) L is symmetric; the library samples
 * x ~ N(A^-1 b, kT A^-1) with A = -S/h^3 (on coarse cells the uniform-grid rows of -L, on fine
 * cells -L/8), which is C = -2 L^-1 Ccal (Sec. "Performance of the Stochastic Samplers in
 * Practice") with Ccal = (kT/2) h^3 diag(volume)^-1, and solves A u = f.
 *
 * FAC cycle (Algs. 1-3 with the variational property): the coarse space of the composite mesh
 * is the whole base grid, mapped onto the composite unknowns by P (identity on coarse cells,
 * trilinear onto fine cells); b_0 = P^T (b - A x); a stochastic V(mu1, mu2) cycle on the
 * Galerkin base hierarchy A_0 = P^T A P, A_{l+1} = P_l^T A_l P_l (2x2x2 block heat baths,
 * exact coarsest draw) from y = 0; x += P y; then nu composite sweeps, each a point heat bath
 * over twelve uncoupled classes (coarse cells by parity; fine cells off the interface layer by
 * parity; interface-layer fine cells by the eight parities (x%2) + 2(y%2) + 4(z%2)).
 *
 * Fields: coarse part on the whole base grid, float64 [nz][ny][nx] (entries of covered cells
 * are ignored on input; outputs write them as 0 only where stated); fine part float64
 * [2(box[5]-box[4])][2(box[3]-box[2])][2(box[1]-box[0])].  One component per field.  Noise
 * streams as for the uniform grid with kind 2 (composite passes: level 0, colour = class,
 * slot = sweep, site = index in its own array, halved in the four parity classes 0..3, whose
 * cells are one of each pair (2q, 2q+1) of their array), kind 3 (base block levels) and kind 4
 * (the coarsest base level).  Memory, stream and error conventions as above. */
typedef struct smg_composite smg_composite;

typedef struct {
  int32_t nx, ny, nz;   /* base grid: nx, ny even and >= 4 */
  int32_t box[6];       /* x0, x1, y0, y1, z0, z1 (base cells), not spanning a periodic extent */
  double h;
  double kT;
} smg_composite_desc;

typedef struct {
  int32_t nu;           /* composite sweeps per cycle (Alg. 2 step 5) */
  int32_t mu1, mu2;     /* pre/post sweeps of the base V-cycle (Alg. 3) */
  int32_t levels;       /* base levels (0 = automatic by coarsest_max) */
  int32_t coarsest_max; /* automatic-depth threshold, 1..4096 */
  int32_t gs_only;      /* 1: composite sweeps only -- the stochastic Gauss-Seidel sampler on the
                           composite mesh, without the coarse correction (for comparisons) */
  int32_t precision;    /* SMG_FP64, or SMG_FP32_REFINED: FP32 sweeps and transfers of the cycle in
                           the correction form, with the residual b - A x, the update of x and the
                           coarsest draw in FP64 (Alg. 1); the component entry points need FP64 */
  int32_t row_lanes;    /* lanes per row in the block passes and residuals over long Galerkin rows:
                           0 = by the launch's row count (2 for large launches, 8 for small), or
                           2 or 8 for every such launch; the results agree up to summation order */
} smg_fac_params;

typedef struct {
  size_t workspace_bytes;
  int64_t base_cells;       /* nx*ny*nz: length of a coarse-part field */
  int64_t fine_cells;       /* length of a fine-part field */
  int64_t unknowns;         /* composite unknowns: uncovered base cells + fine cells */
  int32_t fine_dims[3];     /* (fx, fy, fz) */
  int32_t n_levels;         /* base levels, finest first */
  int32_t dims[16][3];
  int32_t stencils[16];     /* distinct rows per base level */
  int32_t block_types[16];  /* distinct 2x2x2 diagonal blocks per block level */
  int32_t layer_cells;
  int32_t coarsest_unknowns;
} smg_composite_info;

/* Plans the composite hierarchy on the host: the Galerkin base operators (rows near the box
 * cell by cell, the rest per z-plane, equal rows shared), block factors and the dense coarsest
 * factor.  No device work.  Errors: SMG_EINVAL (shape, box, parameters, a base level that
 * cannot be coarsened or block-smoothed), SMG_ENOMEM. */
int smg_composite_create(const smg_composite_desc* desc, const smg_fac_params* params,
                         smg_composite** out);
int smg_composite_get_info(const smg_composite* h, smg_composite_info* info);
/* Binds caller-owned device memory (>= workspace_bytes, 256-byte aligned) and uploads the
 * tables on `stream`, then synchronises it. */
int smg_composite_bind(smg_composite* h, void* dev_ptr, size_t bytes, void* stream);
/* One FAC cycle in place on (xc, xf) with right-hand side (bc, bf) (both NULL = 0), noise
 * counters (seed, cycle); with_noise == 0 gives the deterministic cycle. */
int smg_composite_cycle(smg_composite* h, void* xc, void* xf, const void* bc, const void* bf,
                        uint64_t seed, uint64_t cycle, int32_t with_noise, void* stream);
/* ncycles stochastic cycles with b = 0 in place, cycle indices first_cycle, first_cycle+1, ... */
int smg_composite_sample(smg_composite* h, int64_t ncycles, uint64_t seed, uint64_t first_cycle,
                         void* xc, void* xf, void* stream);
/* (rc, rf) = (bc, bf) - A (xc, xf); rc is written on every base cell, 0 on covered cells. */
int smg_composite_residual(smg_composite* h, const void* xc, const void* xf, const void* bc,
                           const void* bf, void* rc, void* rf, void* stream);
/* Solves A u = f from u = 0 with noise-free cycles until ||f - A u||_2 <= rtol ||f||_2 (norms
 * over the composite unknowns; covered entries of fc are ignored).  Synchronises `stream`
 * after every cycle.  Errors as smg_solve. */
int smg_composite_solve(smg_composite* h, const void* fc, const void* ff, void* uc, void* uf,
                        double rtol, int32_t max_cycles, void* stream, smg_solve_info* info);
/* Field noise for a non-symmetric discretization (Appendix A).  On the composite mesh L = M^-1 S
 * (M the diagonal of cell volumes) is not symmetric, and for a forcing Q = diag(q) that is not
 * proportional to volume^-1/2 neither is L^-1 C (C the stationary covariance, L C + C L^T =
 * -Q Q^T).  The appendix's noise covariance -(L^-1 C + C L^-T) equals L^-1 Q Q^T L^-T, so a
 * draw is w = L^-1 Q eta with eta ~ N(0, I): this call forms b = -(volume/h^3) q eta (volume/h^3
 * = 1 on coarse cells, 1/8 on fine cells) and solves A w = b like smg_composite_solve, once per
 * draw.  Draw i uses eta from the streams (seed, counter cycle first_sample + i, level 0, slot 0,
 * colour 0 for the coarse part with site = base cell, colour 1 for the fine part with site =
 * fine index, component 0, kind 5).
 * qc: base-grid float64 amplitudes (covered entries ignored), qf: fine-box float64 amplitudes,
 * each NULL = 1.  wc: n x base_cells float64 (covered entries written 0), wf: n x fine_cells
 * float64, the draws one after another.  infos: NULL or n records.  Uses the workspace's
 * right-hand-side fields, so calls on one composite must not overlap.  Synchronises `stream`
 * after every cycle.  Errors: SMG_EINVAL (arguments), SMG_ENOTCONV (a draw's solve did not
 * reach rtol in max_cycles; earlier draws are complete), SMG_ENONFINITE, SMG_EHIP. */
int smg_composite_forced_field(smg_composite* h, int64_t n, uint64_t seed, uint64_t first_sample,
                               const void* qc, const void* qf, void* wc, void* wf, double rtol,
                               int32_t max_cycles, void* stream, smg_solve_info* infos);
/* Component entry points for the parity tests: one class pass (0..11) of a composite sweep;
 * one block-colour pass (0..7) on base level `level` (x, b natural layout of that level, b
 * NULL = 0); the stored row of base cell `cell` on level `level` (host only, up to 125
 * entries: absolute target cells and coefficients). */
int smg_composite_debug_pass(smg_composite* h, int32_t cls, void* xc, void* xf, const void* bc,
                             const void* bf, uint64_t seed, uint64_t cycle, int32_t slot,
                             int32_t with_noise, void* stream);
int smg_composite_debug_base_pass(smg_composite* h, int32_t level, int32_t colour, void* x,
                                  const void* b, uint64_t seed, uint64_t cycle, int32_t slot,
                                  int32_t with_noise, void* stream);
int smg_composite_debug_row(const smg_composite* h, int32_t level, int64_t cell,
                            int64_t* targets, double* vals, int32_t* count);
void smg_composite_destroy(smg_composite* h);

/* ==== Two-dimensional wall-bounded grid ==================================================
 * The paper compares the multigrid sampler with stochastic Gauss-Seidel on 2D and 3D meshes
 * (Sec. "Performance of the Stochastic Samplers in Practice").  Cells (x, z) of width h on
 * nx x nz, periodic in x, no-slip walls on the faces z = 0 and z = nz h (antisymmetric ghost);
 * A = -L the 5-point operator.  Level 0 smooths by a red-black point heat bath (nx even); a
 * Galerkin level (A_{l+1} = P^T A_l P, bilinear P) by a 2 x 2 block heat bath with block colour
 * (bx % 2) + 2 (bz % 2) when nx_l % 4 == 0 and nz_l is even; the coarsest level is drawn exactly
 * (dense Cholesky, <= 4096 unknowns) or smoothed (coarsest_mode); levels as for the 3D grid
 * (0 = coarsen while a level has more than coarsest_max unknowns).  With levels = 1 and
 * SMG_COARSEST_SMOOTH the chain is the plain stochastic Gauss-Seidel sampler.  Fields: device
 * float64 [ncomp][nz][nx]; components are independent chains (comp id in the noise counter:
 * site pair, level | slot<<4 | colour<<12 | comp<<16 | kind<<24, cycle; level-0 site =
 * (x + nx z) >> 1, block-level site = 4 block + in-block index dx + 2 dz, coarsest site = row). */
typedef struct smg2d smg2d;
typedef struct {
  int32_t nx, nz, ncomp;
  double h, kT;
  int32_t levels, nu1, nu2, coarsest_max, coarsest_mode;
  int32_t stride;       /* cycles per emitted sample (>= 1) */
} smg2d_desc;
typedef struct {
  size_t workspace_bytes;
  int32_t n_levels;
  int32_t dims[16][2];  /* (nx, nz) per level, finest first */
} smg2d_info;
/* Plans the 2D hierarchy on the host.  Errors: SMG_EINVAL (shape or parameters). */
int smg2d_create(const smg2d_desc* desc, smg2d** out);
int smg2d_get_info(const smg2d* h, smg2d_info* info);
/* Binds caller-owned device memory (>= workspace_bytes, 256-byte aligned), uploads the tables
 * on `stream` and synchronises it. */
int smg2d_bind(smg2d* h, void* ws, size_t bytes, void* stream);
/* n * stride cycles from `state` (read, and written at the end), cycle indices first_cycle, ...;
 * out[i] (device [n][ncomp][nz][nx]) receives the field after cycle (i + 1) * stride. */
int smg2d_sample(smg2d* h, int64_t n, uint64_t seed, uint64_t first_cycle, void* state,
                 void* out, void* stream);
/* A u = f by noise-free cycles from u = 0 until the largest relative residual over the
 * components is <= rtol; synchronises every cycle.  Errors as smg_solve. */
int smg2d_solve(smg2d* h, const void* f, void* u, double rtol, int32_t max_cycles, void* stream,
                smg_solve_info* info);
void smg2d_destroy(smg2d* h);

/* ==== SELM coupling of elastic structures to the wall-bounded Stokes fluid ===============
 * Sec. "Stochastic Eulerian-Lagrangian Method for Fluid-Structure Interactions", Sec.
 * "Discretization of SELM Hydrodynamic Coupling Tensor", Sec. "Generation of the Stochastic
 * Driving Fields Accounting for Thermal Fluctuations" and the algorithm "Stochastic Dynamics of
 * Elastic Structures with Hydrodynamic Coupling".  Fluid: three cell-centred velocity
 * components on the grid of smg_grid_desc (periodic x, y; no-slip walls on the z faces), each
 * with the viscous operator L = -mu A.  Structure points X: device float64 [m][3] positions with
 * 0 < z < nz h (points outside get zero weights).
 *   P = I - D^T A^-1 D with D = delta_x u_x + delta_y u_y + a_z^{1/2} u_z (periodic forward
 *     differences, the symmetric square root of the 1D wall operator), so D D^T = A: P is
 *     symmetric, idempotent, D P = 0, and P commutes with L (the properties the paper asks of
 *     the discrete projection); applying it takes one multigrid solve to rtol.
 *   Gamma: Peskin's 4-point interpolation (cells beyond a wall enter as antisymmetric ghosts);
 *     Lambda = alpha Gamma^T with alpha = 1/h^3.
 *   H F = -Gamma P L^-1 P Lambda F (eq. H_selm_discr); g = sqrt(2 kT alpha) Gamma P xi with
 *     xi ~ N(0, A^-1 / mu) drawn by the stochastic multigrid chain, so <g g^T> = 2 kT H
 *     (eqs. G_special_form, g_gen_xi).
 *   Step: X <- X + dt H(X) F + sqrt(dt) g(X) (Euler-Maruyama), F given by the caller. */
typedef struct smg_selm smg_selm;
typedef struct {
  int32_t nx, ny, nz;   /* fluid grid: nx, ny even */
  double h, mu, kT;     /* grid width, viscosity, temperature */
  int32_t levels;       /* multigrid depth (0: automatic, coarsest <= 512 unknowns) */
  int32_t stride;       /* chain cycles between successive driving fields (>= 1) */
  int32_t max_points;   /* largest number of structure points per call */
} smg_selm_desc;
typedef struct {
  size_t workspace_bytes;  /* device bytes smg_selm_bind needs */
  size_t state_bytes;      /* bytes of the driving-field chain state: 3 nx ny nz float64 */
  int32_t n_levels;
} smg_selm_info;
/* Plans the two hierarchies (the 3-component sampler/solver and the scalar projection solve)
 * and the square root of the wall operator (from its closed-form eigenvectors).  Host only. */
int smg_selm_create(const smg_selm_desc* desc, smg_selm** out);
int smg_selm_get_info(const smg_selm* s, smg_selm_info* info);
/* Binds caller-owned device memory (>= workspace_bytes, 256-byte aligned), uploads the tables
 * on `stream` and synchronises it. */
int smg_selm_bind(smg_selm* s, void* ws, size_t bytes, void* stream);
/* pu = P u for a velocity field u [3][nz][ny][nx] (pu may be u).  Synchronises (solve). */
int smg_selm_project(smg_selm* s, const void* u, void* pu, double rtol, void* stream);
/* V = H F for m points (X, F, V device float64 [m][3]).  Synchronises (solves). */
int smg_selm_mobility(smg_selm* s, int32_t m, const void* X, const void* F, void* V, double rtol,
                      void* stream);
/* g = sqrt(2 kT alpha) Gamma P xi: advances the driving-field chain `state` (device, state_bytes,
 * zero for a new chain) by `stride` cycles of the stochastic multigrid sampler (noise counters
 * from seed and first_cycle) and projects and interpolates its field.  Synchronises. */
int smg_selm_drive(smg_selm* s, int32_t m, const void* X, uint64_t seed, uint64_t first_cycle,
                   void* state, void* g, double rtol, void* stream);
/* One Euler-Maruyama step: X <- X + dt H F + sqrt(dt) g with g from the chain at cycle
 * step * stride.  Errors: SMG_EINVAL, SMG_ESTATE, SMG_EHIP, SMG_ENOTCONV (a solve). */
int smg_selm_step(smg_selm* s, int32_t m, void* X, const void* F, double dt, uint64_t seed,
                  uint64_t step, void* state, double rtol, void* stream);
void smg_selm_destroy(smg_selm* s);

#ifdef __cplusplus
}
#endif
#endif /* SMG_H */
