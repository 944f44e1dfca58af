/*
 * lsr.h - C ABI of the narrow-band semi-Lagrangian level-set solver for
 * surface reconstruction from point clouds on AMD Instinct MI355X (gfx950).
 *
 * Method: S. Preda and M. Semplice, "Surface reconstruction from point cloud
 * using a semi-Lagrangian scheme with local interpolator", arXiv:2410.22205.
 * The library runs Algorithm 1: the distance field to the cloud (Sections 2
 * and 3.4, exact, or the paper's approximation), the initial data (3.6, from
 * the cloud or in closed form), the narrow band (3.8), the energy functional
 * and its p = 2 regime (3.5), the semi-Lagrangian update with Q1 or tensor
 * WENO interpolation (3.1, 3.2), the reinitialisation plus cut (3.7, 3.8), the
 * stopping test and the multi-run coarse-to-fine schedule (Section 4).
 *
 * General rules
 *  - Every function returns an lsr_status; none throws.  On failure the job is
 *    left as it was and lsr_last_error() describes the cause.
 *  - Device memory for data is owned by the caller: lsr_create and
 *    lsr_batch_create carve the caller's workspace (sizes from
 *    lsr_workspace_bytes, lsr_batch_workspace_bytes) and never allocate
 *    device memory for data themselves.  The library creates only HIP
 *    objects: events, a second stream per batch (lsr_batch_set_streams)
 *    and instantiated graphs of step loops (lsr_set_graphs), whose memory
 *    the HIP runtime manages.  Pointers marked "device" are HIP device
 *    pointers.
 *  - All device work is enqueued on the caller's HIP stream given to
 *    lsr_create (a batch's on its own stream, with its second stream
 *    joined back into it within every call); only calls that return
 *    host-side values from the device (the loads' input checks, the
 *    convergence tests of lsr_load_cloud_approx and lsr_init_phi_cloud,
 *    lsr_extract with n_band, lsr_energy, lsr_run_to_steady,
 *    lsr_cloud_spacing, lsr_counters, lsr_profile_read, lsr_batch_tune)
 *    and the switches of the graph, stream and timing hooks synchronise
 *    that stream.
 *  - Nodal arrays are in C order: 2D index i*n[1] + j, 3D index
 *    (i*n[1] + j)*n[2] + k, axis 0 <-> x.  Node (i,j,k) sits at
 *    lo + (i,j,k)*h.
 *  - A job is used from one host thread at a time.
 */
#ifndef LSR_H
#define LSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSR_OK = 0,
  LSR_E_INVALID = -1,     /* bad argument (shape, parameter, non-finite input) */
  LSR_E_NOMEM = -2,       /* workspace too small */
  LSR_E_DEVICE = -3,      /* HIP error; text in lsr_last_error() */
  LSR_E_STATE = -4,       /* call out of order (e.g. step before init_phi) */
  LSR_E_UNSUPPORTED = -5  /* valid but not implemented (p other than 1 or 2; a batch
                             mixing dimensions or precisions) */
} lsr_status;

/* Interpolation operator I[phi] of Section 3.2. */
typedef enum { LSR_Q1 = 0, LSR_WENO = 1 } lsr_interp;

/* Precision of the state (phi, the packed distance gradient) and of the
 * arithmetic of the step and reinitialisation kernels.  The distance field
 * itself is always computed in double. */
enum { LSR_FP32 = 0, LSR_FP64 = 1 };

/* Initial-data kinds for lsr_init_phi. */
enum { LSR_PHI_ARRAY = 0, LSR_PHI_SPHERE = 1, LSR_PHI_TORUS = 2 };

/* Uniform Cartesian grid (Section 3): dim 2 or 3, n[a] >= 4 nodes per axis
 * (the WENO stencil spans 4 nodes), n[2] ignored in 2D, node spacing h > 0.
 * Limits: total nodes < 2^32 and the per-axis index bit widths sum to <= 32. */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double lo[3];
  double h;
} lsr_grid;

/* Parameters (see lsr_params_default for the values the paper uses). */
typedef struct {
  double p;          /* energy exponent of Section 2: 1 or 2 (the values the
                        paper runs; else LSR_E_UNSUPPORTED).  For p = 2 every
                        step first computes E_2 of the current phi (Section
                        3.5, R = 5; see lsr_energy) on the device and scales
                        the update's C by d / E_2; E_2 = 0 (no front) stops
                        the motion */
  double delta;      /* curvature weight, eq. (levelset:pde); >= 0 */
  double gamma;      /* narrow-band half width, eq. (subgrid); band |phi| < gamma */
  double beta;       /* cut-off inner radius, eq. (cutoff); 0 < beta < gamma */
  double grad_C;     /* degenerate-gradient threshold C dt^alpha, Section 3.1 */
  double grad_alpha;
  int32_t reinit_every;  /* reinitialise after every K-th step (0: never) */
  int32_t reinit_iters;  /* forward-Euler pseudo-time iterations per reinit */
  double reinit_dtau;    /* pseudo-time step, <= h/sqrt(dim) */
  double interface_floor;/* lower bound on |grad phi| in the interface fix */
  int32_t precision;     /* LSR_FP32 or LSR_FP64 */
} lsr_params;

typedef struct lsr_job lsr_job;
typedef struct lsr_batch lsr_batch;

/* Device counters returned by lsr_counters (cumulative since init_phi). */
enum {
  LSR_CNT_NODE_UPDATES = 0, /* sum over steps of the band size |G~^n| */
  LSR_CNT_FALLBACKS = 1,    /* updates through eq. (SL:2) */
  LSR_CNT_FRAME0 = 2,       /* 3D updates with the regularised frame (e1, e3) */
  LSR_CNT_REINITS = 3,      /* reinitialisations run */
  LSR_CNT_GBAR = 4,         /* sum of |band + face neighbours| over reinits */
  LSR_CNT_INTERFACE = 5,    /* sum of interface-set sizes over reinits */
  LSR_CNT_STEPS = 6,        /* steps run */
  LSR_CNT_COUNT = 7
};

/* Paper values for a grid of spacing h: p = delta = 1; gamma = 4h, beta = 2h
 * in 2D and gamma = 6h, beta = 3h in 3D (Section 3.8); C = 1e-3, alpha = 1
 * (Section 3.1); reinitialisation after every step in 2D and every 10th in
 * 3D, pseudo-time step h/2, ceil((gamma + h)/dtau) iterations, floor 1e-3
 * (Section 3.7 gives no values; these are this library's choice);
 * precision LSR_FP32. */
lsr_status lsr_params_default(int32_t dim, double h, lsr_params* out);

/* Device workspace a job needs for this grid, these parameters (only the
 * precision matters; NULL means LSR_FP32) and at most max_points cloud
 * points. */
lsr_status lsr_workspace_bytes(const lsr_grid* grid, const lsr_params* params, int64_t max_points,
                               size_t* bytes);

/* Create a job on the current HIP device.  dev_workspace: device memory of
 * at least lsr_workspace_bytes bytes, 256-byte aligned, owned by the caller
 * and untouched by other work while the job lives.  hip_stream: a
 * hipStream_t (NULL = default stream).  Enqueues the clearing of the
 * workspace.  LSR_E_INVALID on a bad grid or parameters, LSR_E_NOMEM if the
 * workspace is too small, LSR_E_UNSUPPORTED for p other than 1 or 2. */
lsr_status lsr_create(const lsr_grid* grid, const lsr_params* params, void* dev_workspace,
                      size_t ws_bytes, void* hip_stream, lsr_job** out);

/* Distance field of Section 2, d(x) = min_Q |x - Q|, computed exactly at
 * every node from the cloud.  dev_xyz: device, n x dim doubles, row major;
 * it is copied into the workspace and may be freed afterwards.  Every point
 * must be finite and inside the grid's box (Algorithm 1, step 1: the grid
 * encompasses the cloud); otherwise LSR_E_INVALID, and the stored cloud and
 * distance field are left as they were (the points are checked before
 * anything is written).  Synchronises the stream twice: to check the points
 * and to choose the bin width.  The current phi and band are kept. */
lsr_status lsr_load_cloud(lsr_job* job, const double* dev_xyz, int64_t n);

/* The paper's approximate distance field (Section 3.4): the exact distance
 * to the cloud at the nodes of the box of 4 nodes per axis around each point
 * (the two nodes on either side of the cell holding it, clamped to the
 * grid), and elsewhere the solution of the first-order Godunov
 * discretisation of |grad d| = 1 that Zhao's fast sweeping computes from
 * those nodes (reached here by tiled passes to the same fixed point).
 * Arguments, checks and synchronisations as lsr_load_cloud, plus one
 * synchronisation per four passes of the solve; LSR_E_DEVICE if the solve
 * does not settle within about eight passes per node along the axes. */
lsr_status lsr_load_cloud_approx(lsr_job* job, const double* dev_xyz, int64_t n);

/* Test and restart hook: use the given distance field instead of a cloud.
 * dev_d: device, one double per node, C order, finite and >= 0 (not
 * checked).  The current phi and band are kept. */
lsr_status lsr_set_distance(lsr_job* job, const double* dev_d);

/* Copy the distance field (double, as computed) to dev_out (device, one
 * double per node, C order). */
lsr_status lsr_get_distance(lsr_job* job, double* dev_out);

/* Initial data phi^0 (Algorithm 1, step 3), cut to [-gamma, gamma] by
 * eq. (cut), and the first band.  kind LSR_PHI_ARRAY: dev_phi0 (device, one
 * value per node in the job's precision, C order) is copied; LSR_PHI_SPHERE: signed distance to the
 * sphere (circle in 2D) with centre args[0..2] and radius args[3];
 * LSR_PHI_TORUS (3D): torus with axis z, centre args[0..2], radii R = args[3],
 * r = args[4].  args is host memory.  step0 is the global index of the next
 * step, which fixes the reinitialisation phase after a restart. */
lsr_status lsr_init_phi(lsr_job* job, const void* dev_phi0, int32_t kind, const double* args,
                        int64_t step0);

/* Initial data from the cloud (Section 3.6) from the job's distance field d
 * and the threshold gamma_s > 0 (the paper: gamma_S = K_S h_S, K_S = 2 by
 * default, Section 4): nodes on the grid's boundary with d >= gamma_s are
 * external, and so is every node with d >= gamma_s reachable from them
 * through face neighbours that are; phi0 = d - gamma_s there; on the other
 * nodes phi0 = -u with u the fast-sweeping solution of |grad u| = 1 from the
 * external values (first-order Godunov, the external nodes held fixed;
 * 1e30 where no external node leads); cut to [-gamma, gamma] as in
 * lsr_init_phi, with the first band.  step0 as in lsr_init_phi.  LSR_E_STATE
 * without a distance field; one synchronisation per four passes of the
 * marking and of the solve; LSR_E_DEVICE if either does not settle (see
 * lsr_load_cloud_approx). */
lsr_status lsr_init_phi_cloud(lsr_job* job, double gamma_s, int64_t step0);

/* Warm start of a finer run (Section 4, after eq. dxdt): phi0 at every node
 * x of the job's grid is I[phi](x) with phi the current phi of `coarse` (a
 * job of the same dimension and precision on another grid) and I the
 * interpolator `interp` (Section 3.2; a node outside coarse's box is moved
 * onto it), cut to [-gamma, gamma], with the first band.  The job's stream
 * is ordered after the work queued on coarse's, and coarse's after the
 * read.  step0 as in lsr_init_phi. */
lsr_status lsr_init_phi_resample(lsr_job* job, const lsr_job* coarse, lsr_interp interp,
                                 int64_t step0);

/* Grid, parameters and time step of run r >= 1 of the coarse-to-fine
 * schedule (Section 4) for a cloud with bounding box [box_lo, box_hi] (host,
 * dim values each) and resolution h_s (see lsr_cloud_spacing): dx = h_s /
 * 2^(r-1) and dt = dx / 4 (eq. dxdt); p = 1, delta = 0 in run 1, p = 2,
 * delta = 0 in run 2 and p = 2, delta = 1 after (Table param); the other
 * parameters as lsr_params_default(dim, dx).  The grid (the paper says only
 * that it encompasses the cloud; these sizes reproduce every grid the paper
 * lists): per axis ceil(extent / dx) + 1 nodes plus m on each side, node 0
 * at box_lo - m dx, with m the band half width in cells plus 4, and in run 1
 * also ceil(k_s h_s / dx) (the threshold gamma_S = k_s h_s of the initial
 * data).  Host only. */
lsr_status lsr_schedule_run(int32_t r, int32_t dim, const double* box_lo, const double* box_hi,
                            double h_s, double k_s, lsr_grid* grid, lsr_params* params,
                            double* dt);

/* n_steps iterations of Algorithm 1's loop: band (eq. subgrid, read as
 * |phi| < gamma), the update of eqs. (SL2d)/(SL3d) with the cut-off factor of
 * Section 3.8 and the fallback of eq. (SL:2), the cut of eq. (cut) and, after
 * every step whose global index s satisfies (s + 1) % reinit_every == 0, the
 * reinitialisation on the pre-update band plus its face neighbours.  dt > 0.
 * Enqueued on the stream; returns before the work finishes. */
lsr_status lsr_step(lsr_job* job, int32_t n_steps, double dt, lsr_interp interp);

/* One reinitialisation (Section 3.7) plus cut, on the current band and its
 * face neighbours, outside the step loop. */
lsr_status lsr_reinit(lsr_job* job);

/* Energy functional E_p(phi) of Section 3.5 of the current phi with the
 * job's distance field: over the front cells (the cells whose vertices do
 * not all lie on one side of the front, a vertex being inside when
 * phi < 0), in 2D the trapezoidal rule on the segment between the linear
 * edge crossings (eq. energyApprox), in 3D the sum of |d|^p h'^2 over the R^3
 * subcells of side h' = h / R per front cell whose trilinear phi at the
 * centre lies within (sqrt 3 / 2) h' of zero (eq. energyApproxFiner; the
 * paper uses R = 5).  Computed in double over every cell of the grid (the
 * job keeps one sign bit per node, which shows the front cells 32 at a
 * time).  *out (host) receives E_p.  p:
 * finite, > 0; R: 1..64 (ignored in 2D); else LSR_E_INVALID.  LSR_E_STATE
 * without phi or d, or for a job in a batch.  Synchronises the stream. */
lsr_status lsr_energy(lsr_job* job, double p, int32_t R, double* out);

/* Cloud resolution h_S (Section 4, the text after eq. dxdt): the mean over
 * the sampled points of the distance to their nearest neighbour in the
 * cloud loaded by lsr_load_cloud (the second smallest distance counting the
 * point itself; an exact duplicate is a neighbour at distance 0).
 * dev_sample: device, n_sample indices into the cloud as it was given (the
 * paper draws a random 10 %; the caller draws them), 1 <= n_sample <=
 * max_points.  *out (host) receives h_S.  LSR_E_STATE without a loaded
 * cloud of at least two points or for a job in a batch; LSR_E_INVALID for
 * an index outside the cloud.  Synchronises the stream. */
lsr_status lsr_cloud_spacing(lsr_job* job, const int64_t* dev_sample, int64_t n_sample,
                             double* out);

/* Stopping test of eq. (deltaEn) after iteration n.  e (host): E_2(phi^i)
 * for i = 0..n.  With k = min(n, LSR_ENERGY_WINDOW) and e_m the mean of the
 * k values ending at m, returns 1 when |e_(n-1) - e_n| / e_n < tol (n >=
 * min_steps) or when n >= max_steps, else 0; -1 for e NULL or n < 0.  Both
 * means use the same k, so the one at n - 1 reaches back to phi^0 while
 * n <= LSR_ENERGY_WINDOW; a zero mean stops.  Host only (no device work). */
#define LSR_ENERGY_WINDOW 10
int32_t lsr_energy_stop(const double* e, int32_t n, int32_t min_steps, int32_t max_steps,
                        double tol);

/* Steps the job one step at a time until lsr_energy_stop says stop (the
 * paper: min_steps 10, max_steps 100, tol 1e-4), computing E_2 (R = 5) of
 * phi^0 and after every step; synchronises the stream once per step.
 * *n_done: steps taken; energies (host, may be NULL): room for
 * max_steps + 1 values, receives E_2(phi^0..phi^n_done).  Errors as
 * lsr_step and lsr_energy, LSR_E_INVALID for bad limits. */
lsr_status lsr_run_to_steady(lsr_job* job, double dt, lsr_interp interp, int32_t min_steps,
                             int32_t max_steps, double tol, double* energies, int32_t* n_done);

/* Copy out the current phi (dev_phi: device, one value per node in the job's
 * precision) and the band
 * mask (dev_band: device, one byte per node, 1 iff |phi| < gamma); either may
 * be NULL.  If n_band is not NULL the stream is synchronised and the band
 * size stored there; step_index (may be NULL) receives the global index of
 * the next step. */
lsr_status lsr_extract(lsr_job* job, void* dev_phi, uint8_t* dev_band, int64_t* n_band,
                       int64_t* step_index);

/* Read up to n cumulative counters (LSR_CNT_*) into host memory; syncs. */
lsr_status lsr_counters(lsr_job* job, int64_t* out, int32_t n);

/* Destroy the host-side job object.  Does not free the workspace; waits for
 * the job's queued work to finish. */
lsr_status lsr_destroy(lsr_job* job);

/* Batched execution of independent jobs on one device (one dimension and one
 * precision per batch).  A batch step launches each kernel of the step once
 * for all member jobs (per-job arguments from packed tables in the batch's
 * workspace); every job keeps its own dt, interpolator, reinitialisation
 * phase and state, and its results are bitwise those of lsr_step on the job
 * alone with the same launch shape.  All work of a batch, including calls on
 * member jobs (lsr_extract, lsr_counters, ...), goes to the batch's stream.
 *
 * lsr_batch_workspace_bytes: device workspace for up to max_jobs members,
 * tables for group_steps steps per upload, members with at most
 * max_reinit_iters reinitialisation iterations.
 * lsr_batch_create: dev_workspace (device, caller-owned, 256-byte aligned),
 * hip_stream (NULL = default stream).  Host staging is pinned memory.
 * lsr_batch_add: the job joins at the next batch step, after the work
 * already queued on its own stream (no host synchronisation); a job in a
 * batch refuses lsr_step, lsr_reinit, lsr_init_phi, lsr_load_cloud,
 * lsr_set_distance, lsr_set_launch and lsr_destroy.  A p = 2 member gets
 * its own energy launch before each batched step.
 * lsr_batch_remove: the job leaves at the current step boundary; its own
 * stream is ordered after the batch's queued work.  Its state (phi, lists,
 * step index, reinitialisation phase) stays in its workspace, so it can be
 * stepped alone or added to a batch again and continues where it left.
 * lsr_batch_step: n_steps steps of every member (uploads one table per group).
 * lsr_batch_set_launch: launch shape as in lsr_set_launch.
 * lsr_batch_set_streams: members whose state does not fit the device's
 * last-level cache together are stepped in cache groups, each with its own
 * launches; with 2 streams (the default) every other group runs on a second
 * stream that the batch creates, forked from and joined back into the
 * batch's stream within each lsr_batch_step, so that groups overlap; 1 runs
 * all groups on the batch's stream.  Results are the same either way.
 * Synchronises the stream; other values give LSR_E_INVALID.
 * lsr_batch_set_graphs: 1 (default) records a group of steps whose launch
 * sequence was seen before (the same kernels, table offsets and job counts
 * per launch, and the same launch shape and stream count) as a HIP graph
 * and replays it for later such groups, whose tables are copied anew
 * before the replay; 0 launches every kernel directly.  Results are the
 * same either way.  Synchronises the stream.
 * lsr_batch_tune: times the next step under each candidate launch shape
 * (lanes per node, blocks per CU) without changing the jobs, keeps the
 * fastest and returns it with its time in ms (synchronises).  The choice is
 * kept for the process under the batch's signature (dimension, precision,
 * jobs per interpolator, total grid nodes rounded up to a power of two), and
 * in the file of lsr_set_tune_cache if one is set; a later call with the
 * same signature applies it without timing and returns the time measured
 * then.
 * lsr_batch_destroy: removes the members, waits for the stream and
 * releases the batch's graphs, second stream and events. */
lsr_status lsr_batch_workspace_bytes(int32_t max_jobs, int32_t group_steps, int32_t max_reinit_iters,
                                     size_t* bytes);
lsr_status lsr_batch_create(int32_t max_jobs, int32_t group_steps, int32_t max_reinit_iters,
                            void* dev_workspace, size_t ws_bytes, void* hip_stream,
                            lsr_batch** out);
lsr_status lsr_batch_add(lsr_batch* batch, lsr_job* job, double dt, lsr_interp interp);
lsr_status lsr_batch_remove(lsr_batch* batch, lsr_job* job);
lsr_status lsr_batch_step(lsr_batch* batch, int32_t n_steps);
lsr_status lsr_batch_set_launch(lsr_batch* batch, int32_t lanes, int32_t blocks_per_cu);
lsr_status lsr_batch_set_streams(lsr_batch* batch, int32_t n_streams);
lsr_status lsr_batch_set_graphs(lsr_batch* batch, int32_t enable);
lsr_status lsr_batch_tune(lsr_batch* batch, int32_t* lanes, int32_t* blocks_per_cu, double* ms);
/* Keep tuned launch shapes in a text file as well (path NULL or empty: in
 * the process only): the file's choices are read now (a missing file is an
 * empty one; choices already made in this process win), and every later
 * tuning appends its line: dimension, precision, Q1 jobs, WENO jobs, nodes
 * rounded up to a power of two, lanes, blocks per CU, time in ms.
 * LSR_E_INVALID for a malformed line (nothing is read then).  Host only. */
lsr_status lsr_set_tune_cache(const char* path);
lsr_status lsr_batch_destroy(lsr_batch* batch);

/* Launch shape of the list kernels (results are bitwise the same for every
 * shape): lanes = 1 (one lane per band node) or the number of foot points
 * per node (2 in 2D, 4 in 3D: one lane per foot point).  blocks_per_cu in
 * 1..64 bounds the persistent grid, which never exceeds the blocks of the
 * kernel that fit on the device at once.  Defaults: 1 lane, 8. */
lsr_status lsr_set_launch(lsr_job* job, int32_t lanes, int32_t blocks_per_cu);

/* Step loops as HIP graphs.  With enable = 1 (the default) lsr_step runs
 * whole chunks of 2 * reinit_every steps (16 without reinitialisation)
 * through recorded graphs: a chunk is recorded the second time the job
 * starts one in the same state (buffer roles, counter slots, phase in the
 * reinitialisation period, dt, interpolator, launch shape) and replayed after
 * that; the remaining steps, jobs on the null stream and step loops while
 * kernel timing is on (lsr_profile_enable) launch directly.  Results are the same either way.
 * Synchronises the stream and drops the recorded graphs. */
lsr_status lsr_set_graphs(lsr_job* job, int32_t enable);

/* Graphs recorded and replayed so far by a job's lsr_step or a batch's
 * lsr_batch_step (exactly one of job, batch non-NULL), into host memory. */
lsr_status lsr_graph_counts(lsr_job* job, lsr_batch* batch, int64_t* captured, int64_t* replayed);

/* Measurement hook.  While enabled, lsr_step launches directly and every
 * semi-Lagrangian step kernel of the job carries a pair of HIP events tied
 * to its dispatch (hipExtLaunchKernel), whose elapsed time is the kernel's
 * execution time; at most max_launches pairs, later launches are
 * not timed.  Enabling or disabling clears earlier records.
 * lsr_profile_read synchronises the stream and returns the summed kernel
 * time in milliseconds and the number of timed launches. */
lsr_status lsr_profile_enable(lsr_job* job, int32_t enable, int32_t max_launches);
lsr_status lsr_profile_read(lsr_job* job, double* total_ms, int64_t* launches);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * energy functional of lsr_energy (Section 3.5, same kernels up to the order
 * of summation) of nodal fields the caller holds, without a job or a
 * workspace.  grid: as for lsr_create (nodes < 2^32); dev_phi: device, one
 * value per node in `precision` (LSR_FP32 or LSR_FP64), C order; dev_d:
 * device, one double per node; p finite > 0; R in 1..64; dev_out: device,
 * one double, receives E_p.  The kernels' per-block partial sums live in a
 * file-scope device array of this library (1024 doubles, 8 KiB, one copy per
 * device, held until the process ends; every block writes its own slot on
 * every call, so nothing needs clearing); its address is taken once per
 * device, with that device current, on the first call.  Calls that overlap
 * on one device race on that array; calls on different devices do not.
 * Enqueued on hip_stream (NULL = default stream), no synchronisation, no
 * allocation.  LSR_E_INVALID for bad arguments, LSR_E_UNSUPPORTED for a
 * grid of 2^32 nodes or more or a device index above 63. */
lsr_status lsr_energy_noalloc(const lsr_grid* grid, int32_t precision, const void* dev_phi,
                              const double* dev_d, double p, int32_t R, double* dev_out,
                              void* hip_stream);

/* Text of the last error on this host thread; valid until the next call. */
const char* lsr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LSR_H */
