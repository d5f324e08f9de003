/* jetles.h -- C ABI of the MI355X jet-LES hot path.
 *
 * One solver object owns one structured curvilinear block of
 * ni x nj x nk nodes (xi = i streamwise, eta = j, zeta = k) resident in the
 * HBM of one GPU, and advances the filtered compressible Navier-Stokes
 * equations (Sec. 3 of arXiv:2003.09926, Eq. (les) with the closure of
 * Eqs. (q_mod), (sutherland), (tau_mod)) by the explicit five-stage
 * Runge-Kutta scheme (Sec. 3, closing paragraph; per-stage order of work in
 * Sec. 4.2 and its flow chart).  The spatial operator is the centred
 * second-order finite difference on curvilinear coordinates with anisotropic
 * scalar artificial dissipation (Sec. 3) on a five-point stencil (two ghost
 * layers, Sec. 4.3), plus a Smagorinsky subgrid viscosity.
 *
 * Conventions used by every entry point:
 *   - node (i, j, k) sits at linear index n = i + ni * (j + nj * k);
 *     N = ni * nj * nk;
 *   - a state is 5 x N doubles, structure of arrays, variable-major:
 *     q[v * N + n], v = rho, rho u, rho v, rho w, e (total energy per volume);
 *   - a metric set is 10 x N doubles: m[(3 d + a) * N + n] = S^d_a, the
 *     derivative of xi_d with respect to x_a divided by J, for d, a in
 *     {0, 1, 2}; m[9 * N + n] = J = 1 / det d(x, y, z) / d(xi, eta, zeta);
 *   - each direction is periodic (the wrap stands in for the neighbour
 *     ranks' ghost layers of Sec. 4.3) unless jz_params.bc gives its two
 *     faces physical boundary conditions (see jz_bc);
 *   - units: ambient rho = 1, p = 1/gamma, sound speed 1, jet diameter 1,
 *     mu_inf = mach_j / re_d, Sutherland reference temperature 1;
 *   - every function returns an int status (JZ_OK = 0, negative = error) and
 *     never throws; jz_last_error() gives a thread-local message;
 *   - host arrays are owned by the caller and only read (or written) during
 *     the call; "on_device" arguments select a device pointer instead;
 *   - all GPU work is issued on the solver's stream in call order; only the
 *     jz_get_* calls and the calls that validate input synchronise it.
 */
#ifndef JETLES_H
#define JETLES_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  JZ_OK = 0,
  JZ_EINVAL = -1,     /* null pointer, size < 1, bad parameter, workspace too small, bad grid */
  JZ_ENOMEM = -2,     /* device allocation failed */
  JZ_EHIP = -3,       /* HIP runtime error; message in jz_last_error() */
  JZ_ENONFINITE = -4, /* NaN/Inf in the state or residual norms, or dt <= 0 */
  JZ_ESTATE = -5      /* call out of order (advance before grid and state are set) */
};

typedef struct jz_solver jz_solver; /* opaque, library-owned */

typedef enum { JZ_FP64 = 0, JZ_FP32_FLUX = 1 } jz_precision;

/* Boundary types of the six faces, indexed xi-, xi+, eta-, eta+, zeta-,
 * zeta+ in jz_params.bc (Sec. 3, boundary conditions).  A direction is
 * either periodic at both faces or bounded at both.  Along a bounded
 * direction (at least 5 nodes) the two outermost node layers at each end are
 * boundary layers: the residual advances only the nodes between them, and
 * after every Runge-Kutta stage the layers are set by their face's rule --
 *   JZ_BC_INFLOW:   supersonic inflow (the jet exit): the layer keeps the
 *                   state it was given by jz_set_state;
 *   JZ_BC_FARFIELD: far field from Riemann invariants: the state of the
 *                   first interior node along the face normal (index 2, or
 *                   n-3) and the free stream (rho = 1, u = (mach_inf, 0, 0),
 *                   p = 1/gamma) give the outgoing and incoming invariants
 *                   u_n +- 2a/(gamma-1); entropy and tangential velocity come
 *                   from the upwind side; a supersonic normal flow takes all
 *                   values from its upwind side.  Both layers get that state.
 *   JZ_BC_AXIS:     the centreline of a cylindrical mesh (eta- face only,
 *                   zeta periodic: eta = radius index, j = 0 on the axis,
 *                   zeta = azimuth): ring j = 1 takes the state of ring j = 2
 *                   (extrapolation from the adjacent ring, per azimuth); every
 *                   axis node j = 0 takes the average over all nk azimuths of
 *                   ring j = 2, summed in the order k = 0..nk-1 (bitwise the
 *                   same value for all k).  Axis nodes have no metrics (zero
 *                   cell volume); they are never used and not validated.
 * A node in the layers of an inflow face is always held; otherwise the
 * bounded directions are processed in the order xi, eta, zeta, so a node in
 * the layers of several directions keeps the last one's value.  Residual
 * norms and the CFL maximum run over the advanced nodes only; jz_eval_residual
 * returns 0 on boundary layers.  Batches take periodic blocks only. */
typedef enum { JZ_BC_PERIODIC = 0, JZ_BC_INFLOW = 1, JZ_BC_FARFIELD = 2, JZ_BC_AXIS = 3 } jz_bc;

/* Physical and numerical parameters.  Values the paper leaves open carry the
 * defaults of jz_params_default(); the paper fixes Pr = 0.72 (Sec. 3) and the
 * number of stages (5, Sec. 3). */
typedef struct {
  double gamma;        /* ratio of specific heats (1.4) */
  double prandtl;      /* molecular Prandtl number (0.72) */
  double prandtl_t;    /* subgrid Prandtl number (0.9) */
  double mach_j;       /* jet Mach number; also the velocity scale of mu_inf */
  double re_d;         /* jet Reynolds number; +inf or <= 0 gives mu_inf = 0 */
  double sutherland_s; /* Sutherland constant / reference temperature (110.4/288.15) */
  double cs;           /* Smagorinsky constant (0.17); 0 switches the SGS model off */
  double k2, k4;       /* dissipation coefficients (1/4, 1/64) */
  double tv_alpha;     /* anisotropic scaling exponent (0.5) */
  double cfl;          /* Courant number of the global time step (0.5) */
  double dt_fixed;     /* > 0: fixed time step instead of the CFL rule (0) */
  double rk_alpha[5];  /* stage coefficients (1/4, 1/6, 3/8, 1/2, 1) */
  int n_stages;        /* 1..5 (5); with one stage (forward Euler) the stage writes a
                          stage buffer that is then copied into the state */
  int precision;       /* jz_precision (JZ_FP64) */
  int tile_i, tile_j;  /* launch shape of the stage kernel; 0 = library default */
  int kchunk;          /* planes marched per workgroup; 0 = chosen by the library for
                          the current device (fills the last round of workgroups) */
  int bc[6];           /* jz_bc of the faces xi-, xi+, eta-, eta+, zeta-, zeta+ (all periodic) */
  double mach_inf;     /* free-stream velocity along x of the far field, in ambient
                          sound speeds (0) */
  int stats_interval;  /* > 0: accumulate time-averaged statistics of the state after
                          every stats_interval-th step of jz_advance (0: off; the
                          workspace then holds no statistics) */
} jz_params;

/* Fill *p with the defaults listed above. */
int jz_params_default(jz_params* p);

/* Bytes of device memory a solver of this size and precision needs when the
 * caller provides the workspace (see jz_create).  0 on invalid sizes. */
size_t jz_workspace_bytes(int ni, int nj, int nk, const jz_params* p);

/* Create a solver for an ni x nj x nk block (each >= 1).
 * dev_workspace: NULL = the library allocates (hipMalloc) and frees in
 *   jz_destroy; otherwise a device buffer of at least ws_bytes >=
 *   jz_workspace_bytes(...) bytes, 256-byte aligned, owned by the caller
 *   (for example a torch tensor) and kept alive until jz_destroy.
 * hip_stream: the hipStream_t all work is issued on (NULL = null stream).
 * The parameters are copied.  JZ_EINVAL on bad sizes/parameters. */
int jz_create(int ni, int nj, int nk, const jz_params* p, void* dev_workspace, size_t ws_bytes,
              void* hip_stream, jz_solver** out);

/* Geometry from node coordinates (host arrays x, y, z of N doubles each) and
 * the periodic shift vectors period[3 d + a] (the change of coordinate a when
 * index d wraps once forwards).  Computes the Thomas-Lombard metric set and J
 * on the GPU in FP64 (Sec. 3: curvilinear form; Sec. 4.2: metrics computed
 * once after the mesh is read).  Along a bounded direction the shifts are
 * ignored and the differences at its two end nodes are one-sided.  JZ_EINVAL
 * if any J is non-positive or not finite.  Synchronises. */
int jz_set_grid_coords(jz_solver* s, const double* x, const double* y, const double* z,
                       const double* period);

/* Geometry from a metric set computed elsewhere (10 x N, layout above), e.g.
 * the analytic metrics of a separable grid.  on_device selects a device
 * pointer.  JZ_EINVAL if any J is non-positive or not finite.  Synchronises. */
int jz_set_grid_metrics(jz_solver* s, const double* m, int on_device);

/* Copy the metric set (10 x N) out.  Synchronises. */
int jz_get_grid_metrics(jz_solver* s, double* m, int on_device);

/* Set the conserved state (5 x N).  JZ_ENONFINITE if it holds NaN/Inf,
 * JZ_EINVAL if rho or p is not positive somewhere; the previous state is then
 * kept.  The next step recomputes dt from this state.  Synchronises. */
int jz_set_state(jz_solver* s, const double* q, int on_device);

/* Advance nsteps explicit five-stage steps.  Each step takes
 * dt = cfl / max_nodes sum_d lambda^d from the state at its start (or
 * dt_fixed), runs the stages Q(k) = Q(0) - alpha_k dt R(Q(k-1)), records the
 * norms of the first-stage residual and advances the clock.  Asynchronous:
 * returns once the work is queued.  If a step produces NaN/Inf norms or a
 * non-positive dt, later kernels leave the state at that step and the next
 * jz_get_* call returns JZ_ENONFINITE. */
int jz_advance(jz_solver* s, int nsteps);

/* Copy the state (5 x N) out.  Synchronises; JZ_ENONFINITE after a failed step
 * (the state of the failing step is still copied). */
int jz_get_state(jz_solver* s, double* q, int on_device);

/* RMS and max-norm per conserved variable of R(Q^n) (the first stage of the
 * last step).  Synchronises. */
int jz_get_residual_norms(jz_solver* s, double rms[5], double linf[5]);

/* Simulated time, the step size the next step will use, and the step count.
 * Synchronises. */
int jz_get_clock(jz_solver* s, double* t, double* next_dt, long long* steps);

/* Set the simulated time and step count (checkpoint/resume). */
int jz_set_clock(jz_solver* s, double t, long long steps);

/* One evaluation of the residual R(Q) of the current state into r (5 x N),
 * with the same kernels the stages use.  Synchronises. */
int jz_eval_residual(jz_solver* s, double* r, int on_device);

/* Time step the CFL rule gives for the current state and the maximum of
 * sum_d lambda^d it came from.  Synchronises. */
int jz_eval_dt(jz_solver* s, double* dt, double* lambda_max);

/* Kernel timing with hipEvents on the solver's stream: enable = 1 starts
 * recording each stage-kernel launch of jz_advance, 0 stops (enabling creates
 * a pool of events up front, so that jz_advance creates none for the first
 * 640 launches).  jz_get_timing
 * synchronises and returns the summed milliseconds and launch count of the
 * stage kernels since timing was enabled, and the algorithmic HBM bytes of
 * those launches (each array read or written once per stage). */
int jz_set_timing(jz_solver* s, int enable);
int jz_get_timing(jz_solver* s, double* stage_ms, long long* stage_launches, double* stage_bytes);

/* Time-averaged statistics (Sec. 6: the time average of the axial velocity
 * <U> and the RMS of its fluctuation, from samples of the flow taken at a
 * fixed frequency; here also the pressure).  With jz_params.stats_interval =
 * m > 0 the library keeps, per node and in FP64, the sums of u, u^2, p and p^2
 * (u = rho u / rho, the x component; p from the equation of state) over the
 * samples, and jz_advance adds a sample of the new state after every m-th step
 * counted from creation or the last jz_stats_reset.  Not available in batches.
 * All four return JZ_ESTATE if statistics were not enabled. */
int jz_stats_reset(jz_solver* s);   /* clears the sums and the step count */
int jz_stats_sample(jz_solver* s);  /* adds a sample of the current state now */
/* Per-node mean and RMS of the fluctuation, sqrt(max(<x^2> - <x>^2, 0)), of u
 * and p (N doubles each; any pointer may be NULL; host arrays, or device
 * pointers when on_device) and the sample count.  JZ_ESTATE without samples.
 * Synchronises. */
int jz_get_stats(jz_solver* s, double* mean_u, double* rms_u, double* mean_p, double* rms_p, long long* nsamples,
                 int on_device);
/* Azimuthal average over the cross-section xi = i (Sec. 6: radial profiles of
 * the statistics averaged in the azimuthal direction).  bins (host, nj * nk
 * ints, entry j + nj k for node (i, j, k)) assigns each node of the section
 * to a bin 0..nbins-1 or -1 (not used); for every bin the node values of the
 * four statistics are averaged over its nodes, visited in the fixed order
 * k = 0.., j = 0.. (reproducible), and counts[b] is its node count.  Output
 * host arrays of nbins entries (any may be NULL).  Synchronises. */
int jz_stats_profile(jz_solver* s, int i, const int* bins, int nbins, double* mean_u, double* rms_u,
                     double* mean_p, double* rms_p, long long* counts);

/* Change the launch shape (tile_i x tile_j owned columns per workgroup, kchunk
 * planes marched per workgroup; 0 = default) of an existing solver.  Results
 * do not depend on it (each node's arithmetic is the same for every shape).
 * JZ_EINVAL for an unsupported shape. */
int jz_set_tiling(jz_solver* s, int tile_i, int tile_j, int kchunk);
int jz_get_tiling(jz_solver* s, int* tile_i, int* tile_j, int* kchunk);
/* Workgroups of the solver's stage kernel that one CU holds at once, and the
 * device's CU count (their product is one round of workgroups). */
int jz_get_occupancy(jz_solver* s, int* wg_per_cu, int* cus);

/* Release the solver (and the workspace if the library allocated it). */
int jz_destroy(jz_solver* s);

/* ---- batches: many uneven blocks advanced together ----------------------
 * A batch advances several solvers (its members, which keep their own
 * grids, states, clocks, dt and flags) with one persistent launch per RK
 * stage over the tiles of all members, and one finalize launch; the step is
 * captured once in a hipGraph and replayed.  Members must share precision,
 * stage count and coefficients, and a tile shape with a batch kernel
 * (FP64: 16x12, 32x8, 16x16, 28x12, 12x12; FP32-flux: 32x16, 28x20, 28x12, 12x12), and must have their
 * grid and state set.  Each member's results are bitwise those of the member
 * advanced alone with the same tile shape.  Members need n_stages >= 2 (JZ_EINVAL
 * otherwise).  The caller keeps ownership of the members, must not advance
 * them on their own while they belong to the batch, and must take a member
 * out (jz_batch_remove) or destroy the batch before destroying the member.
 * hip_stream orders the batch against the caller's work (NULL = null
 * stream); the batch runs on an internal non-blocking stream. */
typedef struct jz_batch jz_batch;
int jz_batch_create(jz_solver* const* members, int nmembers, void* hip_stream, jz_batch** out);
int jz_batch_advance(jz_batch* b, int nsteps);
/* Continuous batching: change the resident set between steps.  The step's
 * launches read the member table and the work list from device memory, so
 * the captured graph is replayed as it is (a new capture only when the
 * tables must grow beyond their slots, which double each time).  add: the
 * solver must match the batch (precision, stages, coefficients, tile shape;
 * periodic, no statistics; grid and state set; JZ_EINVAL / JZ_ESTATE
 * otherwise) and not be a member yet; it joins at the next jz_batch_advance
 * with its own clock (its set-up on its own stream is ordered before the
 * batch's next step).  remove: takes the member out; work issued afterwards
 * on the member's own stream follows the batch steps queued so far (the
 * last ones that include it); the caller keeps the solver.  Neither call
 * waits for the device: the table change is staged in pinned host memory
 * and queued behind the steps in flight (the call waits only when the
 * tables must grow, or when 32 earlier changes are still queued behind
 * unfinished steps).  A batch may be empty (its steps then do nothing).
 * members: the current member count. */
int jz_batch_add(jz_batch* b, jz_solver* s);
int jz_batch_remove(jz_batch* b, jz_solver* s);
int jz_batch_members(jz_batch* b);
/* Rebuild the member table after jz_set_tiling on members. */
int jz_batch_refresh(jz_batch* b);
/* 1 (default): replay a captured hipGraph per step; 0: launch directly. */
int jz_batch_set_graph(jz_batch* b, int enable);
/* Pick the fastest launch shape by timing trial_steps steps per candidate;
 * member states and clocks are restored afterwards.  cache_path (may be NULL)
 * names a text file of earlier choices keyed by the batch's shapes. */
int jz_batch_autotune(jz_batch* b, int trial_steps, const char* cache_path, int* tile_i, int* tile_j,
                      int* kchunk, double* best_step_ms);
/* Step timing with hipEvents: summed milliseconds and number of steps since
 * timing was enabled, and the total node count of the members. */
int jz_batch_set_timing(jz_batch* b, int enable);
int jz_batch_get_timing(jz_batch* b, double* step_ms, long long* steps, long long* points);
int jz_batch_synchronize(jz_batch* b);
int jz_batch_destroy(jz_batch* b);

/* ---- domains: one block split into padded sub-blocks ------------------
 * The one-device part of the paper's domain decomposition (Sec. 4.1, the
 * 2-D partitioning of Fig. comm_2d and its balancing rule; Sec. 4.3, the
 * two-layer ghost fringe of Fig. ghost).  A periodic ni x nj x nk block is
 * split into parts_i parts along xi and parts_k along zeta (eta whole);
 * the part sizes along a direction differ by at most one node, the larger
 * parts first.  Each part is a solver of its own with two ghost layers at
 * both ends of each split direction, which it reads but does not advance;
 * after every RK stage halo-copy kernels refill them from the neighbouring
 * parts' stage results (periodic wrap between the first and last part),
 * first along xi over all zeta layers, then along zeta over the whole
 * padded xi width, which carries the corners.  dt is the CFL rule over all
 * parts, the norms are summed over all parts, and the states are bitwise
 * those of the unsplit block advanced with jz_advance.
 *   p:    all six faces JZ_BC_PERIODIC, stats_interval 0, n_stages >= 2;
 *   parts_i, parts_k >= 1, every part at least 2 nodes long;
 *   hip_stream: all work is ordered on it (NULL = null stream).
 * set_grid_metrics / set_state take the whole block's host arrays in the
 * jz_set_grid_metrics / jz_set_state layouts (10 x N and 5 x N doubles);
 * get_state writes the whole block's 5 x N host array.  get_clock and
 * get_residual_norms report the common clock and the whole block's norms.
 * Error codes as for the solver calls (JZ_EINVAL for bad sizes or
 * parameters, JZ_ESTATE before the grid and state are set). */
typedef struct jz_domain jz_domain;
int jz_domain_create(int ni, int nj, int nk, const jz_params* p, int parts_i, int parts_k, void* hip_stream,
                     jz_domain** out);
int jz_domain_set_grid_metrics(jz_domain* d, const double* m);
int jz_domain_set_state(jz_domain* d, const double* q);
int jz_domain_advance(jz_domain* d, int nsteps);
int jz_domain_get_state(jz_domain* d, double* q);
int jz_domain_get_clock(jz_domain* d, double* t, double* next_dt, long long* steps);
int jz_domain_get_residual_norms(jz_domain* d, double rms[5], double linf[5]);
int jz_domain_destroy(jz_domain* d);

/* ---- steps without device allocation -----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * jz_advance_static runs what jz_create + jz_set_grid_metrics + jz_set_state
 * + jz_advance(nsteps) would, with the same kernels and launch shape (so the
 * same results, bitwise), but keeps everything beyond the caller's buffers --
 * node-major copies of state and metrics, stage buffers, partial sums, clock,
 * failure flag -- in one static device array of the library,
 * JZ_STATIC_SCRATCH_BYTES per GPU, which each GPU holds from the time the
 * library's code is loaded there until the process ends.  It calls no
 * hipMalloc/hipFree, no memset and no host copy, and never synchronises: all
 * work is issued on hip_stream (NULL = null stream) and the call returns once
 * it is queued.
 *   met:   device, 10 x N metric set (the jz_set_grid_metrics layout), read;
 *   q:     device, 5 x N state, advanced in place by nsteps steps (>= 0);
 *   info:  device, 14 doubles or NULL: t, dt of the next step, rms[5],
 *          linf[5] of the last step's first-stage residual, step count, and
 *          the failure flag (0 = healthy; otherwise NaN/Inf or dt <= 0 was
 *          met and the state was left at the failing step);
 *   p:     parameters as for jz_create; stats_interval must be 0.
 * Every run starts at t = 0 with dt from the given state.  The inputs are not
 * validated (a non-positive density or pressure shows up in the flag).
 * JZ_EINVAL for bad sizes or parameters and when the block needs more than
 * JZ_STATIC_SCRATCH_BYTES (the need is jz_workspace_bytes of the same block:
 * up to about 330 k nodes in FP64, 400 k in the FP32-flux form).  Calls on
 * one GPU share its array and keep no state between them: calls that overlap
 * on one GPU (other streams or threads) race and give wrong results. */
#define JZ_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int jz_advance_static(int ni, int nj, int nk, const jz_params* p, const double* met, double* q, double* info,
                      int nsteps, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* jz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* JETLES_H */
