/*
 * clb.h -- C ABI of libclb, the MI355X (gfx950) implementation of the central-moment lattice
 * Boltzmann (CLB) method for incompressible thermal flow of Fei, Luo, Lin and Li
 * (arXiv 1710.10569).
 *
 * One time step advances two populations on a 2D lattice in a single fused pass:
 *   - D2Q9 flow populations f_i (Sec. 2.1): raw moments (Eqs. 6, 7a), central moments through the
 *     shift matrix N(u) (Eq. 7b), relaxation with the block matrix S, equilibrium central moments
 *     (Eq. 9) and consistent forcing C (Eq. 11) in Eq. 8, back-transform, streaming (Eq. 12);
 *   - D2Q5 temperature populations g_i (Sec. 2.2): Eqs. 15-22, T from Eq. 23;
 *   - coupling: F = -g beta (T - T0) + F_v with gravity along -y (Eq. 3), u from Eq. 13;
 *   - walls on nodes: non-equilibrium bounce-back (Zou-He) for f and non-equilibrium
 *     extrapolation for g (Sec. 3, boundary conditions).
 *
 * Conventions for every call:
 *   - Host arrays are borrowed for the duration of the call, FP64, row-major with x fastest:
 *     element (x, y) of an nx-by-ny field is at index y*nx + x.
 *   - Return value: CLB_OK (0) or a negative error code; a message for the last error of the
 *     calling thread is available from clb_last_error().  No call aborts the process.
 *   - A lattice handle owns its device memory; a batch owns its pool unless the caller passes one
 *     to clb_batch_create.  A handle is used by one host thread at a time.
 *   - Work is enqueued on the handle's HIP stream.  clb_step does not block; calls that return
 *     data to the host (clb_moments, clb_get_populations, clb_diagnostics) synchronise the stream.
 *   - Edge order everywhere: west (x = 0), east (x = nx-1), south (y = 0), north (y = ny-1).
 */
#ifndef CLB_H
#define CLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
enum {
    CLB_OK = 0,
    CLB_EINVAL = -1,     /* invalid argument (NULL pointer, size, relaxation time, NaN ...) */
    CLB_ENOMEM = -2,     /* device or host allocation failed, or a memory budget is exceeded */
    CLB_EDEVICE = -3,    /* a HIP runtime call failed (no device, launch failure ...) */
    CLB_ESTATE = -4,     /* call not valid in the handle's current state */
    CLB_EDIVERGED = -5   /* a diagnostic found a non-finite density, velocity or temperature */
};

/* Storage and arithmetic precision of the populations. */
enum {
    CLB_FP64 = 0,        /* f_i, g_i stored and collided in FP64 */
    CLB_FP32_DEV = 1,    /* stored and collided in FP32 as deviations f_i - w_i and g_i - w^T_i T0
                            from the rest equilibrium (w: D2Q9 weights; w^T = (1/2, 1/8 x 4)) */
    CLB_FP64_DEV = 2,    /* the deviation algebra of CLB_FP32_DEV carried out in FP64 */
    CLB_FP32_SR = 3      /* stored as FP32 deviations (as CLB_FP32_DEV, same bytes), collided in FP64,
                            and rounded to FP32 on store stochastically (up or down with probability
                            given by the dropped fraction, from a counter-based hash of node, step
                            and population): unbiased storage rounding, so a long steady-state solve
                            does not drift from the FP64 solution.  Deterministic: the same inputs
                            and step count give bitwise the same state, alone or in a batch. */
};

/* Kind of an edge of the domain.  West/east must both be periodic or both walls; same for
 * south/north. */
enum {
    CLB_PERIODIC = 0,
    CLB_WALL_DIRICHLET = 1,   /* wall with velocity (ux, uy) and temperature T */
    CLB_WALL_ADIABATIC = 2    /* wall with velocity (ux, uy) and zero normal temperature gradient */
};

typedef struct {
    int kind;          /* CLB_PERIODIC, CLB_WALL_DIRICHLET or CLB_WALL_ADIABATIC */
    double ux, uy;     /* wall velocity (a normal component makes the wall permeable) */
    double T;          /* wall temperature (CLB_WALL_DIRICHLET only) */
} clb_edge;

typedef struct {
    int nx, ny;        /* nodes; >= 3 each, >= 4 along the normal of an adiabatic wall pair;
                          nx <= 2^20, ny <= 2^18, nx * ny <= 2^30 */
    int precision;     /* CLB_FP64, CLB_FP32_DEV, CLB_FP64_DEV or CLB_FP32_SR */
    clb_edge west, east, south, north;
    double T0;         /* reference temperature of the Boussinesq force (Eq. 3) */
    int prescribed_u;  /* 1: temperature-only lattice (Sec. 3.1): the velocity is prescribed,
                          uniform and constant, and only the D2Q5 equation is advanced; 0: the
                          coupled flow and temperature problem */
    int in_place;      /* 1: in-place streaming (one population buffer, half the footprint; same
                          results bitwise as 0, the two-buffer pull streaming of Eqs. 12 and 22).
                          Not with prescribed_u; at least 4 nodes across a walled direction.  An
                          in-place lattice runs one step kernel in rows of 64 or 256 nodes: of its
                          tile shape only the width (64, else 256) and the non-temporal-store flag
                          apply, and it is not autotuned */
} clb_desc;

typedef struct clb_lattice clb_lattice;

/* FP64 diagnostics of the current time step (Sec. 3 quantities).  All sums are over nodes. */
typedef struct {
    long long step;        /* time steps taken since clb_init */
    double mass;           /* sum rho (Eq. 13) */
    double heat;           /* sum T (Eq. 23) */
    double mom_x, mom_y;   /* sum rho u (Eq. 13) */
    double sum_w;          /* sum of the averaging weights w(x, y) = wx(x) wy(y), with w = 1/2 on
                              wall nodes of a non-periodic direction and 1 elsewhere */
    double sum_w_ux_T;     /* sum w u_x T  -> <u_x T> = sum_w_ux_T / sum_w (Eq. 29) */
    double sum_w_uy_T;     /* sum w u_y T */
    double wall_flux[4];   /* per edge W, E, S, N: sum over the edge's nodes with trapezoid weights
                              of (3 T_b - 4 T_1 + T_2)/2, the second-order inward-normal gradient of
                              T with the sign of heat entering the domain; 0 for periodic edges */
    double u_max;          /* max |u| */
    double du_max;         /* max over nodes of max(|ux - ux_snap|, |uy - uy_snap|); -1 if no snapshot */
    double dT_max;         /* max |T - T_snap|; -1 if no snapshot */
    int nonfinite;         /* 1 if any rho, u or T is NaN or infinite */
} clb_diag;

/* ---------------------------------------------------------------------------------------------
 * Core calls.
 * ------------------------------------------------------------------------------------------- */

/* Create a lattice on the current HIP device.  hip_stream: a hipStream_t to enqueue work on, or
 * NULL for a stream owned by the handle.  Allocates two population buffers (ping-pong) of
 * 14 values per node (rows of 64-node chunks, each chunk holding its nodes' 14 populations as
 * 14 runs of 64 values), and sets the defaults: rho = 1, u = 0, T = T0 everywhere, all
 * relaxation rates 1 (tau = 1), g*beta = 0, no body force.
 * Errors: CLB_EINVAL (NULL desc/out, bad sizes or kinds, prescribed_u not 0 or 1), CLB_ENOMEM,
 * CLB_EDEVICE. */
int clb_create(const clb_desc* desc, void* hip_stream, clb_lattice** out);

/* Relaxation times and buoyancy.  tau_nu = 1/s_nu, nu = (tau_nu - 1/2)/3 (Sec. 2.1);
 * tau_alpha = 1/lambda1, alpha = (tau_alpha - 1/2)/4 with c_{T,s}^2 = 1/4 (Sec. 2.2, Sec. 3);
 * g_beta: the Boussinesq coefficient of Eq. 3, F_y = g_beta (T - T0).  Ma is informational
 * (the flow's Mach number u_c/c_s of Sec. 3.3) and is kept for reporting only, except on a
 * temperature-only lattice (prescribed_u = 1) whose velocity has not been set with
 * clb_set_prescribed_velocity: there it sets the frame velocity u = (0, Ma c_s) of Sec. 3.1.
 * Errors: CLB_EINVAL if a tau <= 1/2 or any value is not finite. */
int clb_set_params(clb_lattice* h, double tau_nu, double tau_alpha, double g_beta, double Ma);

/* Advance n >= 0 time steps (wall step, macroscopic quantities, both collisions, streaming).
 * Asynchronous on the handle's stream. */
int clb_step(clb_lattice* h, long long n);

/* rho, u and T of the current time step (the wall step and Eqs. 3, 13, 23 applied to the
 * post-streaming populations).  rho, T: nx*ny each; u: 2*nx*ny, the u_x plane then the u_y plane.
 * Any pointer may be NULL.  Synchronises the stream. */
int clb_moments(clb_lattice* h, double* rho, double* u, double* T);

/* Release the handle and its device memory.  NULL-safe. */
void clb_destroy(clb_lattice* h);

/* ---------------------------------------------------------------------------------------------
 * Extensions.
 * ------------------------------------------------------------------------------------------- */

/* Initial state from FP64 fields (NULL: rho = 1, u = 0, T = T0).  u as in clb_moments.  The
 * populations are set to the equilibria whose central moments are Eq. 9 and Eq. 20, at the
 * velocity u - F/(2 rho) for f (F from T by Eq. 3) and u for g, so that clb_moments returns the
 * given fields at interior nodes.  Resets the step counter and the residual snapshot. */
int clb_init(clb_lattice* h, const double* rho, const double* u, const double* T);

/* The tunable rates (Sec. 2.1 matrix S, Sec. 2.2 matrix S_T): bulk rate s_b (bulk viscosity
 * xi = (1/s_b - 1/2)/3), third-order rate s3, fourth-order rate s4, D2Q5 second-order rate
 * lambda2.  Defaults 1.  Errors: CLB_EINVAL unless each is in (0, 2). */
int clb_set_relaxation(clb_lattice* h, double s_b, double s3, double s4, double lambda2);

/* Constant external force density F_v of Eq. 3. */
int clb_set_body_force(clb_lattice* h, double Fvx, double Fvy);

/* Prescribed velocity (ux, uy) of a temperature-only lattice (prescribed_u = 1; Sec. 3.1, where
 * the velocity field is given and only the D2Q5 CLB equation is solved).  The velocity is uniform
 * and constant; it enters the D2Q5 collision (Sec. 2.2) and the temperature wall step at every
 * node, and clb_moments returns rho = 1 and u = (ux, uy).  Takes effect at the next clb_init and
 * clb_step.  Errors: CLB_ESTATE if the lattice is not temperature-only, CLB_EINVAL if a value is
 * not finite or |u|^2 >= 1/2 (where g^eq would turn negative). */
int clb_set_prescribed_velocity(clb_lattice* h, double ux, double uy);

/* FP64 diagnostics of the current step; if snapshot != 0, the current u and T become the new
 * residual snapshot after the residual is measured.  Returns CLB_EDIVERGED (with *out filled)
 * if any value is non-finite.  Synchronises the stream. */
int clb_diagnostics(clb_lattice* h, int snapshot, clb_diag* out);

/* clb_diagnostics without allocating: for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Computes the same
 * record with the same kernels, bitwise equal to clb_diagnostics(h, 0, out); the residual is
 * measured against the snapshot a clb_diagnostics call took, and no snapshot is taken.  The
 * reduction's scratch is a fixed device array of the library (4 MiB per GPU, held until the
 * process ends), so the lattice may have at most 8,388,608 nodes; calls on the same GPU share
 * it, and overlapping calls on one GPU race.  Synchronises the stream.  Errors: CLB_EINVAL for a
 * NULL argument or a larger lattice, CLB_EDEVICE if the scratch cannot be located,
 * CLB_EDIVERGED as clb_diagnostics. */
int clb_diagnostics_noalloc(clb_lattice* h, clb_diag* out);

/* The post-streaming populations of the current step (before the wall step), as full FP64
 * values: f as 9 planes and g as 5 planes of nx*ny, direction order of Eq. 4.  A population
 * whose streaming source lies outside the domain is unknown and returned as NaN.  Either pointer
 * may be NULL.  Synchronises the stream. */
int clb_get_populations(clb_lattice* h, double* f, double* g);

/* Checkpoint / resume (for callers that must stop and continue a run, possibly in another process on
 * the same library build).  clb_checkpoint_size writes the bytes a checkpoint of this lattice takes;
 * clb_checkpoint_save copies into the caller's host buffer `host` (at least that many bytes) a
 * header -- description, parameters, step count, whether a residual snapshot exists -- followed by
 * the raw device state: the current population buffer (in place: the buffer and its two
 * wall-band snapshot copies) and the FP64 residual snapshot of clb_diagnostics.  Synchronises.
 * clb_checkpoint_load restores such a blob into a lattice created with the same description (every
 * field of clb_desc equal), replacing its state, parameters and step count; stepping on then gives
 * bitwise the results of the run that was not interrupted (the stochastic rounding is keyed by the
 * step count).  Errors: CLB_EINVAL for NULL arguments, a buffer that is too small, or a blob of
 * another library version or lattice description; CLB_EDEVICE for a failed copy. */
int clb_checkpoint_size(clb_lattice* h, size_t* bytes);
int clb_checkpoint_save(clb_lattice* h, void* host, size_t bytes);
int clb_checkpoint_load(clb_lattice* h, const void* host, size_t bytes);

/* Physical parameters -> relaxation times (Sec. 3.3): nu = Ma c_s H sqrt(Pr/Ra), alpha = nu/Pr,
 * g*beta = Ra nu alpha / (dT H^3), tau_nu = 3 nu + 1/2, tau_alpha = 4 alpha + 1/2.
 * Host-only.  Errors: CLB_EINVAL for non-positive or non-finite inputs or NULL outputs. */
int clb_params_from_physics(double Ra, double Pr, double Ma, double H, double dT,
                            double* tau_nu, double* tau_alpha, double* g_beta);

/* Time n steps on the handle's stream with HIP events (inputs already on the device); writes the
 * elapsed milliseconds of the n launches.  Synchronises the stream. */
int clb_time_steps(clb_lattice* h, long long n, double* ms);

/* ---------------------------------------------------------------------------------------------
 * Launch shapes and the autotuner.  The step kernel is compiled for a fixed set of workgroup tile
 * shapes (nodes per row segment tx, thread rows ty, nodes per thread spt stacked ty rows apart,
 * non-temporal stores or not).  Results do not depend on the shape; only speed does.
 * ------------------------------------------------------------------------------------------- */

/* Number of compiled tile shapes. */
int clb_tile_shape_count(void);

/* Geometry of shape `shape` (0 <= shape < clb_tile_shape_count()); any output may be NULL.
 * Errors: CLB_EINVAL for an out-of-range shape. */
int clb_tile_shape_info(int shape, int* tx, int* ty, int* spt, int* nontemporal);

/* Select / read the shape used by clb_step.  A new handle starts with the shape the autotuner
 * last chose in this process for the same precision and size class (ceil(log2 nx),
 * ceil(log2 ny)), else a default by footprint: one-wavefront 64 x 1 tiles -- shape 12 (plain
 * stores) for FP32 populations whose two buffers fit the 256 MiB Infinity Cache, 13 (non-temporal,
 * occupancy-8 budget) for plain FP32 beyond it, 11 (non-temporal) otherwise; an in-place lattice
 * takes 256-node rows, shape 2 for FP32 populations that fit the cache, else 6. */
int clb_set_tile_shape(clb_lattice* h, int shape);
int clb_get_tile_shape(clb_lattice* h, int* shape);

/* Time every shape for `launches_per_shape` launches on this lattice, select the fastest for the
 * handle and record it for its size class.  The timed steps ping-pong between two temporary device
 * buffers that start as a copy of the current state (the access pattern of real stepping); the
 * lattice state and step count are unchanged.  If the temporary pair cannot be allocated, each
 * launch instead reads the current state and writes the spare buffer.  best_shape and best_us
 * (average launch time of the winner, microseconds) may be NULL.  Synchronises. */
int clb_autotune(clb_lattice* h, int launches_per_shape, int* best_shape, double* best_us);

/* Average launch time in microseconds of `launches` step launches with shape `shape`, measured
 * as in clb_autotune; state unchanged.  Synchronises. */
int clb_time_shape(clb_lattice* h, int shape, int launches, double* us);

/* Wait for the handle's stream. */
int clb_synchronize(clb_lattice* h);

/* Message for the last error on the calling thread ("" if none). */
const char* clb_last_error(void);

/* ---------------------------------------------------------------------------------------------
 * Batches: many lattices of different sizes resident in one HBM pool and advanced together.
 *
 * A batch owns (or borrows) one device pool and carves it into per-lattice regions: two
 * population buffers (an in-place lattice: one, plus its two wall-band snapshots) and an FP64
 * snapshot of (u_x, u_y, T) for the residual test.  Adding a lattice
 * is admission: it fails with CLB_ENOMEM when its region does not fit in the pool's free space.
 * All lattices of a batch use the batch's precision.  Every schedule below runs the same per-node
 * update, so a lattice's results do not depend on the schedule or on which other lattices share
 * the batch.  Work is enqueued on the batch's stream; calls returning data synchronise it.
 * ------------------------------------------------------------------------------------------- */
typedef struct clb_batch clb_batch;

/* Pool bytes one lattice of this description occupies in a batch. */
int clb_batch_footprint(const clb_desc* desc, size_t* bytes);

/* Create a batch of at most `capacity` lattices.  pool == NULL: the library allocates
 * hbm_budget_bytes of device memory for the pool.  pool != NULL: [pool, pool + pool_bytes) is used
 * (e.g. a framework-allocated tensor, 256-byte aligned; it must outlive the batch) and
 * hbm_budget_bytes is ignored.  hip_stream as in clb_create.
 * Errors: CLB_EINVAL, CLB_ENOMEM, CLB_EDEVICE. */
int clb_batch_create(int capacity, int precision, size_t hbm_budget_bytes, void* pool, size_t pool_bytes,
                     void* hip_stream, clb_batch** out);

/* Admit a lattice (desc->precision must equal the batch's) with the parameters of
 * clb_set_params; it starts at rest (rho = 1, u = 0, T = T0) with step count 0.  *slot receives its
 * index.  Two-buffer and in-place lattices may share a batch; temperature-only lattices
 * (prescribed_u = 1) are single-lattice only.  A batch lattice's population buffer must be under
 * 4 GiB (the grouped step addresses it with 32-bit byte offsets: up to about 76 M nodes in FP32
 * storage, 38 M in FP64); larger lattices run as single lattices.  Errors: CLB_EINVAL (bad
 * description, precision other than the batch's, prescribed_u = 1, a buffer of 4 GiB or more);
 * CLB_ENOMEM if the batch is full or the pool lacks space. */
int clb_batch_add(clb_batch* b, const clb_desc* desc, double tau_nu, double tau_alpha, double g_beta, double Ma,
                  int* slot);

/* Per-slot counterparts of clb_set_relaxation, clb_set_body_force, clb_init, clb_moments,
 * clb_diagnostics. */
int clb_batch_set_relaxation(clb_batch* b, int slot, double s_b, double s3, double s4, double lambda2);
int clb_batch_set_body_force(clb_batch* b, int slot, double Fvx, double Fvy);
int clb_batch_init(clb_batch* b, int slot, const double* rho, const double* u, const double* T);
int clb_batch_moments(clb_batch* b, int slot, double* rho, double* u, double* T);
int clb_batch_diagnostics(clb_batch* b, int slot, int snapshot, clb_diag* out);

/* Residual of every resident lattice in one pass: for each slot, the max-norm change of
 * (u_x, u_y) and of T since the slot's last snapshot, then the snapshot is replaced by the current
 * fields.  A slot's snapshot starts as its initial fields (clb_batch_add / clb_batch_init), so
 * calling this every k steps measures the change per k steps.  Arrays have `capacity` entries
 * indexed by slot; unused slots get -1 and 0.  nonfinite[i] = 1 if lattice i holds a NaN or
 * infinity in rho, u or T.  Any output may be NULL.  Synchronises. */
int clb_batch_residuals(clb_batch* b, double* du, double* dT, int* nonfinite);

/* Release a slot and its pool region (stream-ordered after the work already enqueued). */
int clb_batch_remove(clb_batch* b, int slot);

/* Advance every resident lattice n steps: one launch per step over all lattices' tiles. */
int clb_batch_step(clb_batch* b, long long n);

/* The same n steps with one launch per lattice per step (the one-lattice-at-a-time schedule). */
int clb_batch_step_each(clb_batch* b, long long n);

/* The same n steps with small lattices workgroup-resident when there are many of them (at least 256
 * lattices of at most 64*64 nodes): one launch runs all n steps, each such lattice owned by one
 * 1024-thread workgroup with a workgroup barrier between steps, on a second stream; larger
 * lattices (and all of them when the small ones are fewer) take the grouped launches concurrently
 * on the batch's stream.  Suited to many tiny lattices, whose grouped steps are latency-bound. */
int clb_batch_step_persistent(clb_batch* b, long long n);

/* Synchronise the batch's stream and report any pending launch error (CLB_EDEVICE). */
int clb_batch_check(clb_batch* b);

/* Time n steps of schedule mode (0 grouped, 1 one launch per lattice, 2 persistent) with HIP events
 * on the batch's stream; writes the elapsed milliseconds.  Synchronises. */
int clb_batch_time_steps(clb_batch* b, int mode, long long n, double* ms);

/* Tile width of one lattice: 64, 128 or 256 nodes per row segment (256 nodes per tile), or 0 for
 * wrapped rows: each row is cut into 32-node runs from x = 0 (the last may be short), the runs of
 * all rows are taken in row-major order, shifted by one run, two per wavefront, so that the last
 * run of a row and the first run of the next share one wavefront (on lattices with walls in x this
 * halves the wavefronts that take the wall branch) and every access stays cache-line aligned.
 * Results do not depend on it. */
int clb_batch_set_tile_width(clb_batch* b, int slot, int tile_width);

/* The lattice's current tile width (64, 128, 256, or 0 for wrapped rows), as set by
 * clb_batch_set_tile_width, clb_batch_autotune or the default: wrapped rows when x has walls; else
 * for two-buffer lattices by width (64 up to 96 nodes, 128 up to 192, 256 beyond) and 64 for
 * in-place lattices, which the autotuner does not time.  Errors: CLB_EINVAL for an unused slot or
 * a NULL output. */
int clb_batch_get_tile_width(clb_batch* b, int slot, int* tile_width);

/* Store form of the batch's step kernels: 1 = non-temporal stores (populations written this step
 * are read next step, but at batch footprints they leave every cache before that), 0 = ordinary
 * stores.  Default (until this call or clb_batch_autotune): non-temporal once the resident lattices
 * take more than 256 MiB, and always for FP64 storage.  Results do not depend on it. */
int clb_batch_set_nontemporal(clb_batch* b, int nontemporal);

/* The store form the next grouped step uses (1 non-temporal, 0 ordinary), from
 * clb_batch_set_nontemporal, clb_batch_autotune or the default above.  Errors: CLB_EINVAL. */
int clb_batch_get_nontemporal(clb_batch* b, int* nontemporal);

/* For each size class (ceil(log2 nx), ceil(log2 ny)) present, time the grouped step over that
 * class's lattices with each tile width, wrapped rows included (state unchanged), and keep the
 * fastest for the class;
 * lattices added later take the class's choice.  Then time the grouped step over the whole batch
 * with ordinary and with non-temporal stores and keep the faster.  Synchronises. */
int clb_batch_autotune(clb_batch* b, int launches);

/* Lattices resident, pool bytes in use, pool size, total nodes.  Any output may be NULL. */
int clb_batch_info(clb_batch* b, int* count, size_t* used_bytes, size_t* budget_bytes, long long* sites);

int clb_batch_synchronize(clb_batch* b);

/* NULL-safe. */
void clb_batch_destroy(clb_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* CLB_H */
