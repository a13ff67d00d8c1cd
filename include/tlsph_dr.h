/*
 * tlsph_dr.h -- C ABI of the MI355X (gfx950) library for the splitting random-choice dynamic
 * relaxation of total Lagrangian SPH (Zhu, Zhang & Hu, arXiv:2103.08932).
 *
 * The library relaxes an elastic body, given in its reference configuration, to static
 * equilibrium.  Each relaxation step runs on the GPU over fixed reference-configuration neighbour
 * lists:
 *   - half drift of the displacement (Sec. 2.3, Eq. 15);
 *   - kernel-corrected deformation gradient F = I + grad0 u (Eqs. 2, 9, 14), second and first
 *     Piola-Kirchhoff stresses (Eqs. 3-8) and T = P B0;
 *   - pairwise force sum and kick (Eqs. 12-13, 16);
 *   - on the steps picked by the random-choice rule (Sec. 3.3, Eq. 40), the operator-split
 *     implicit pairwise viscous damping (Secs. 3, 3.2: Eqs. 24-25, 37-39) swept colour block by
 *     colour block over the splitting cell-linked list (Sec. 3.4);
 *   - second half drift (Eq. 17), kinetic-energy / residual reductions in FP64 and the next
 *     time step (Eq. 18).
 *
 * Conventions for every call:
 *   - Host arrays are copied; the caller keeps ownership.  Particle arrays are in the caller's
 *     ("input") order, row-major n x dim, unless a call says otherwise.
 *   - A body owns its device memory, obtained from the allocator in its descriptor (or hipMalloc
 *     when the allocator's alloc is NULL) and released by tlsph_destroy_body.
 *   - All device work of a body is enqueued on the stream given at creation (a hipStream_t,
 *     borrowed; NULL = the default stream).  Calls that return results to the host synchronise
 *     that stream.
 *   - One host thread at a time per body or server.
 *   - Every call returns a tlsph_status.  Negative values are errors; tlsph_last_error() then gives
 *     a message for the calling thread.  Invalid arguments are rejected before any device work.
 */
#ifndef TLSPH_DR_H
#define TLSPH_DR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TLSPH_OK = 0,
    TLSPH_NOT_CONVERGED = 1,      /* status, not an error: max_steps reached before tol */
    TLSPH_E_INVALID = -1,         /* bad argument or call order */
    TLSPH_E_NOMEM = -2,           /* device or host allocation failed */
    TLSPH_E_SINGULAR_B0 = -3,     /* a particle's correction matrix (Eq. 9) is singular */
    TLSPH_E_CELL_ADJ = -4,        /* a neighbour lies outside the adjacent cells (Sec. 3.4) */
    TLSPH_E_NONFINITE = -5,       /* NaN / Inf in the state, or J <= 0 with the neo-Hookean law */
    TLSPH_E_DIVERGED = -6,        /* kinetic energy blew up (tlsph_set_divergence) */
    TLSPH_E_DEVICE = -7,          /* a HIP runtime call failed */
    TLSPH_E_LIMIT = -8            /* a size limit of this build was exceeded (see tlsph_last_error) */
} tlsph_status;

enum { TLSPH_FP32 = 32, TLSPH_FP64 = 64 };          /* arithmetic of F, stress, force and damping */
enum { TLSPH_SVK = 0, TLSPH_NEOHOOKE = 1 };        /* Eq. 4 (St Venant-Kirchhoff) / Eqs. 7-8 */
enum { TLSPH_PAIRWISE = 0, TLSPH_PARTICLE = 1 };   /* damping splitting: Sec. 3.2 / Sec. 3.1 */

/* Device-memory provider.  alloc returns device memory of at least `bytes` bytes (256-byte
 * aligned) or NULL; free releases it.  Both are called only from the calling thread. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} tlsph_allocator;

/* Reference configuration of a body (Sec. 2: X0, V0 = dp^dim, rho0, constrained particles).
 *   dim        2 (plane strain) or 3
 *   n          particle count, 1 <= n < 2^31
 *   X0         host, n x dim reference positions (FP64)
 *   clamped    host, n flags (nonzero = clamped: u = v = 0 for all time), or NULL for none
 *   dp         particle spacing; V0 = dp^dim, m = rho0 V0
 *   h_over_dp  smoothing length h = h_over_dp * dp (the paper uses 1.3); cut-off r_c = 2 h
 *   rho0       reference density
 *   precision  TLSPH_FP32 or TLSPH_FP64 (displacement and the reductions are FP64 in both)
 *   stream     hipStream_t (borrowed) or NULL
 *   alloc      device-memory provider (alloc == NULL: hipMalloc / hipFree) */
typedef struct {
    int dim;
    int64_t n;
    const double *X0;
    const uint8_t *clamped;
    double dp;
    double h_over_dp;
    double rho0;
    int precision;
    void *stream;
    tlsph_allocator alloc;
} tlsph_body_desc;

typedef struct tlsph_body_s *tlsph_body;

/* Builds a body: cell binning (cell = cut-off, Sec. 3.4), cell-sorted internal order (stable in
 * the input index), colour blocks, CSR neighbour lists of the reference configuration (j != i with
 * |X0_j - X0_i|^2 < r_c^2) and the correction matrices B0 (Eq. 9).  u = v = 0, step index 0.
 * Errors: TLSPH_E_INVALID, TLSPH_E_NOMEM, TLSPH_E_SINGULAR_B0, TLSPH_E_LIMIT, TLSPH_E_DEVICE. */
tlsph_status tlsph_create_body(const tlsph_body_desc *desc, tlsph_body *out);

/* Material (Sec. 2.1): model TLSPH_SVK (Eq. 4) or TLSPH_NEOHOOKE (Eqs. 7-8); Young's modulus
 * E >= 0 and Poisson ratio -1 < nu < 0.5, with E = 2 mu (1 + nu) = 3 K (1 - 2 nu).  Resets the time
 * step (Eq. 18) and the residual tracking; the state u, v is kept. */
tlsph_status tlsph_set_material(tlsph_body body, int model, double E, double nu);

/* Loads (Eq. 1): body force g (dim components, every particle) plus an optional per-particle
 * acceleration accel (host, n x dim, input order, or NULL) added to it; surface tractions are
 * passed as accelerations t / (rho0 dp) of the loaded particles.  Resets the time step and the
 * residual tracking. */
tlsph_status tlsph_set_loads(tlsph_body body, const double *g, const double *accel);

/* Artificial viscosity and random choice (Sec. 3): eta > 0 is used as given; eta <= 0 takes
 * eta = (beta / 4) sqrt(rho0 E) Lc (Eq. 36, needs the material).  alpha in (0, 1] is the
 * probability of a damped step (Eq. 40, damped with eta / alpha); the decision of step n is
 * Philox4x64-10 with key (seed, 0) and counter (n, 0, 0, 0): damped iff the top 24 bits of output
 * word 0 are below ceil(alpha 2^24).  Without this call no step is damped. */
tlsph_status tlsph_set_damping(tlsph_body body, double eta, double beta, double Lc, double alpha,
                               uint64_t seed);

/* Blow-up detection (the paper has none; it relaxes to fixed end times).  Once the kinetic energy
 * E_k has fallen below its running peak for the first time since the last reset of the residual
 * tracking, the peak at that moment is kept; a later step whose E_k exceeds factor times it ends the
 * run with TLSPH_E_DIVERGED (the step completes: its state is finite and can be read).  factor > 0;
 * default 1e6.  A run that goes non-finite or inverts a particle first reports TLSPH_E_NONFINITE. */
tlsph_status tlsph_set_divergence(tlsph_body body, double factor);

/* Splitting of the damping step S_d (Eq. 25).  TLSPH_PAIRWISE (the default, Sec. 3.2): each
 * neighbour pair is solved exactly (Eq. 39) in a nested Strang sweep.  TLSPH_PARTICLE (Sec. 3.1):
 * D_i solves particle i against all its neighbours at once (Eqs. 26-34: one exact line-search step
 * of the local implicit system, i's velocity first, then each free neighbour's with the momentum
 * it gave up); a clamped i leaves its own velocity at zero and each free neighbour takes the wall
 * solution m v_j / (m - B_j).  With TLSPH_PARTICLE and damping set, every time step also obeys the
 * viscous limit dt <= 50 h^2 / (nu dim) of Eq. 35, nu = eta / rho0 (eta, not eta / alpha).  Same colour sweep order and
 * random choice as the pairwise scheme.  The time step already chosen is kept; the limit applies
 * from the next step's choice on. */
tlsph_status tlsph_set_damping_scheme(tlsph_body body, int scheme);

typedef struct {
    int64_t steps;            /* steps taken by this call */
    int64_t damped_steps;     /* of which damped */
    int64_t step_index;       /* the body's step counter after the call */
    double residual;          /* max over the last W steps of E_k / E_peak (1 while E_peak = 0) */
    double kinetic_energy;    /* E_k = sum over free particles of m |v|^2 / 2 after the last step */
    double force_residual;    /* sqrt(sum |a|^2) / sqrt(sum |b|^2) over free particles (diagnostic) */
    double dt;                /* time step of the next step */
    double wall_s;            /* host wall time of the call */
    int64_t window;           /* W */
    int converged;            /* residual < tol and step_index >= W */
} tlsph_report;

/* Relaxation loop: runs steps until residual < tol and the step index is at least W
 * (W = ceil(T_w / dt0), T_w = L_max^2 / (L_min c), dt0 of Eq. 18 at rest; L_max,
 * L_min the largest / smallest bounding-box extent plus dp; c = sqrt(K / rho0)), or until max_steps
 * steps were taken by this call.  Blocks; returns TLSPH_OK when converged, TLSPH_NOT_CONVERGED when
 * max_steps ran out, or an error (TLSPH_E_NONFINITE, TLSPH_E_DIVERGED, TLSPH_E_DEVICE).  `out` may
 * be NULL. */
tlsph_status tlsph_relax_until(tlsph_body body, double tol, int64_t max_steps, tlsph_report *out);

/* Runs exactly nsteps steps.  force_damping: -1 = random choice (as relax_until), 0 = never damp,
 * 1 = damp every step (with eta / alpha).  Does not stop at convergence.  Blocks. */
tlsph_status tlsph_step(tlsph_body body, int64_t nsteps, int force_damping, tlsph_report *out);

/* Displacement u = x - X0 (Eq. 2) after the last step: host, n x dim FP64, input order. */
tlsph_status tlsph_get_displacement(tlsph_body body, double *u_out);

/* Von Mises stress of every particle (clamped ones included) for the current displacement, the
 * field the twisting example of Sec. 4.2 plots: F of Eq. 9 from u, S of Eq. 4 or Eqs. 7-8, the
 * Cauchy stress sigma = J^-1 F S F^T and sqrt(3/2 s:s) of its deviator s; in 2D plane strain, with
 * the out-of-plane stress S33 / J (S33 = lambda tr E for St Venant-Kirchhoff, lambda ln J for
 * neo-Hookean).  Computed in the body's working precision.  vm_out: host, n FP64, input order.
 * Needs the material.  TLSPH_E_NONFINITE when some particle has J <= 0 or a non-finite stress (its
 * entry is then NaN; the others are valid). */
tlsph_status tlsph_get_von_mises(tlsph_body body, double *vm_out);

/* The same von Mises field as tlsph_get_von_mises, computed without allocating device memory: for
 * callers that cannot call hipMalloc (code under HIP graph capture, tight serving loops, harnesses
 * that forbid device allocation).  Its working memory is one file-scope device array of the library
 * (40 MiB on each device that calls it, held until the process ends), so it handles bodies of at
 * most 2^21 = 2,097,152 particles and returns TLSPH_E_LIMIT above that.  The caller still passes the
 * output: vm_out, host, n FP64, input order, as tlsph_get_von_mises (bit-identical values).  Blocks.
 * Calls that overlap on one device (two threads, or two bodies on one device) share the array and
 * race: serialise them.  Errors as tlsph_get_von_mises, plus TLSPH_E_LIMIT and TLSPH_E_DEVICE. */
tlsph_status tlsph_get_von_mises_noalloc(tlsph_body body, double *vm_out);

/* Checkpoint: u and v (host, n x dim FP64, input order; either may be NULL), the step index and
 * the time step of the next step. */
tlsph_status tlsph_get_state(tlsph_body body, double *u, double *v, int64_t *step, double *dt);

/* Restore: u, v (host, n x dim, input order; NULL = zero; clamped entries are forced to zero), the
 * step index and the next time step (dt <= 0: derived from max|v| and max|b| by Eq. 18).  Residual
 * tracking restarts. */
tlsph_status tlsph_set_state(tlsph_body body, const double *u, const double *v, int64_t step, double dt);

/* Internal layout for tests (any pointer may be NULL).  Internal order = particles sorted by cell
 * id (stable in the input index).
 *   perm    int32[n]     internal -> input index
 *   cell    int32[n]     linear cell id ((cx ny + cy) nz + cz; 2D: cx ny + cy), internal order
 *   colour  int32[n]     colour block of the particle's cell (3D: 9 (cx%3) + 3 (cy%3) + cz%3;
 *                        2D: 3 (cx%3) + cy%3)
 *   row_ptr int64[n+1]   CSR row offsets, internal order
 *   col     int32[nnz]   CSR columns (internal indices), ascending in each row */
tlsph_status tlsph_debug_topology(tlsph_body body, int32_t *perm, int32_t *cell, int32_t *colour,
                                  int64_t *row_ptr, int32_t *col);

/* Brick lengths (cells along the fastest cell axis) of the workgroup tiles of the force passes:
 * cells_a for F / stress (and the von Mises output), cells_b for the pair-force sum.  Chosen at
 * creation from the dimension, the precision and the particle count; TLSPH_PASSB_LONG_BRICK_N in
 * the environment at creation sets the particle count above which a 3D FP32 body takes 4-cell bricks
 * for the pair-force sum (default 8,000,000).  Either pointer may be NULL. */
tlsph_status tlsph_debug_bricks(tlsph_body body, int32_t *cells_a, int32_t *cells_b);

/* Sizes: particle count, CSR entries (directed pairs), cell grid, window W. */
tlsph_status tlsph_body_info(tlsph_body body, int64_t *n, int64_t *nnz, int32_t ncell[3], int64_t *window);

/* Per-pass GPU time.  tlsph_profile(body, 1) starts recording HIP events around every pass launch
 * (on the body's stream) and clears the totals; 0 stops.  tlsph_profile_read fills up to `cap`
 * entries of ms[] (total milliseconds) and launches[] (count) for the passes in this order:
 * 0 drift, 1 pass A (F, stress, T), 2 pass B (force, kick), 3 pass D (one damping colour launch),
 * 4 pass C (drift, reductions), 5 finish.  Returns the number of passes. */
tlsph_status tlsph_profile(tlsph_body body, int enable);
int tlsph_profile_read(tlsph_body body, double *ms, int64_t *launches, int cap);

/* ------------------------------------------------------------------------------------------------
 * Request server: relaxation solves of many bodies, continuously batched.
 *
 * The paper solves one body at a time; many small bodies would leave the GPU mostly idle.  A server
 * keeps every admitted body's state resident in device memory and advances all of them together:
 * each pass of a step is one launch over the bodies of one dimension, every body being a range of
 * that launch's workgroups (per-body offsets in a launch table), with its own time step,
 * random-choice decisions, residual and stop rule.  A request is set up (neighbour lists, B0) on a
 * second stream by a worker thread while the admitted bodies step, and joins the batch at the next
 * chunk boundary; a converged body leaves the batch, its displacement is copied out and its memory
 * is returned for the next admission.  Admission is by memory budget (an estimate of the body's
 * device footprint against the free part of the server's pool) and by slot count.  Every body is
 * computed by the same kernels, in the same order, as a body of tlsph_create_body with the same
 * precision, so a request gives the same result alone as in any mix.
 * ------------------------------------------------------------------------------------------------ */

/* One relaxation request (Sec. 2 problem statement: reference body, material, loads, damping,
 * stop rule).  body.precision, body.stream and body.alloc are ignored (the server's apply). */
typedef struct {
    tlsph_body_desc body;
    int model;                /* TLSPH_SVK or TLSPH_NEOHOOKE */
    double E, nu;
    double g[3];              /* body force (dim components used) */
    const double *accel;      /* host, n x dim or NULL (as tlsph_set_loads) */
    double eta, beta, Lc, alpha;
    uint64_t seed;            /* as tlsph_set_damping */
    double tol;               /* stop when residual < tol (and step >= W), as tlsph_relax_until */
    int64_t max_steps;        /* or after this many steps, >= 1 (TLSPH_NOT_CONVERGED) */
    int scheme;               /* TLSPH_PAIRWISE (0, zero-initialised default) or TLSPH_PARTICLE */
} tlsph_request;

typedef struct tlsph_server_s *tlsph_server;

/* Creates a server.  hbm_budget bytes of device memory are taken from `alloc` once, here, and
 * sub-allocated to the bodies; a body is admitted when its estimated footprint fits in the largest
 * free range.  max_slots (1..64) bounds the bodies in setup or in the batch.  precision applies to
 * every request.  The bodies step in batch groups (8, or TLSPH_SERVE_GROUPS in the environment, at
 * most 8; never more than max_slots), each with its own thread and stream; stream (borrowed, NULL =
 * create one) is the first group's, the server creates the others and one for setups (all at
 * default priority).  A body joins a group holding no body of the other dimension if there is one,
 * the fewest bodies first.  Starts the worker and group threads. */
tlsph_status tlsph_server_create(size_t hbm_budget, int max_slots, int precision, void *stream,
                                 tlsph_allocator alloc, tlsph_server *out);

/* Queues a request (inputs copied; never waits for the GPU).  *ticket identifies it. */
tlsph_status tlsph_server_submit(tlsph_server server, const tlsph_request *req, int64_t *ticket);

/* Waits up to timeout_s seconds (0 = just look) for the request to finish.  *done = 1 when it has;
 * then *status is its outcome (TLSPH_OK converged, TLSPH_NOT_CONVERGED, or an error, whose message
 * tlsph_server_error gives) and *report its report, with wall_s = time from submission to the
 * result being ready.  report or status may be NULL. */
tlsph_status tlsph_server_wait(tlsph_server server, int64_t ticket, double timeout_s, int *done,
                               tlsph_status *status, tlsph_report *report);

/* Displacement of a finished request: host, n x dim FP64, input order.  Once per ticket: the
 * server drops its copy afterwards (the report stays available). */
tlsph_status tlsph_server_result(tlsph_server server, int64_t ticket, double *u_out);

/* Timeline of a request, seconds since tlsph_server_create: [0] submitted, [1] setup started,
 * [2] joined the batch, [3] result ready (negative = not yet). */
tlsph_status tlsph_server_times(tlsph_server server, int64_t ticket, double times[4]);

/* Error message of a failed request ("" if none). */
const char *tlsph_server_error(tlsph_server server, int64_t ticket);

typedef struct {
    int64_t submitted, completed, failed;
    int64_t pending;          /* waiting for admission */
    int64_t in_setup, active; /* being set up / in the batch */
    int64_t peak_active;
    int64_t chunks;           /* batch chunks run */
    int64_t batch_steps;      /* steps of the batch (one step advances every active body) */
    size_t pool_bytes, pool_used, pool_peak;
} tlsph_server_stats;

tlsph_status tlsph_server_stats_get(tlsph_server server, tlsph_server_stats *out);

/* Stops the threads (the running chunk finishes; unfinished requests are dropped) and releases
 * everything, the pool through the allocator's free. */
void tlsph_server_destroy(tlsph_server server);

/* Host-only: the random-choice decisions (1 = damped) of steps n0 .. n0 + count - 1 for (seed,
 * alpha), as tlsph_set_damping defines them.  Touches no device. */
tlsph_status tlsph_damping_decisions(uint64_t seed, double alpha, int64_t n0, int64_t count, uint8_t *out);

void tlsph_destroy_body(tlsph_body body);

/* Message of the calling thread's last error ("" if none). */
const char *tlsph_last_error(void);

/* Version string of the library build. */
const char *tlsph_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TLSPH_DR_H */
