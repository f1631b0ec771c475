/*
 * hawkes.h -- C ABI of libhawkes, the gfx950 (MI355X) implementation of the
 * spatiotemporal Hawkes log-likelihood and its gradient.
 *
 * Model: Holbrook, Ji & Suchard, "Bayesian mitigation of spatial coarsening for
 * a Hawkes model applied to gunfire, wildfire and viral contagion"
 * (arXiv 2010.02994).  For events (x_n, t_n), n = 1..N, x_n in R^D:
 *
 *   lambda_n = sum_{n' != n} mu_{nn'} + xi_{nn'}                  (Sec. 2.1, eq. "likelihood")
 *   mu_{nn'} = mu0 (2 pi)^{-(D+1)/2} tau_x^{-D} tau_t^{-1}
 *              exp(-|x_n - x_n'|^2 / (2 tau_x^2) - (t_n - t_n')^2 / (2 tau_t^2)),  only if t_n != t_n'
 *   xi_{nn'} = theta omega (2 pi)^{-D/2} h^{-D}
 *              exp(-omega (t_n - t_n') - |x_n - x_n'|^2 / (2 h^2)),                only if t_n' < t_n
 *   Lambda_n = mu0 [Phi((t_N - t_n)/tau_t) - Phi(-t_n/tau_t)] + theta [1 - exp(-omega (t_N - t_n))]
 *   ell      = sum_n log lambda_n - sum_n Lambda_n                  (Sec. 2.1)
 *   d ell/d x_n as in App. A;  d ell/d Theta by differentiating the above.
 *
 * t_N is the largest event time; the spatial integral runs over R^D.
 *
 * Conventions for every entry point:
 *  - Return a hawkes_status_t.  Nothing aborts; nothing throws across the ABI.
 *  - Pointers are device pointers unless marked "host".  The caller owns every
 *    buffer.  The library never allocates device memory on the evaluation path:
 *    scratch comes from the caller's workspace (size: hawkes_workspace_bytes).
 *  - x is row-major N x D float64, t is N float64 sorted non-decreasing, t >= 0.
 *  - Work is ordered on the given HIP stream (NULL = the default stream).
 *  - Host-side argument errors return at once and launch nothing.  Errors found
 *    on the device (unsorted or non-finite data) leave grad_x untouched.
 *  - Results are bitwise reproducible for the same (N, D, precision, inputs):
 *    every reduction runs in a fixed order and no float atomics touch global memory.
 *  - Calls are re-entrant with distinct workspaces.
 */
#ifndef HAWKES_H_
#define HAWKES_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Model parameters in API order.  Paper symbols (Theta of Sec. 2.1):
 *   mu = mu0 (background weight), h = tau_x (background spatial bandwidth),
 *   tau = tau_t (background temporal bandwidth), theta (self-excitation weight),
 *   omega (self-excitation decay rate), xi = the paper's h (self-excitation
 *   spatial bandwidth).  Domain: h, tau, omega, xi > 0; mu, theta >= 0, not both 0. */
typedef struct {
  double mu, h, tau, theta, omega, xi;
} hawkes_params_t;

typedef enum {
  HAWKES_FP64 = 0,  /* every step in float64; the pair terms' exp by a table-driven
                       method (Tang, 2^8 entries) good to a few ulp, the other
                       special functions from the device math library */
  HAWKES_MIXED = 1, /* pair arithmetic and exp in float32, all sums, logs, the
                       compensator and final reductions in float64 */
  HAWKES_CULL = 0x10 /* flag, OR-ed into either precision: skip the column tiles
                        whose every pair is so far apart in time that both pair
                        terms are exactly zero in that precision's arithmetic
                        (float64: exponents below -750; mixed: base-2 exponents
                        below -160 after the shift).  Results are bitwise equal
                        to the run without the flag; only time changes. */
} hawkes_prec_t;

typedef enum {
  HAWKES_OK = 0,
  HAWKES_EINVAL = -1,     /* n < 2, d outside [1, 8], null pointer, workspace too small */
  HAWKES_EPARAM = -2,     /* non-finite or out-of-domain parameter */
  HAWKES_EDATA = -3,      /* t unsorted, negative or non-finite; x non-finite */
  HAWKES_EZERORATE = -4,  /* some lambda_n == 0: loglik = -inf, gradients NaN */
  HAWKES_ENOMEM = -5,     /* serving: request footprint exceeds the memory budget */
  HAWKES_EDEVICE = -6,    /* a HIP runtime call failed */
  HAWKES_ESTATE = -7,     /* serving: unknown ticket / dataset, or server shutting down */
  HAWKES_ETIMEOUT = -8,   /* serving: wait timed out (request still pending) */
  HAWKES_EPENDING = 1     /* serving poll: not finished yet */
} hawkes_status_t;

/* Device workspace needed by hawkes_loglik / hawkes_grad for (n, d, prec).
 * Returns 0 for invalid (n, d, prec).  Layout is private to the library. */
size_t hawkes_workspace_bytes(int64_t n, int d, int prec);

/* Log-likelihood only (rate pass, finalize).  loglik is a host pointer.
 * Synchronizes the stream to deliver the scalar. */
int hawkes_loglik(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                  int prec, void* ws, size_t ws_bytes, void* stream, double* loglik /* host */);

/* Log-likelihood and full gradient.  grad_x: device, n*d row-major, overwritten.
 * loglik (host, 1) and grad_params (host, 6, API order) receive the scalars;
 * either may be NULL.  Synchronizes the stream to deliver them; the last
 * kernel writes them to a library-owned pinned host buffer of 64 bytes (one
 * per concurrent call, kept until the process ends), read after the
 * synchronization.
 * Gradient calls also use a library-owned side stream (non-blocking, default
 * priority; one per concurrent caller, kept until the process ends): the
 * float64 fix-ups and the finalize kernels run there while the gradient pass
 * runs on `stream`, and `stream` waits for them before the last kernel, so to
 * the caller all of the call's work is ordered on `stream`.  Calls on one
 * stream must come from one thread at a time.  The enqueue-only calls
 * (hawkes_grad_async, hawkes_leapfrog, hawkes_mwg_step, hawkes_bmds) may be
 * captured into a HIP graph: the side stream joins the capture through its
 * events (while capturing, a call that finds no pooled side stream runs in
 * order on `stream` instead of creating one). */
int hawkes_grad(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                int prec, void* ws, size_t ws_bytes, void* stream,
                double* loglik /* host or NULL */, double* grad_x /* device */, double* grad_params /* host or NULL */);

/* Same work as hawkes_grad without any host synchronization: out8 (device, 8
 * doubles) receives [loglik, d/dmu, d/dh, d/dtau, d/dtheta, d/domega, d/dxi,
 * status-as-double] when the stream reaches it.  grad_x may be NULL (then only
 * the rate pass and finalize run).  Returns only host-side argument errors. */
int hawkes_grad_async(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                      int prec, void* ws, size_t ws_bytes, void* stream, double* out8 /* device */,
                      double* grad_x /* device or NULL */);

/* hawkes_grad plus per-stage device durations: stage_ms (host, 9 floats)
 * receives the milliseconds between HIP events recorded on the call's stream
 * before and after each kernel; every stage runs in order on that stream
 * (no side stream), in launch order: prep, pack, pass1 (rates), reduce1,
 * fix-up 1 (with the flagged-row list), finalize, pass2 (gradient), fix-up 2
 * (with the finalize reduction), reduce2.  Used by the benchmark to price
 * each kernel against its roofline; the numerical results equal hawkes_grad's. */
int hawkes_grad_timed(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                      int prec, void* ws, size_t ws_bytes, void* stream,
                      double* loglik /* host or NULL */, double* grad_x /* device */,
                      double* grad_params /* host or NULL */, float* stage_ms /* host, 9 */);

/* Diagnostics of the last evaluation enqueued with workspace ws for (n, d,
 * prec, p) (hawkes_loglik, hawkes_grad, hawkes_grad_async, hawkes_grad_timed
 * or hawkes_event_terms): which rows the float64 fix-up recomputed.  The pair
 * passes take each rate lambda_n (Sec. 2.1) from sums whose terms carry the
 * scale 2^S (S = shift_log2; 0 in HAWKES_FP64); a row whose scaled rate falls
 * below cmax 2^floor_log2 (cmax = the larger pair-term weight, c_bg or c_se)
 * is recomputed exactly in float64 relative to its largest pair term instead.
 * flags (device, n int32, or NULL) receives 1 for each recomputed row and 0
 * otherwise.  Reads the workspace on `stream` after the evaluation and
 * synchronizes the stream.  Host-side argument errors: EINVAL / EPARAM. */
typedef struct {
  int64_t flagged_rows;  /* rows recomputed by the float64 fix-up */
  double shift_log2;     /* S */
  double floor_log2;     /* recompute when lambda_n 2^S < cmax 2^floor_log2 */
  double cmax;           /* max(c_bg, c_se) of Sec. 2.1's pair terms */
} hawkes_diag_t;

int hawkes_diagnostics(const void* ws /* device */, size_t ws_bytes, int64_t n, int d, int prec,
                       const hawkes_params_t* p /* host */, void* stream, int32_t* flags /* device n, or NULL */,
                       hawkes_diag_t* out /* host */);

/* hawkes_grad for callers that cannot allocate device memory: code running
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The workspace is a library-owned static device array of
 * HAWKES_NOALLOC_SCRATCH_BYTES per GPU (each GPU the library runs on holds
 * its own copy until the process ends), so the call allocates nothing and
 * creates no stream: the fix-up and finalize kernels share `stream` unless
 * a side stream is already pooled, and the scalars come back through a
 * pooled pinned buffer only if one already exists (else by a copy).  Limit: hawkes_workspace_bytes(n, d,
 * prec) <= HAWKES_NOALLOC_SCRATCH_BYTES (about n <= 18,000 at d = 2), else
 * HAWKES_ENOMEM and nothing runs.  Every call on one GPU shares its array,
 * which keeps the last call's contents (each call writes every part it
 * reads), so calls that overlap on one GPU -- from two threads, or on two
 * streams without ordering -- race and must not be issued.  Arguments,
 * outputs, synchronization and results as hawkes_grad (bitwise equal to
 * hawkes_grad with its own workspace). */
#define HAWKES_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hawkes_grad_noalloc(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                        int prec, void* stream, double* loglik /* host or NULL */, double* grad_x /* device */,
                        double* grad_params /* host or NULL */);

/* Per-event terms of the rate pass (Sec. 2.1) and the branching probability
 * used to colour events in the influenza application (Sec. 4.3): the
 * self-excitation share of the rate, xi(x_n, t_n) / lambda_n.  terms (device,
 * n x 4 row-major float64) receives per event
 *   [0] a_n = background rate at event n per unit mu0,
 *   [1] b_n = self-excitation rate at event n per unit theta,
 *   [2] log lambda_n, lambda_n = mu0 a_n + theta b_n (exact even where lambda_n
 *       underflows float64; a_n and b_n are then 0),
 *   [3] theta b_n / lambda_n.
 * Runs the rate pass and finalize (no gradient pass); loglik (host or NULL)
 * receives ell.  Synchronizes the stream.  Returns HAWKES_EZERORATE, with the
 * terms written, when some lambda_n is 0. */
int hawkes_event_terms(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                       int prec, void* ws, size_t ws_bytes, void* stream, double* terms /* device, n*4 */,
                       double* loglik /* host or NULL */);

/* ------------------------------------------------------------------------
 * Metropolis-within-Gibbs location updates (Sec. 3: block-wise Metropolis
 * moves of individual latent locations).  Moving the locations of a block of
 * events changes each rate only through its pairs with the moved events and
 * leaves every compensator term unchanged, so with the per-event terms of
 * hawkes_event_terms cached, the change of the log-likelihood costs
 * O(N * nmove) pair terms instead of a full O(N^2) pass.  All float64.
 */

/* Device workspace of hawkes_mwg_step for n events (0 if n is invalid). */
size_t hawkes_mwg_workspace_bytes(int64_t n);

/* One Metropolis step for the block of events idx[0..nmove) (device, int64,
 * strictly increasing, each in [0, n)) proposed at x_new (device, nmove x d).
 * Computes Delta ell = ell(x with the block moved) - ell(x) and accepts iff
 * Delta ell > *log_thresh (device, 1 double), where the caller folds the
 * uniform draw, the proposal ratio and the prior ratio into the threshold:
 * log u - log q(x*|x) + log q(x|x*) - log p(x*) + log p(x).
 * On accept the moved rows of x (device, n x d) are overwritten and terms
 * (device, n x 4, from hawkes_event_terms with the same parameters, every
 * lambda_n > 0) is updated in place; on reject nothing changes.
 * out3 (device, 3 doubles) receives [Delta ell, accepted (0 or 1), status].
 * Rows whose rate, or either part of it (a or b), the move cancels to below
 * 2^-16 of the terms it is formed from are recomputed exactly; other rows are
 * updated incrementally, so after many accepted moves a periodic
 * hawkes_event_terms refresh bounds the drift.
 * Enqueue only: no host synchronization.  Host-side argument errors return at
 * once; an invalid idx or non-finite x_new is reported in out3 (status
 * HAWKES_EDATA, Delta ell NaN, rejected).  Calls sharing a workspace must be
 * ordered on one stream. */
int hawkes_mwg_step(double* x /* device, n*d */, const double* t, int64_t n, int d,
                    const hawkes_params_t* p /* host */, double* terms /* device, n*4 */,
                    const int64_t* idx /* device, nmove */, const double* x_new /* device, nmove*d */,
                    int64_t nmove, const double* log_thresh /* device, 1 */, void* ws, size_t ws_bytes,
                    void* stream, double* out3 /* device, 3 */);

/* Log-likelihood at new weights mu0 = p->mu and theta = p->theta with every
 * other parameter equal to those the terms were computed with (Sec. 2.1:
 * lambda_n is linear in mu0 and theta, and so is Lambda_n), in O(N) from the
 * cached terms.  out3 (device) receives [ell, d ell/d mu, d ell/d theta].
 * Enqueue only. */
int hawkes_loglik_reweight(const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                           const double* terms /* device, n*4 */, void* stream, double* out3 /* device, 3 */);

/* ------------------------------------------------------------------------
 * Hamiltonian Monte Carlo trajectories over the latent locations (Sec. 3:
 * leapfrog with unit mass; Sec. 2.2: each location confined to a box or a
 * disc around its observed position).  A wall mirrors the motion: in a box
 * the momentum component normal to the wall changes sign; on a disc (a ball
 * when d > 2) the momentum is reflected about the normal at the contact point.
 */
typedef enum {
  HAWKES_BOUND_NONE = 0,  /* unconstrained */
  HAWKES_BOUND_BOX = 1,   /* b0 = lower corners (n x d), b1 = upper corners (n x d); equal bounds pin the coordinate */
  HAWKES_BOUND_DISC = 2   /* b0 = centres (n x d), b1 = radii (n); radius 0 pins the location */
} hawkes_bound_t;

/* `steps` leapfrog steps of size eps for the potential -ell(x):
 *   p += eps/2 grad_x ell;  repeat { x flies for time eps with reflections;
 *   p += eps grad_x ell (eps/2 after the last flight) }.
 * x, p (device, n x d) are updated in place.  grad_x (device, n x d) holds
 * grad_x ell at the entry x when have_grad != 0 (else it is computed first) and
 * receives the gradient at the final x, so consecutive trajectories can chain.
 * out8 (device) receives the final evaluation's [ell, 6 parameter gradients,
 * status].  Every gradient is a full evaluation at precision prec enqueued on
 * `stream`; no host synchronization.  ws: as for hawkes_grad.  The locations
 * must start inside their bounds.  A flight that meets more than 64 disc walls
 * stops at the wall.  Host-side argument errors return at once. */
int hawkes_leapfrog(double* x /* device, n*d */, double* p /* device, n*d */, const double* t, int64_t n, int d,
                    const hawkes_params_t* prm /* host */, int prec, double eps, int steps, int bound,
                    const double* b0 /* device or NULL */, const double* b1 /* device or NULL */, void* ws,
                    size_t ws_bytes, void* stream, double* grad_x /* device, n*d */, int have_grad,
                    double* out8 /* device, 8 */);

/* ------------------------------------------------------------------------
 * Bayesian multidimensional scaling (Sec. 2.2.3, eq. bmdsLikelihood): the
 * second pairwise term of the influenza model's posterior.  Observed
 * dissimilarities delta_{nn'} (n > n') are independent normals with mean
 * d_{nn'} = |x_n - x_n'| and variance sigma^2, truncated to positive values:
 *   ell = -(M/2) log sigma^2 - sum_{n>n'} [ (delta - d)^2/(2 sigma^2) + log Phi(d/sigma) ]
 * (the paper's density up to its constant), M = number of observed pairs.
 */

/* Device workspace of hawkes_bmds (0 if n or d is invalid; n <= 2^20). */
size_t hawkes_bmds_workspace_bytes(int64_t n, int d);

/* ell, d ell/d sigma and (unless grad_x is NULL) d ell/d x for the latent
 * locations x (device, n x d row-major float64) and the dissimilarities delta
 * (device, n x n row-major float64; only the strict lower triangle
 * delta[i*n + j], j < i, is read; NaN marks an unobserved pair, a negative or
 * infinite entry is a data error).  prec: HAWKES_FP64, or HAWKES_MIXED (float32
 * pair arithmetic, float64 sums).  out4 (device) receives [ell, d ell/d sigma,
 * M, status]; on a data error ell and d ell/d sigma are NaN, status is
 * HAWKES_EDATA and grad_x is NaN.  A coincident pair (d = 0) adds no direction
 * to the gradient.  Enqueue only; host-side argument errors return at once
 * (sigma must be finite and > 0: HAWKES_EPARAM). */
int hawkes_bmds(const double* x, const double* delta, int64_t n, int d, double sigma, int prec, void* ws,
                size_t ws_bytes, void* stream, double* out4 /* device, 4 */, double* grad_x /* device or NULL */);

/* Leapfrog trajectory for the influenza model (Sec. 3: HMC over the latent
 * locations evaluates both the Hawkes likelihood and the MDS likelihood of
 * eq. bmdsLikelihood, and both gradients, at every step): as hawkes_leapfrog
 * with the potential -(ell_hawkes(x) + ell_mds(x)), so every gradient is the
 * sum of hawkes_grad's and hawkes_bmds's location gradients (formed as the
 * Hawkes gradient, then the MDS gradient added in place).  delta, sigma: as
 * for hawkes_bmds; bws (device, hawkes_bmds_workspace_bytes(n, d) bytes) is
 * the MDS workspace.  out8 receives the final Hawkes evaluation and out4
 * (device, 4) the final MDS evaluation, both as from the single calls.  The
 * MDS term runs at prec without HAWKES_CULL.  Host-side argument errors return
 * at once; enqueue only. */
int hawkes_leapfrog_bmds(double* x /* device, n*d */, double* p /* device, n*d */, const double* t, int64_t n, int d,
                         const hawkes_params_t* prm /* host */, int prec, const double* delta /* device, n*n */,
                         double sigma, double eps, int steps, int bound, const double* b0 /* device or NULL */,
                         const double* b1 /* device or NULL */, void* ws, size_t ws_bytes, void* bws,
                         size_t bws_bytes, void* stream, double* grad_x /* device, n*d */, int have_grad,
                         double* out8 /* device, 8 */, double* out4 /* device, 4 */);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of evaluation requests from many HMC chains
 * (one request = one log-likelihood + gradient at new latent locations).
 *
 * A server owns an HBM arena of hbm_budget_bytes, allocated once by
 * hawkes_serve_create (the only allocation; evaluation never allocates).  A
 * scheduler thread admits submitted requests in arrival order while fewer
 * than max_slots are in flight and the request's footprint
 * (hawkes_serve_footprint) fits in the arena; admitted requests of the same
 * (d, precision) form a batch that runs as one kernel launch per phase on one
 * of several HIP streams, so batches overlap on the device and requests that
 * arrive meanwhile are admitted as slots and memory free up.  A request's
 * result is bitwise identical whether it runs alone or in any batch.
 *
 * Threading: every call may come from any host thread.  x and grad_x stay
 * owned by the client and must stay alive until the request completes.
 * ------------------------------------------------------------------------ */
typedef struct hawkes_server hawkes_server_t;

typedef struct {
  int status;              /* HAWKES_OK, or the request's error (e.g. HAWKES_EDATA) */
  double loglik;           /* ell */
  double grad_params[6];   /* API order */
  uint64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns;   /* steady clock */
} hawkes_result_t;

typedef struct {
  int64_t pending;             /* submitted, not yet admitted */
  int64_t active;              /* admitted, not yet complete */
  uint64_t batches_launched;
  uint64_t requests_submitted;
  uint64_t arena_bytes, arena_free_bytes;
} hawkes_serve_stats_t;

/* flags for hawkes_serve_create: low 8 bits = number of streams (0: 2, max 8);
 * HAWKES_SERVE_SIMULATE runs the scheduler without a GPU (requests complete
 * after a virtual delay with loglik 0), for testing admission and queueing. */
#define HAWKES_SERVE_SIMULATE 0x100

/* Device bytes one admitted request of (n, d, prec) holds (0 if invalid). */
size_t hawkes_serve_footprint(int64_t n, int d, int prec);

/* Create a server (allocates the arena, streams and pinned staging).
 * EINVAL: max_slots outside [1, 1024] or budget below 1 MiB; EDEVICE: HIP failure. */
int hawkes_serve_create(size_t hbm_budget_bytes, int max_slots, int flags, hawkes_server_t** out);

/* A source of device memory for a server, e.g. a framework's caching
 * allocator, so the server's memory shows in the framework's accounting.
 * alloc returns `bytes` of device memory aligned to 256 bytes (NULL on
 * failure); free takes back a pointer alloc returned.  Both are called only
 * from hawkes_serve_create_with, hawkes_serve_register and
 * hawkes_serve_destroy, on the calling thread (never by the scheduler). */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} hawkes_allocator_t;

/* As hawkes_serve_create, with every device buffer of the server (the arena,
 * the per-stream descriptor and result slots, the registered datasets' times)
 * taken from `alloc` and given back to it by hawkes_serve_destroy; the pinned
 * host staging still comes from hipHostMalloc.  alloc == NULL: hipMalloc.  A
 * buffer that comes back misaligned is returned and counts as a failure
 * (EDEVICE); alloc with a NULL function: EINVAL. */
int hawkes_serve_create_with(const hawkes_allocator_t* alloc, size_t hbm_budget_bytes, int max_slots, int flags,
                             hawkes_server_t** out);

/* Register a dataset's event times (device, n, sorted) for dimension d; the
 * server keeps its own device copy.  Returns the dataset id. */
int hawkes_serve_register(hawkes_server_t* s, const double* t /* device */, int64_t n, int d, int32_t* dataset_id);

/* Queue one evaluation.  x: device n*d float64 of the registered dataset's n
 * and d; grad_x: device n*d output or NULL.  Checked on the host: EPARAM for
 * invalid parameters, ENOMEM if the footprint can never fit the arena, ESTATE
 * for an unknown dataset or a server being destroyed.  Data errors (NaN in x)
 * surface later as that request's result status only. */
int hawkes_serve_submit(hawkes_server_t* s, int32_t dataset_id, const double* x /* device */,
                        const hawkes_params_t* p /* host */, int prec, double* grad_x /* device or NULL */,
                        uint64_t* ticket);

/* HAWKES_EPENDING until done; then copies the result, forgets the ticket and
 * returns HAWKES_OK.  ESTATE for an unknown (or already collected) ticket. */
int hawkes_serve_poll(hawkes_server_t* s, uint64_t ticket, hawkes_result_t* out);

/* Blocks until done (timeout_ns < 0: no limit); ETIMEOUT leaves it pending. */
int hawkes_serve_wait(hawkes_server_t* s, uint64_t ticket, hawkes_result_t* out, int64_t timeout_ns);

int hawkes_serve_stats(hawkes_server_t* s, hawkes_serve_stats_t* out);

/* Stops admission of new submissions, drains every queued and in-flight
 * request, and frees the server. */
int hawkes_serve_destroy(hawkes_server_t* s);

/* Human-readable text for a status code (static storage). */
const char* hawkes_strerror(int status);

/* Library version string "major.minor.patch" (static storage). */
const char* hawkes_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HAWKES_H_ */
