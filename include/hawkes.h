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
  HAWKES_FP64 = 0,  /* every step in float64; exp from the device math library */
  HAWKES_MIXED = 1  /* pair arithmetic and exp in float32, all sums, logs, the
                       compensator and final reductions in float64 */
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
 * either may be NULL.  Synchronizes the stream to deliver them. */
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

/* hawkes_grad plus per-stage device durations: stage_ms (host, 12 floats)
 * receives the milliseconds between HIP events recorded on the call's stream
 * before and after each kernel, in launch order: prep, pack, pass1 (rates),
 * reduce1, flag list, fix-up 1, finalize, finalize reduction, pass2
 * (gradient), fix-up 2b, fix-up 2a, reduce2.  Used by the benchmark to price
 * each kernel against its roofline; the numerical results equal hawkes_grad's. */
int hawkes_grad_timed(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p /* host */,
                      int prec, void* ws, size_t ws_bytes, void* stream,
                      double* loglik /* host or NULL */, double* grad_x /* device */,
                      double* grad_params /* host or NULL */, float* stage_ms /* host, 12 */);

/* Human-readable text for a status code (static storage). */
const char* hawkes_strerror(int status);

/* Library version string "major.minor.patch" (static storage). */
const char* hawkes_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HAWKES_H_ */
