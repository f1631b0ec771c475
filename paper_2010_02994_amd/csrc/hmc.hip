// libhawkes: device-resident Hamiltonian Monte Carlo trajectories over the
// latent locations (arXiv 2010.02994, Sec. 3: leapfrog integration with unit
// mass; Sec. 2.2: each location confined to a box or a disc around its
// observed position, the walls reflecting the motion).
//
// One trajectory of L steps of size eps is
//   p += eps/2 grad ell(x);  then L times { x moves for time eps with
//   reflections (momentum mirrored at each wall);  g = grad ell(x);
//   p += eps g (eps/2 on the last step) }
// where every gradient is the full evaluation of the library, enqueued on the
// caller's stream; nothing returns to the host between steps.  For the
// influenza model ell is the Hawkes log-likelihood plus the Bayesian MDS
// log-likelihood of the same locations (Sec. 3), and g sums both gradients.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/hawkes.h"
#include "hawkes_common.hpp"
#include "hawkes_internal.hpp"

namespace hawkes {
namespace hmc {

constexpr int kBlock = 256;
constexpr int kMaxBounces = 64;   // disc walls hit within one step before the motion stops at the wall

// Free flight for time eps inside [lo, hi] in one coordinate: the unfolded
// offset u = x - lo + eps p folds back with period 2 (hi - lo); an odd number
// of wall hits mirrors the momentum.  A zero-width interval pins x at lo.
__device__ __forceinline__ void fly_box(double& x, double& p, double lo, double hi, double eps) {
  const double w = hi - lo;
  if (!(w > 0.0)) {
    x = lo;
    return;
  }
  const double u = (x - lo) + eps * p;
  double m = fmod(u, 2.0 * w);
  if (m < 0.0) m += 2.0 * w;
  if (m <= w) {
    x = lo + m;
  } else {
    x = lo + (2.0 * w - m);
    p = -p;
  }
}

// Free flight for time eps inside the ball |x - c| <= r with specular
// reflection at the sphere: time to the wall from the root of
// |y + s p|^2 = r^2 (the form without cancellation for either sign of y.p),
// then p -= 2 (p.n) n with n the outward normal at the contact point.
template <int D>
__device__ __forceinline__ void fly_disc(double* x, double* p, const double* c, double r, double eps) {
  double y[D];
#pragma unroll
  for (int q = 0; q < D; ++q) y[q] = x[q] - c[q];
  if (!(r > 0.0)) {
#pragma unroll
    for (int q = 0; q < D; ++q) x[q] = c[q];
    return;
  }
  const double r2 = r * r;
  double rem = eps;
  for (int it = 0; it < kMaxBounces && rem > 0.0; ++it) {
    double pp = 0.0, yp = 0.0, yy = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      pp = fma(p[q], p[q], pp);
      yp = fma(y[q], p[q], yp);
      yy = fma(y[q], y[q], yy);
    }
    if (pp == 0.0) break;
    const double room = fmax(r2 - yy, 0.0);
    const double sq = sqrt(fma(yp, yp, pp * room));
    const double s = yp > 0.0 ? room / (yp + sq) : (sq - yp) / pp;
    if (s >= rem) {
#pragma unroll
      for (int q = 0; q < D; ++q) y[q] = fma(rem, p[q], y[q]);
      rem = 0.0;
      break;
    }
#pragma unroll
    for (int q = 0; q < D; ++q) y[q] = fma(s, p[q], y[q]);
    rem -= s;
    double ny = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) ny = fma(y[q], y[q], ny);
    const double inv = 1.0 / sqrt(ny);
    double pn = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) pn = fma(p[q], y[q] * inv, pn);
#pragma unroll
    for (int q = 0; q < D; ++q) p[q] -= 2.0 * pn * y[q] * inv;
  }
  // rounding can leave the point a hair outside: put it back on the wall
  double yy = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) yy = fma(y[q], y[q], yy);
  if (yy > r2) {
    const double k = r / sqrt(yy);
#pragma unroll
    for (int q = 0; q < D; ++q) y[q] *= k;
  }
#pragma unroll
  for (int q = 0; q < D; ++q) x[q] = c[q] + y[q];
}

// p += kick * g, then free flight for time eps (flight = 0: kick only).
template <int D>
__global__ void __launch_bounds__(kBlock) k_kick_fly(double* __restrict__ x, double* __restrict__ p,
                                                     const double* __restrict__ g, int n, double kick, double eps,
                                                     int bound, const double* __restrict__ b0,
                                                     const double* __restrict__ b1, int flight) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double xi[D], pi[D];
#pragma unroll
  for (int q = 0; q < D; ++q) {
    xi[q] = x[(int64_t)i * D + q];
    pi[q] = fma(kick, g[(int64_t)i * D + q], p[(int64_t)i * D + q]);
  }
  if (flight) {
    if (bound == HAWKES_BOUND_BOX) {
#pragma unroll
      for (int q = 0; q < D; ++q) fly_box(xi[q], pi[q], b0[(int64_t)i * D + q], b1[(int64_t)i * D + q], eps);
    } else if (bound == HAWKES_BOUND_DISC) {
      double c[D];
#pragma unroll
      for (int q = 0; q < D; ++q) c[q] = b0[(int64_t)i * D + q];
      fly_disc<D>(xi, pi, c, b1[i], eps);
    } else {
#pragma unroll
      for (int q = 0; q < D; ++q) xi[q] = fma(eps, pi[q], xi[q]);
    }
#pragma unroll
    for (int q = 0; q < D; ++q) x[(int64_t)i * D + q] = xi[q];
  }
#pragma unroll
  for (int q = 0; q < D; ++q) p[(int64_t)i * D + q] = pi[q];
}

template <int D>
static void kick_fly(double* x, double* p, const double* g, int n, double kick, double eps, int bound,
                     const double* b0, const double* b1, bool flight, hipStream_t s) {
  k_kick_fly<D><<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(x, p, g, n, kick, eps, bound, b0, b1, flight ? 1 : 0);
}

static void kick_fly_d(int d, double* x, double* p, const double* g, int n, double kick, double eps, int bound,
                       const double* b0, const double* b1, bool flight, hipStream_t s) {
  switch (d) {
    case 1: kick_fly<1>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 2: kick_fly<2>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 3: kick_fly<3>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 4: kick_fly<4>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 5: kick_fly<5>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 6: kick_fly<6>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 7: kick_fly<7>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
    case 8: kick_fly<8>(x, p, g, n, kick, eps, bound, b0, b1, flight, s); break;
  }
}

// The optional second term of the potential: the Bayesian MDS likelihood of
// the same locations (the influenza model, whose HMC over the latent
// locations needs the gradients of both the Hawkes and the MDS likelihoods).
struct MdsTerm {
  const double* delta;
  double sigma;
  void* ws;
  size_t ws_bytes;
  double* out4;
};

// grad_x = the location gradient of the potential's log density at x.  With
// the MDS term, its pair pass runs on a side stream beside the Hawkes
// evaluation (both only read x), and its gradient is added on the caller's
// stream once both are done.
static int gradient(double* x, const double* t, int64_t n, int d, const hawkes_params_t* prm, int prec, void* ws,
                    size_t ws_bytes, hipStream_t s, double* grad_x, double* out8, const MdsTerm* mds) {
  const int mprec = prec & ~HAWKES_CULL;
  Fork* fk = nullptr;
  int dev = -1;
  if (mds && hipGetDevice(&dev) == hipSuccess) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    fk = fork_take(dev, !capturing);
  }
  int st = HAWKES_OK;
  if (fk) {
    if (hipEventRecord(fk->ready, s) != hipSuccess || hipStreamWaitEvent(fk->side, fk->ready, 0) != hipSuccess)
      st = HAWKES_EDEVICE;
    if (st == HAWKES_OK)
      st = bmds_enqueue(x, mds->delta, n, d, mds->sigma, mprec, mds->ws, mds->ws_bytes, fk->side, mds->out4,
                        grad_x, true, 1);
    if (st == HAWKES_OK && hipEventRecord(fk->done, fk->side) != hipSuccess) st = HAWKES_EDEVICE;
  }
  if (st == HAWKES_OK) st = run_async(x, t, n, d, prm, prec, ws, ws_bytes, s, out8, grad_x);
  if (st == HAWKES_OK && mds) {
    if (fk) {
      st = hipStreamWaitEvent(s, fk->done, 0) == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
      if (st == HAWKES_OK)
        st = bmds_enqueue(x, mds->delta, n, d, mds->sigma, mprec, mds->ws, mds->ws_bytes, s, mds->out4, grad_x,
                          true, 2);
    } else {
      st = bmds_enqueue(x, mds->delta, n, d, mds->sigma, mprec, mds->ws, mds->ws_bytes, s, mds->out4, grad_x,
                        true, 0);
    }
  }
  if (fk) {
    // an early error leaves the side stream's work unjoined: join it so the
    // fork goes back to the pool with nothing pending against this call
    if (st != HAWKES_OK) (void)hipStreamWaitEvent(s, fk->done, 0);
    fork_give(dev, fk);
  }
  return st;
}

static int leapfrog(double* x, double* p, const double* t, int64_t n, int d, const hawkes_params_t* prm, int prec,
                    double eps, int steps, int bound, const double* b0, const double* b1, void* ws, size_t ws_bytes,
                    void* stream, double* grad_x, int have_grad, double* out8, const MdsTerm* mds) {
  if (!x || !p || !t || !prm || !ws || !grad_x || !out8) return HAWKES_EINVAL;
  if (steps < 1 || !std::isfinite(eps) || !(eps > 0.0)) return HAWKES_EINVAL;
  if (bound != HAWKES_BOUND_NONE && bound != HAWKES_BOUND_BOX && bound != HAWKES_BOUND_DISC) return HAWKES_EINVAL;
  if (bound != HAWKES_BOUND_NONE && (!b0 || !b1)) return HAWKES_EINVAL;
  const size_t need = hawkes_workspace_bytes(n, d, prec);
  if (need == 0 || ws_bytes < need) return HAWKES_EINVAL;
  if (!valid_params(prm)) return HAWKES_EPARAM;
  if (mds) {
    if (!mds->delta || !mds->ws || !mds->out4) return HAWKES_EINVAL;
    const size_t bneed = hawkes_bmds_workspace_bytes(n, d);
    if (bneed == 0 || mds->ws_bytes < bneed) return HAWKES_EINVAL;
    if (!std::isfinite(mds->sigma) || !(mds->sigma > 0.0)) return HAWKES_EPARAM;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = HAWKES_OK;
  if (!have_grad) st = gradient(x, t, n, d, prm, prec, ws, ws_bytes, s, grad_x, out8, mds);
  for (int k = 0; k < steps && st == HAWKES_OK; ++k) {
    (void)hipGetLastError();
    kick_fly_d(d, x, p, grad_x, (int)n, k == 0 ? 0.5 * eps : eps, eps, bound, b0, b1, true, s);
    if (hipGetLastError() != hipSuccess) return HAWKES_EDEVICE;
    st = gradient(x, t, n, d, prm, prec, ws, ws_bytes, s, grad_x, out8, mds);
  }
  if (st != HAWKES_OK) return st;
  (void)hipGetLastError();
  kick_fly_d(d, x, p, grad_x, (int)n, 0.5 * eps, eps, bound, b0, b1, false, s);
  return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // namespace hmc
}  // namespace hawkes

extern "C" {

int hawkes_leapfrog(double* x, double* p, const double* t, int64_t n, int d, const hawkes_params_t* prm, int prec,
                    double eps, int steps, int bound, const double* b0, const double* b1, void* ws, size_t ws_bytes,
                    void* stream, double* grad_x, int have_grad, double* out8) {
  return hawkes::hmc::leapfrog(x, p, t, n, d, prm, prec, eps, steps, bound, b0, b1, ws, ws_bytes, stream, grad_x,
                               have_grad, out8, nullptr);
}

int hawkes_leapfrog_bmds(double* x, double* p, const double* t, int64_t n, int d, const hawkes_params_t* prm,
                         int prec, const double* delta, double sigma, double eps, int steps, int bound,
                         const double* b0, const double* b1, void* ws, size_t ws_bytes, void* bws, size_t bws_bytes,
                         void* stream, double* grad_x, int have_grad, double* out8, double* out4) {
  const hawkes::hmc::MdsTerm mds{delta, sigma, bws, bws_bytes, out4};
  return hawkes::hmc::leapfrog(x, p, t, n, d, prm, prec, eps, steps, bound, b0, b1, ws, ws_bytes, stream, grad_x,
                               have_grad, out8, &mds);
}

}  // extern "C"
