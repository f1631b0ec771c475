// libhawkes: Bayesian multidimensional scaling log-likelihood and its
// gradients (arXiv 2010.02994, Sec. 2.2.3, eq. bmdsLikelihood), the second
// pairwise term of the influenza model's posterior.
//
// For observed dissimilarities delta_{nn'} (n > n'), d_{nn'} = |x_n - x_n'|:
//   ell = -(M/2) log sigma^2 - sum_{n>n'} [ (delta - d)^2 / (2 sigma^2) + log Phi(d / sigma) ]
//   d ell/d x_n   = sum_{n'} [ (delta - d)/sigma^2 - rho/sigma ] (x_n - x_n') / d,  rho = phi(z)/Phi(z), z = d/sigma
//   d ell/d sigma = -M/sigma + sum [ (delta - d)^2/sigma^3 + rho z / sigma ]
// M counts the observed pairs (a NaN delta is unobserved).  The pass streams
// the strict lower triangle of the N x N matrix once: it is bound by HBM when
// the pair arithmetic is float32 and close to balanced in float64.
//
// Tiles: row band I (rows [64 I, 64 I + 64)) meets column chunks
// J = 0 .. floor(I / 4) of 256 columns.  A workgroup takes one tile, C columns
// per lane (C runs of 64 columns per wave), and walks the 64 rows: the lanes
// of a wave read consecutive delta entries (coalesced 512 B row segments).
// Column sums stay in each lane.  A row's sum is first formed in the lane over
// its C columns, then over each 16-lane row of the wave by DPP row shifts; the
// partials of the 16-lane rows and of the waves are added at the end in a
// fixed order.  With C columns per lane the cross-lane work per pair falls by
// C.  Per-tile partials are reduced per event in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "../../include/hawkes.h"
#include "hawkes_common.hpp"
#include "hawkes_internal.hpp"

namespace hawkes {
namespace bmds {

constexpr int kTR = 64;        // rows per tile
constexpr int kTC = 256;       // columns per tile
constexpr int kFinalThreads = 1024;
constexpr int kPrefetch = 8;   // rows whose entries are loaded ahead of their arithmetic
#ifndef HK_BMDS_COLS_MIXED
#define HK_BMDS_COLS_MIXED 4
#endif
#ifndef HK_BMDS_COLS_FP64
#define HK_BMDS_COLS_FP64 2
#endif
constexpr int kColsMixed = HK_BMDS_COLS_MIXED;   // columns per lane, float32 pairs, many tiles
constexpr int kColsFp64 = HK_BMDS_COLS_FP64;     // columns per lane, float64 pairs, many tiles
constexpr int64_t kWideTiles = 4096;             // fewer tiles: one column per lane

// First tile of row band I: sum over I' < I of (floor(I'/4) + 1).
__host__ __device__ inline int64_t band_offset(int64_t I) {
  const int64_t q = I / 4, r = I % 4;
  return I + 2 * q * (q - 1) + r * q;
}

struct Args {
  const double* x;
  const double* delta;
  int n, nb;
  int64_t ntiles;
  double sigma, inv_sigma, inv_s2;
  double* prow;   // ntiles x kTR x D
  double* pcol;   // ntiles x kTC x D
  double* ptile;  // ntiles x 4: sum of summands, sum of sigma terms, pairs, invalid deltas
  double* out4;   // [ell, d ell/d sigma, pairs, status]
  double* grad_x; // n x D or null
  int accumulate; // 1: grad_x += the gradient (0: grad_x = the gradient)
};

// DPP reads of a lane in the same row of 16 (row shifts); lanes without a
// source read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int ROWS, typename R>
__device__ __forceinline__ R dpp_step(R v) {
  if constexpr (std::is_same<R, float>::value) return dpp_f<CTRL, ROWS>(v);
  else return dpp_d<CTRL, ROWS>(v);
}

// erfc(w) for w >= 0 in float32: the Chebyshev-fitted form
// t exp(-w^2 + P(t)), t = 1/(1 + w/2), of Press et al., Numerical Recipes
// (2nd ed., Sec. 6.2, "erfcc"), relative error below 1.2e-7 for all w >= 0,
// built on the hardware reciprocal and base-2 exponential.
// Beyond z = 6 the upper tail q = erfc(z/sqrt2)/2 < 1e-9 (erfc_cheb's
// relative error is below 1.2e-7), far below half a float32 unit of 1
// (2^-25 = 3.0e-8), so 1 - q rounds to exactly 1.
#ifndef HK_BMDS_FAR_Z
#define HK_BMDS_FAR_Z 6.0f
#endif
constexpr float kFarZ = HK_BMDS_FAR_Z;

__device__ __forceinline__ float erfc_cheb(float w) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, w, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  return t * __builtin_amdgcn_exp2f((p - w * w) * 1.44269504088896341f);
}

// Summand, sigma term and gradient coefficient of one observed pair.  The
// upper tail q = 1 - Phi(z) is formed directly, so log Phi keeps small tails.
template <typename R>
__device__ __forceinline__ void pair_terms(R r2, R delta, R inv_sigma, R inv_s2, R& term, R& dsig, R& coef) {
  if constexpr (std::is_same<R, float>::value) {
    // d and 1/d from one reciprocal square root (d = 0 adds no direction)
    const float rs = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
    const float dist = r2 * rs;
    const float z = dist * inv_sigma;
    const float res = delta - dist;
    const float pdf = 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * z * z);
    float lphi, rho;
    if (__all(z > kFarZ)) {
      // every pair of the wave lies beyond kFarZ standard deviations: there
      // 1 - q rounds to 1 in float32, so log(phi) = 0 and pdf / phi = pdf
      // exactly, and the erfc, log and reciprocal are skipped
      lphi = 0.0f;
      rho = pdf;
    } else {
      const float q = 0.5f * erfc_cheb(z * 0.70710678118654752f);
      const float phi = 1.0f - q;
      lphi = __builtin_amdgcn_logf(phi) * 0.69314718055994531f;
      rho = pdf * __builtin_amdgcn_rcpf(phi);
    }
    term = -0.5f * res * res * inv_s2 - lphi;
    dsig = (res * res * inv_s2 + rho * z) * inv_sigma;
    coef = (res * inv_s2 - rho * inv_sigma) * rs;
  } else {
    const double dist = sqrt(r2);
    const double z = dist * inv_sigma;
    const double res = delta - dist;
    const double q = 0.5 * erfc(z * 0.70710678118654752440);
    const double pdf = 0.39894228040143267794 * exp(-0.5 * z * z);
    double lphi, rho;
    if (__all(z > (double)kFarZ)) {
      // q < 1e-9 on every lane: log(1 - q) = -q (1 + q/2 + q^2/3 + ...) and
      // 1/(1 - q) = 1 + q + q^2 + ..., both truncated below q^3 < 1e-27
      lphi = -q * __builtin_fma(q, __builtin_fma(q, 1.0 / 3.0, 0.5), 1.0);
      rho = pdf * __builtin_fma(q, 1.0 + q, 1.0);
    } else {
      lphi = log1p(-q);
      rho = pdf / (1.0 - q);
    }
    term = -0.5 * res * res * inv_s2 - lphi;
    dsig = (res * res * inv_s2 + rho * z) * inv_sigma;
    coef = dist > 0.0 ? (res * inv_s2 - rho * inv_sigma) / dist : 0.0;
  }
}

// Lanes per workgroup and prefetched rows of a tile pass with C columns per lane.
#ifndef HK_BMDS_PRE_WIDE
#define HK_BMDS_PRE_WIDE 4
#endif
template <int C>
struct TileShape {
  static constexpr int kLanes = kTC / C;                         // workgroup size
  static constexpr int kWavesT = kLanes / 64;
  static constexpr int kPre = C >= 4 ? HK_BMDS_PRE_WIDE : kPrefetch;   // rows loaded ahead
  // partial row sums per wave: one column per lane reduces over the whole
  // wave (row broadcasts 15 and 31 after the row shifts); wider lanes stop at
  // the four 16-lane rows
  static constexpr int kParts = C == 1 ? 1 : 4;
};

template <int D, bool MIX, int C>
__global__ void __launch_bounds__(TileShape<C>::kLanes) k_bmds_tiles(Args a) {
  using R = typename std::conditional<MIX, float, double>::type;
  using TS = TileShape<C>;
  constexpr int NL = TS::kLanes, NW = TS::kWavesT, PRE = TS::kPre, NP = TS::kParts;
  __shared__ R s_x[kTR][D];
  __shared__ R s_row[NW][kTR][NP][D];   // partial row sums
  __shared__ double sh[4 * NL];
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = a.nb - 1;   // band: largest I with band_offset(I) <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (band_offset(mid) <= tile) lo = mid;
    else hi = mid - 1;
  }
  const int I = lo;
  const int J = (int)(tile - band_offset(I));
  const int i0 = I * kTR;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // columns of this lane: C runs of 64, so each row's loads stay coalesced
  int jc[C], jl[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    jl[c] = w * 64 * C + c * 64 + lane;
    jc[c] = J * kTC + jl[c];
  }
  // the band's first tile also counts its rows' non-finite coordinates, so
  // every event is checked once
  int bad = 0;
  for (int e = threadIdx.x; e < kTR * D; e += NL) {
    const int r = e / D, q = e % D;
    const int i = i0 + r;
    const double xv = i < a.n ? a.x[(int64_t)i * D + q] : 0.0;
    if (J == 0 && !isfinite(xv)) ++bad;
    s_x[r][q] = (R)xv;
  }
  R xj[C][D], g[C][D], tsum[C], dsum[C];
  int cnt = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    tsum[c] = R(0);
    dsum[c] = R(0);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      xj[c][q] = jc[c] < a.n ? (R)a.x[(int64_t)jc[c] * D + q] : R(0);
      g[c][q] = R(0);
    }
  }
  const R inv_sigma = (R)a.inv_sigma, inv_s2 = (R)a.inv_s2;
  __syncthreads();
  const int rows = min(kTR, a.n - i0);
  for (int r0 = 0; r0 < rows; r0 += PRE) {
    // the next rows' entries first, so PRE x C loads are in flight at once;
    // every load is issued (its address clamped into the matrix) and the
    // entries outside the triangle are masked afterwards, so no branch
    // separates the loads and each row waits only for its own entries
    double v[PRE][C];
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int i = min(i0 + r0 + u, a.n - 1);
#pragma unroll
      for (int c = 0; c < C; ++c) v[u][c] = a.delta[(int64_t)i * a.n + min(jc[c], a.n - 1)];
    }
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int r = r0 + u;
      if (r >= rows) break;
      R gi[D];
#pragma unroll
      for (int q = 0; q < D; ++q) gi[q] = R(0);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double dv = v[u][c];
        if (jc[c] < i0 + r && !isnan(dv)) {
          if (dv < 0.0 || isinf(dv)) {
            bad += 1;
          } else {
            R diff[D], r2 = R(0);
#pragma unroll
            for (int q = 0; q < D; ++q) {
              diff[q] = s_x[r][q] - xj[c][q];
              r2 += diff[q] * diff[q];
            }
            R term, dsig, coef;
            pair_terms<R>(r2, (R)dv, inv_sigma, inv_s2, term, dsig, coef);
            tsum[c] += term;
            dsum[c] += dsig;
            cnt += 1;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const R gq = coef * diff[q];
              gi[q] += gq;
              g[c][q] -= gq;
            }
          }
        }
      }
      // 16-lane row sums (row shifts 1, 2, 4, 8 leave each row's total in
      // its lane 15), one step at a time across the D values so no DPP read
      // waits on the add just before it
#pragma unroll
      for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x111, 0xf>(gi[q]);
#pragma unroll
      for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x112, 0xf>(gi[q]);
#pragma unroll
      for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x114, 0xf>(gi[q]);
#pragma unroll
      for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x118, 0xf>(gi[q]);
      if constexpr (NP == 1) {
        // lane 63 gains lane 47 (row 2's total), then lane 31 (by then rows
        // 0 and 1's total); rows 0 and 1 may pick up other values, which no
        // one reads
#pragma unroll
        for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x142, 0xf>(gi[q]);   // row_bcast:15
#pragma unroll
        for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x143, 0xf>(gi[q]);   // row_bcast:31
        if (lane == 63)
#pragma unroll
          for (int q = 0; q < D; ++q) s_row[w][r][0][q] = gi[q];
      } else {
        if ((lane & 15) == 15)
#pragma unroll
          for (int q = 0; q < D; ++q) s_row[w][r][lane >> 4][q] = gi[q];
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * D; e += NL) {
    const int r = e / D, q = e % D;
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww)
#pragma unroll
      for (int k = 0; k < NP; ++k) s += (double)s_row[ww][r][k][q];
    a.prow[(tile * kTR + r) * D + q] = s;
  }
  double tot[4] = {0.0, 0.0, (double)cnt, (double)bad};
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int q = 0; q < D; ++q) a.pcol[(tile * kTC + jl[c]) * D + q] = (double)g[c][q];
    tot[0] += (double)tsum[c];
    tot[1] += (double)dsum[c];
  }
  block_sum_n(tot, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.ptile[tile * 4 + k] = tot[k];
}

// One workgroup: the tile totals in tile order, the -M/2 log sigma^2 and
// -M/sigma terms, and the data checks (invalid deltas and non-finite x, both
// counted by the tiles).
__global__ void __launch_bounds__(kFinalThreads) k_bmds_final(Args a) {
  __shared__ double sh[4 * kFinalThreads];
  double v[4] = {0, 0, 0, 0};   // the four tile totals
  for (int64_t t = threadIdx.x; t < a.ntiles; t += kFinalThreads)
    for (int k = 0; k < 4; ++k) v[k] += a.ptile[t * 4 + k];
  block_sum_n(v, sh);
  if (threadIdx.x == 0) {
    const double M = v[2];
    const bool bad = v[3] > 0.0;
    a.out4[0] = bad ? NAN : -0.5 * M * log(a.sigma * a.sigma) + v[0];
    a.out4[1] = bad ? NAN : -M * a.inv_sigma + v[1];
    a.out4[2] = M;
    a.out4[3] = bad ? (double)HAWKES_EDATA : 0.0;
  }
}

// Per event: its row partials over the chunks of its band, then its column
// partials over the bands that reach its chunk.  Four lanes share an event
// (each takes every fourth chunk and band, in order; two butterfly steps
// combine the four sums in a fixed order, the same on every lane), so the
// first events, whose columns collect a partial from nearly every band, do not
// keep one long chain of loads each.
constexpr int kRedEvents = 64;   // events per workgroup of k_bmds_reduce (256 lanes)

template <int D>
__global__ void __launch_bounds__(4 * kRedEvents) k_bmds_reduce(Args a) {
  const int n = blockIdx.x * kRedEvents + (threadIdx.x >> 2);
  const int sub = threadIdx.x & 3;
  const bool live = n < a.n;
  const bool bad = a.out4[3] != 0.0;
  double g[D];
#pragma unroll
  for (int q = 0; q < D; ++q) g[q] = 0.0;
  if (live && !bad) {
    const int I = n / kTR, r = n % kTR;
    const int64_t o = band_offset(I);
    for (int J = sub; J <= I / 4; J += 4)
#pragma unroll
      for (int q = 0; q < D; ++q) g[q] += a.prow[((o + J) * kTR + r) * D + q];
    const int J = n / kTC, c = n % kTC;
    for (int Ib = 4 * J + sub; Ib < a.nb; Ib += 4)
#pragma unroll
      for (int q = 0; q < D; ++q) g[q] += a.pcol[((band_offset(Ib) + J) * kTC + c) * D + q];
  }
  // the four lanes of an event are adjacent lanes of one wave, all present
#pragma unroll
  for (int q = 0; q < D; ++q) {
    g[q] += __shfl_xor(g[q], 1);
    g[q] += __shfl_xor(g[q], 2);
  }
  if (!live || sub != 0) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const int64_t e = (int64_t)n * D + q;
    a.grad_x[e] = bad ? NAN : (a.accumulate ? a.grad_x[e] + g[q] : g[q]);
  }
}

struct Pieces {
  size_t prow, pcol, ptile, total;
};
static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
static Pieces pieces(int64_t n, int d, int64_t& ntiles, int& nb) {
  nb = (int)((n + kTR - 1) / kTR);
  ntiles = band_offset(nb);
  Pieces p;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  p.prow = take(sizeof(double) * (size_t)ntiles * kTR * d);
  p.pcol = take(sizeof(double) * (size_t)ntiles * kTC * d);
  p.ptile = take(sizeof(double) * (size_t)ntiles * 4);
  p.total = o;
  return p;
}

template <int D>
static void launch(const Args& a, int prec, hipStream_t s, int phase) {
  if (phase != 2) {
    // wide lanes need enough tiles to fill the chip with fewer, longer waves
    const bool wide = a.ntiles >= kWideTiles;
    const unsigned nt = (unsigned)a.ntiles;
    if (prec == HAWKES_MIXED) {
      if (wide) k_bmds_tiles<D, true, kColsMixed><<<nt, TileShape<kColsMixed>::kLanes, 0, s>>>(a);
      else k_bmds_tiles<D, true, 1><<<nt, TileShape<1>::kLanes, 0, s>>>(a);
    } else {
      if (wide) k_bmds_tiles<D, false, kColsFp64><<<nt, TileShape<kColsFp64>::kLanes, 0, s>>>(a);
      else k_bmds_tiles<D, false, 1><<<nt, TileShape<1>::kLanes, 0, s>>>(a);
    }
    k_bmds_final<<<1, kFinalThreads, 0, s>>>(a);
  }
  if (phase != 1 && a.grad_x)
    k_bmds_reduce<D><<<(a.n + kRedEvents - 1) / kRedEvents, 4 * kRedEvents, 0, s>>>(a);
}

}  // namespace bmds

int bmds_enqueue(const double* x, const double* delta, int64_t n, int d, double sigma, int prec, void* ws,
                 size_t ws_bytes, hipStream_t s, double* out4, double* grad_x, bool accumulate, int phase) {
  using namespace bmds;
  if (!x || !delta || !ws || !out4) return HAWKES_EINVAL;
  if (prec != HAWKES_FP64 && prec != HAWKES_MIXED) return HAWKES_EINVAL;
  const size_t need = hawkes_bmds_workspace_bytes(n, d);
  if (need == 0 || ws_bytes < need) return HAWKES_EINVAL;
  if (!std::isfinite(sigma) || !(sigma > 0.0)) return HAWKES_EPARAM;
  Args a;
  const Pieces pc = pieces(n, d, a.ntiles, a.nb);
  char* w = static_cast<char*>(ws);
  a.x = x;
  a.delta = delta;
  a.n = (int)n;
  a.sigma = sigma;
  a.inv_sigma = 1.0 / sigma;
  a.inv_s2 = 1.0 / (sigma * sigma);
  a.prow = reinterpret_cast<double*>(w + pc.prow);
  a.pcol = reinterpret_cast<double*>(w + pc.pcol);
  a.ptile = reinterpret_cast<double*>(w + pc.ptile);
  a.out4 = out4;
  a.grad_x = grad_x;
  a.accumulate = accumulate ? 1 : 0;
  (void)hipGetLastError();
  switch (d) {
    case 1: launch<1>(a, prec, s, phase); break;
    case 2: launch<2>(a, prec, s, phase); break;
    case 3: launch<3>(a, prec, s, phase); break;
    case 4: launch<4>(a, prec, s, phase); break;
    case 5: launch<5>(a, prec, s, phase); break;
    case 6: launch<6>(a, prec, s, phase); break;
    case 7: launch<7>(a, prec, s, phase); break;
    case 8: launch<8>(a, prec, s, phase); break;
  }
  return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // namespace hawkes

extern "C" {

size_t hawkes_bmds_workspace_bytes(int64_t n, int d) {
  if (n < 2 || n > (int64_t(1) << 20) || d < 1 || d > hawkes::kMaxD) return 0;
  int64_t ntiles;
  int nb;
  return hawkes::bmds::pieces(n, d, ntiles, nb).total;
}

int hawkes_bmds(const double* x, const double* delta, int64_t n, int d, double sigma, int prec, void* ws,
                size_t ws_bytes, void* stream, double* out4, double* grad_x) {
  return hawkes::bmds_enqueue(x, delta, n, d, sigma, prec, ws, ws_bytes, static_cast<hipStream_t>(stream), out4,
                              grad_x, false);
}

}  // extern "C"
