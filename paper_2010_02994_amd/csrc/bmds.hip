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
// J = 0 .. floor(I / 4) of 256 columns.  The lanes of a wave read consecutive
// delta entries of a row (coalesced row segments), column sums stay in the
// lanes, and a row's sum is formed over each 16-lane row of the wave by DPP row
// shifts, the partials being added in a fixed order.  Two schedules:
//  - few tiles (under 4,096): a workgroup of four waves per tile, one column
//    per lane, rows loaded eight at a time;
//  - many tiles: vertical strips, one wave per chunk and segment of bands,
//    four columns per lane (float64 pairs: two waves of two columns), the
//    rows streamed through a ring of registers refilled row by row, the row's
//    own coordinates read by scalar loads from a packed copy of x, and the
//    partial sums stored in the pair precision.
// Per-tile (or per-segment) partials are reduced per event in a fixed order.
#include <hip/hip_runtime.h>

#include <climits>
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
constexpr int64_t kWideTiles = 4096;   // from this many tiles on: vertical strips (below)

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
  double r2_mid;     // (4 sigma)^2: float64 pairs beyond 4 standard deviations take the tail series
  float r2_mid32;    // (3 sigma)^2: float32 pairs beyond 3 standard deviations take it
  double pdf_c64, pdf_k64;   // phi(z)/sigma = pdf_k64 exp(pdf_c64 r2) (float64 pairs)
  float pdf_c32, pdf_k32;    // phi(z)/sigma = exp2(pdf_c32 r2 + pdf_k32) (float32 pairs)
  int seg_k;       // strips: bands per segment (0: one workgroup per tile)
  int seg_m;      // strips: segment slots per chunk, ceil(nb / seg_k)
  int ncb;        // column chunks met by some band, ceil(nb / 4)
  int64_t nparts; // entries of ptile (tiles, or segments of strips)
  int npack;      // entries of pbad (strips: blocks of the packing kernel)
  void* xs;       // strips: coordinates as R, kXs per event (zero padded)
  double* pbad;   // strips: non-finite coordinates per packing block
  void* prow;     // ntiles x kTR x D partial row sums (double; R for the strips)
  void* pcol;     // ntiles x kTC x D column sums (strips: segments x kTC x D, as R)
  double* ptile;  // nparts x 4: sum of summands, sum of sigma terms, missing pairs, invalid deltas
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

// The upper normal tail q(z) = 1 - Phi(z) as phi(z) S(u) / z, u = 1/z^2,
// where S(u) = z q(z) / phi(z) (the Mills ratio times z) is a polynomial
// fitted here by least squares on Chebyshev nodes to the exact function
// (50-digit values).  Float32 pairs use it beyond z = 3 (u in [0, 1/9]): the
// degree-4 form evaluated in float32 has relative error 4.0e-6, so q
// (<= 1.35e-3) is off by under 5.4e-9, below a float32 pair term's rounding.
// Float64 pairs use it beyond z = 4 (u in [0, 1/16], q <= 3.2e-5): the
// degree-10 form has relative error 2.8e-12.  log Phi = log(1 - q) and
// phi/Phi then follow from short series in q.
__device__ __forceinline__ float mills_s32(float u) {
  float p = 21.182832717895508f;
  p = fmaf(p, u, -9.932043075561523f);
  p = fmaf(p, u, 2.840557336807251f);
  p = fmaf(p, u, -0.9980568289756775f);
  return fmaf(p, u, 0.9999960064888f);
}
__device__ __forceinline__ double mills_s64(double u) {
  double p = 8166022.786010182;
  p = __builtin_fma(p, u, -3394449.479778903);
  p = __builtin_fma(p, u, 669032.215957357);
  p = __builtin_fma(p, u, -87128.92573075247);
  p = __builtin_fma(p, u, 9135.235014291511);
  p = __builtin_fma(p, u, -921.9691254877265);
  p = __builtin_fma(p, u, 104.72455328287757);
  p = __builtin_fma(p, u, -14.998019429918259);
  p = __builtin_fma(p, u, 2.9999925504428386);
  p = __builtin_fma(p, u, -0.9999999889220479);
  return __builtin_fma(p, u, 0.9999999999972508);
}

// 1/sqrt(r2) in float64 for r2 >= 0 (0 for r2 = 0: a coincident pair adds no
// direction): the hardware reciprocal square root refined by two
// Newton-Raphson steps, y <- y + y (1 - r2 y^2) / 2, each of which squares the
// relative error, so the result is within a few units of the last place of
// the correctly rounded value (the library square root and division cost
// about twice the instructions).  Below 2^-1000 (and for infinities) the
// library is used, away from the hardware estimate's denormal range.
__device__ __forceinline__ double rsqrt_f64(double r2) {
  if (__builtin_expect(r2 > 0x1p-1000 && r2 < 0x1p1000, 1)) {
    double y = __builtin_amdgcn_rsq(r2);
    double e = __builtin_fma(-r2 * y, y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-r2 * y, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
  }
  return r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
}

// log Phi(z) and rho/sigma = phi(z)/(sigma Phi(z)) of one observed pair at
// distance dist = r2 rs (rs = 1/dist, 0 for a coincident pair); z = dist/sigma.
// The upper tail is formed directly, so log Phi keeps small tails.  Beyond
// z = 3 (float32) or z = 4 (float64) on every lane of the wave (the usual
// case for well separated points) the tail comes from the Mills-ratio
// polynomial and no erfc, log or reciprocal is evaluated; otherwise from erfc.
template <typename R>
__device__ __forceinline__ void pair_phi(R r2, R dist, R rs, const Args& a, const double* __restrict__ tab, R& lphi,
                                         R& rho_s) {
  if constexpr (std::is_same<R, float>::value) {
    const float sg = (float)a.sigma;
    const float pdf_s = __builtin_amdgcn_exp2f(fmaf(a.pdf_c32, r2, a.pdf_k32));   // phi(z)/sigma
    if (__all(r2 > a.r2_mid32)) {
      const float iz = sg * rs;   // 1/z
      const float q = pdf_s * mills_s32(iz * iz) * (sg * iz);
      lphi = q * fmaf(-0.5f, q, -1.0f);                 // log(1 - q) to O(q^3), q^3/3 < 8.2e-10
      rho_s = fmaf(pdf_s, fmaf(q, q, q), pdf_s);        // pdf_s / (1 - q) to O(q^3)
    } else {
      const float q = 0.5f * erfc_cheb(dist * (float)(a.inv_sigma * 0.70710678118654752440));
      const float phi = 1.0f - q;
      lphi = __builtin_amdgcn_logf(phi) * 0.69314718055994531f;
      rho_s = pdf_s * __builtin_amdgcn_rcpf(phi);
    }
  } else {
    const double pdf_s = a.pdf_k64 * exp_tab(a.pdf_c64 * r2, tab);
    if (__all(r2 > a.r2_mid)) {
      const double iz = a.sigma * rs;
      const double q = pdf_s * mills_s64(iz * iz) * (a.sigma * iz);
      // log(1 - q) and 1/(1 - q) to O(q^4), q <= 3.2e-5
      lphi = q * __builtin_fma(q, __builtin_fma(q, -1.0 / 3.0, -0.5), -1.0);
      rho_s = __builtin_fma(pdf_s * q, __builtin_fma(q, __builtin_fma(q, 1.0, 1.0), 1.0), pdf_s);
    } else {
      const double q = 0.5 * erfc(dist * a.inv_sigma * 0.70710678118654752440);
      lphi = log1p(-q);
      rho_s = pdf_s / (1.0 - q);
    }
  }
}

// Lanes per workgroup and prefetched rows of a tile pass with C columns per
// lane (the library runs it with C = 1 for float64 pairs when tiles are few;
// many tiles, and float32 pairs, take the strips below).
template <int C>
struct TileShape {
  static constexpr int kLanes = kTC / C;   // workgroup size
  static constexpr int kWavesT = kLanes / 64;
  static constexpr int kPre = kPrefetch;   // rows loaded ahead
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
  __shared__ double s_exptab[MIX ? 1 : kExpTab];   // float64 pairs: 2^(j/kExpTab) for exp_tab
  if constexpr (!MIX) fill_exp_table(s_exptab);
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
  R xj[C][D], g[C][D];
  // sums over this lane's pairs of (delta - d)^2, log Phi(z) and rho d/sigma:
  // float32 micro-partials over the pairs of each group of prefetched rows
  // (at most PRE x C terms), folded into float64
  double a_res2 = 0.0, a_lphi = 0.0, a_rz = 0.0;
  int miss = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
      xj[c][q] = jc[c] < a.n ? (R)a.x[(int64_t)jc[c] * D + q] : R(0);
      g[c][q] = R(0);
    }
  }
  const R inv_s2 = (R)a.inv_s2;
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
    R m_res2 = R(0), m_lphi = R(0), m_rz = R(0);
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
      const int r = r0 + u;
      if (r >= rows) break;
      R xi[D], gi[D];
#pragma unroll
      for (int q = 0; q < D; ++q) { xi[q] = s_x[r][q]; gi[q] = R(0); }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double dv = v[u][c];
        if (jc[c] < i0 + r) {
          if (isnan(dv)) {
            miss += 1;
          } else if (dv < 0.0 || isinf(dv)) {
            bad += 1;
          } else {
            R diff[D], r2 = R(0);
#pragma unroll
            for (int q = 0; q < D; ++q) {
              diff[q] = xi[q] - xj[c][q];
              r2 += diff[q] * diff[q];
            }
            R rs, dist;
            if constexpr (MIX) {
              rs = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;   // d = 0 adds no direction
              dist = r2 * rs;
            } else {
              rs = rsqrt_f64(r2);
              dist = r2 * rs;
            }
            R lphi, rho_s;
            pair_phi<R>(r2, dist, rs, a, s_exptab, lphi, rho_s);
            const R res = (R)dv - dist;
            m_res2 = res * res + m_res2;
            m_lphi += lphi;
            m_rz = rho_s * dist + m_rz;
            const R coef = (res * inv_s2 - rho_s) * rs;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              gi[q] = coef * diff[q] + gi[q];
              g[c][q] = -coef * diff[q] + g[c][q];
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
    a_res2 += (double)m_res2;
    a_lphi += (double)m_lphi;
    a_rz += (double)m_rz;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * D; e += NL) {
    const int r = e / D, q = e % D;
    double sum = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww)
#pragma unroll
      for (int k = 0; k < NP; ++k) sum += (double)s_row[ww][r][k][q];
    static_cast<double*>(a.prow)[(tile * kTR + r) * D + q] = sum;
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) static_cast<double*>(a.pcol)[(tile * kTC + jl[c]) * D + q] = (double)g[c][q];
  // the summands -(delta - d)^2/(2 sigma^2) - log Phi(z) and the sigma terms
  // (delta - d)^2/sigma^3 + rho z/sigma of this lane's pairs
  double tot[4] = {-0.5 * a.inv_s2 * a_res2 - a_lphi, a.inv_sigma * (a.inv_s2 * a_res2 + a_rz), (double)miss,
                   (double)bad};
  block_sum_n(tot, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.ptile[tile * 4 + k] = tot[k];
}

// ---- Vertical strips (many tiles) ----
//
// A workgroup takes column chunk J (kTC columns, C per lane over NW waves)
// and a segment of the bands below it: the bands of group m, [m K, m K + K),
// that meet the chunk (band 4J and later).  Its column sums stay in registers
// over up to K x kTR rows and are written once per segment; row sums are
// formed per row as in the tiles above and written per (band, chunk) tile.
// The rows' entries stream through a ring of P rows in registers: the loads
// of row i + P are issued as soon as row i is done, so P rows stay in flight
// while the wave computes, also across band boundaries (the band's row-sum
// barrier waits for LDS only).  The row's own coordinates come by scalar loads
// from a packed copy of x (kXs values per event).
constexpr int kXs = 8;
constexpr int kPackThreads = 256;
#ifndef HK_BMDS_STRIP_K_MIXED
#define HK_BMDS_STRIP_K_MIXED 1
#endif
#ifndef HK_BMDS_STRIP_K_FP64
#define HK_BMDS_STRIP_K_FP64 2
#endif
#ifndef HK_BMDS_RING_MIXED
#define HK_BMDS_RING_MIXED 2
#endif
#ifndef HK_BMDS_RING_FP64
#define HK_BMDS_RING_FP64 4
#endif
#ifndef HK_BMDS_STRIP_COLS_FP64
#define HK_BMDS_STRIP_COLS_FP64 2
#endif
// Bands per segment: 1, 2, 4 or a multiple of 4.  Float32 pairs take one band
// (a tile per workgroup: at N = 20,000 the many short workgroups balance the
// chip better than longer column sums save writes; two bands measured from
// 1 % faster to 9 % slower in two runs, four 8 % slower, eight 35 % slower),
// float64 pairs two.  The ring holds two rows for float32 pairs (four rows:
// 17 more registers, one wave per SIMD fewer, 5 % slower) and four for
// float64 pairs.
constexpr bool valid_strip_k(int k) { return k == 1 || k == 2 || (k >= 4 && k % 4 == 0); }
constexpr int kStripKMixed = HK_BMDS_STRIP_K_MIXED;
constexpr int kStripKFp64 = HK_BMDS_STRIP_K_FP64;
static_assert(valid_strip_k(kStripKMixed) && valid_strip_k(kStripKFp64), "segment length");
constexpr int kRingMixed = HK_BMDS_RING_MIXED;
constexpr int kRingFp64 = HK_BMDS_RING_FP64;
constexpr int kStripColsMixed = 4;                        // one wave per chunk
constexpr int kStripColsFp64 = HK_BMDS_STRIP_COLS_FP64;   // kTC / (64 C) waves per chunk
// Float32 pairs below kWideTiles tiles (the influenza-sized matrices) take the
// strips too, one column per lane over four waves and eight rows in flight:
// the many short workgroups of one band each keep all CUs busy, and the deeper
// ring hides the loads of a chip that holds few waves.  Measured 8 % faster
// than one workgroup per tile at N = 4,733; float64 pairs there measured 7 %
// slower in the strips and keep the tiles.
constexpr int kRingNarrow = 8;

// Segments of chunk J are the band groups m = m0(J) .. M - 1 (M = ceil(nb/K)).
__host__ __device__ inline int seg_m0(int J, int K) { return K <= 4 ? (4 / K) * J : J / (K / 4); }
// Index of chunk J's first segment: the sum over J' < J of (M - m0(J')).
__host__ __device__ inline int64_t seg_base(int J, int K, int M) {
  int64_t before;
  if (K <= 4) {
    before = (int64_t)(4 / K) * ((int64_t)J * (J - 1) / 2);
  } else {
    const int k = K / 4, q = J / k, r = J % k;
    before = (int64_t)k * ((int64_t)q * (q - 1) / 2) + (int64_t)r * q;
  }
  return (int64_t)J * M - before;
}

// s_waitcnt immediate of vmcnt(0) alone (expcnt and lgkmcnt at their maxima).
constexpr int kWaitVm0 = 0x0f70;

// Workgroup barrier that orders LDS only: vector loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// x as R, kXs values per event (zero padded), and per block the count of
// non-finite coordinates.
template <typename R, int D>
__global__ void __launch_bounds__(kPackThreads) k_bmds_pack(Args a) {
  __shared__ double sh[kPackThreads];
  R* xs = static_cast<R*>(a.xs);
  const int i = blockIdx.x * kPackThreads + threadIdx.x;
  double bad[1] = {0.0};
  if (i < a.n) {
#pragma unroll
    for (int q = 0; q < kXs; ++q) {
      const double v = q < D ? a.x[(int64_t)i * D + q] : 0.0;
      if (!isfinite(v)) bad[0] += 1.0;
      xs[(int64_t)i * kXs + q] = (R)v;
    }
  }
  block_sum_n(bad, sh);
  if (threadIdx.x == 0) a.pbad[blockIdx.x] = bad[0];
}

// The pairs of a row with this lane's C columns, those columns below lim
// (the row's index, or INT_MAX for a row below the whole chunk); adds the
// row's sums to gi and the columns' to g.  (Branching around the pairs that
// do not count keeps fewer registers live than computing them with weight 0,
// and the occupancy this keeps is worth more than the branches cost.)
template <int D, bool MIX, int C, typename R>
__device__ __forceinline__ void strip_row(const Args& a, const double* __restrict__ tab, int lim, const R (&xi)[D],
                                          const R (&xj)[C][D], const double (&vr)[C], const int (&jc)[C], R (&g)[C][D],
                                          R (&gi)[D], R& m_res2, R& m_lphi, R& m_rz, int& miss, int& bad) {
  const R inv_s2 = (R)a.inv_s2;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double dv = vr[c];
    if (jc[c] < lim) {
      // an observed dissimilarity is +-0, subnormal or normal and not negative
      if (__builtin_amdgcn_class(dv, 0x1e0)) {
        R diff[D], r2 = R(0);
#pragma unroll
        for (int q = 0; q < D; ++q) {
          diff[q] = xi[q] - xj[c][q];
          r2 += diff[q] * diff[q];
        }
        R rs, dist;
        if constexpr (MIX) {
          rs = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
          dist = r2 * rs;
        } else {
          rs = rsqrt_f64(r2);
          dist = r2 * rs;
        }
        R lphi, rho_s;
        pair_phi<R>(r2, dist, rs, a, tab, lphi, rho_s);
        const R res = (R)dv - dist;
        m_res2 = res * res + m_res2;
        m_lphi += lphi;
        m_rz = rho_s * dist + m_rz;
        const R coef = (res * inv_s2 - rho_s) * rs;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          gi[q] = coef * diff[q] + gi[q];
          g[c][q] = -coef * diff[q] + g[c][q];
        }
      } else if (isnan(dv)) {
        miss += 1;
      } else {
        bad += 1;
      }
    }
  }
}

// Rows i0 .. i0 + nr - 1 of one band against this lane's columns, the ring
// refilled as it goes (rows past the segment re-read its last row).  Unless
// the whole band is below the chunk, only pairs below the diagonal count.
template <int D, bool MIX, int C, int NW, int P, typename R>
__device__ __forceinline__ void strip_band(const Args& a, const double* __restrict__ tab, const R* __restrict__ xs,
                                           const double* __restrict__ delta, int i0, int nr, int rend, bool below,
                                           const int (&jc)[C], const int (&off)[C], const R (&xj)[C][D],
                                           double (&v)[P][C], R (&g)[C][D], R (&s_row)[NW][kTR][4][D],
                                           double& a_res2, double& a_lphi, double& a_rz, int& miss, int& bad) {
  const int n = a.n;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = 0; r < nr; r += P) {
    // float32 micro-partials over the ring's P x C pairs, folded into float64
    R m_res2 = R(0), m_lphi = R(0), m_rz = R(0);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int i = i0 + r + u;
      if (r + u < nr) {
        R xi[D], gi[D];
#pragma unroll
        for (int q = 0; q < D; ++q) {
          xi[q] = xs[(int64_t)i * kXs + q];
          gi[q] = R(0);
        }
        strip_row<D, MIX, C>(a, tab, below ? INT_MAX : i, xi, xj, v[u], jc, g, gi, m_res2, m_lphi, m_rz, miss, bad);
        // 16-lane row sums (row shifts 1, 2, 4, 8: each row's total in its lane 15)
#pragma unroll
        for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x111, 0xf>(gi[q]);
#pragma unroll
        for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x112, 0xf>(gi[q]);
#pragma unroll
        for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x114, 0xf>(gi[q]);
#pragma unroll
        for (int q = 0; q < D; ++q) gi[q] += dpp_step<0x118, 0xf>(gi[q]);
        if ((lane & 15) == 15)
#pragma unroll
          for (int q = 0; q < D; ++q) s_row[w][r + u][lane >> 4][q] = gi[q];
      }
      const int64_t ni = min(i + P, rend - 1);   // refill this ring slot with row i + P
#pragma unroll
      for (int c = 0; c < C; ++c) v[u][c] = delta[ni * n + off[c]];
    }
    a_res2 += (double)m_res2;
    a_lphi += (double)m_lphi;
    a_rz += (double)m_rz;
  }
}

template <int D, bool MIX, int C, int NW, int P>
__global__ void __launch_bounds__(64 * NW) k_bmds_strips(Args a,
                                                         const typename std::conditional<MIX, float, double>::type*
                                                             __restrict__ xs,
                                                         const double* __restrict__ delta) {
  using R = typename std::conditional<MIX, float, double>::type;
  static_assert(64 * C * NW == kTC, "the waves of a workgroup cover one chunk");
  static_assert(kTR % P == 0, "the ring restarts at each band");
  __shared__ R s_row[NW][kTR][4][D];   // 16-lane partial row sums
  __shared__ double sh[4 * 64 * NW];
  __shared__ double s_exptab[MIX ? 1 : kExpTab];
  if constexpr (!MIX) {
    fill_exp_table(s_exptab);
    __syncthreads();
  }
  const int K = a.seg_k, M = a.seg_m, n = a.n;
  const int64_t b = blockIdx.x;
  int lo = 0, hi = a.ncb - 1;   // chunk: largest J with seg_base(J) <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_base(mid, K, M) <= b) lo = mid;
    else hi = mid - 1;
  }
  const int J = lo;
  const int m = seg_m0(J, K) + (int)(b - seg_base(J, K, M));
  const int rbeg = max(4 * J, m * K) * kTR, rend = min(n, min(a.nb, m * K + K) * kTR);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int jc[C], off[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    jc[c] = J * kTC + (w * C + c) * 64 + lane;
    off[c] = min(jc[c], n - 1);
  }
  R xj[C][D], g[C][D];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      xj[c][q] = xs[(int64_t)off[c] * kXs + q];
      g[c][q] = R(0);
    }
  double v[P][C];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int64_t i = min(rbeg + u, n - 1);
#pragma unroll
    for (int c = 0; c < C; ++c) v[u][c] = delta[i * n + off[c]];
  }
  // All of these loads land before the loop (the first row needs the oldest
  // anyway): a load still pending at the loop's entry would make the waits
  // in its body count from the entry's loads on every pass, draining the ring.
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  double a_res2 = 0.0, a_lphi = 0.0, a_rz = 0.0;
  int miss = 0, bad = 0;
  int i0 = rbeg;
  do {   // every segment holds at least one row (rbeg < rend)
    const int nr = min(kTR, rend - i0);
    // bands whose rows are all below every column of the chunk (the bulk)
    // skip the diagonal test; one code path serves both (a second copy of
    // the loop would cost more registers than the test costs issue slots)
    const bool below = J * kTC + kTC <= i0;
    strip_band<D, MIX, C, NW, P>(a, s_exptab, xs, delta, i0, nr, rend, below, jc, off, xj, v, g, s_row, a_res2,
                                 a_lphi, a_rz, miss, bad);
    // the band's row sums over the NW x 4 partials, in a fixed order, stored
    // as R (a float32 row sum over the chunk's columns for float32 pairs; the
    // reduction adds the chunks in float64)
    lds_barrier();
    const int64_t tile = band_offset(i0 / kTR) + J;
    for (int e = threadIdx.x; e < nr * D; e += 64 * NW) {
      const int r = e / D, q = e % D;
      R sum = R(0);
#pragma unroll
      for (int ww = 0; ww < NW; ++ww)
#pragma unroll
        for (int k = 0; k < 4; ++k) sum += s_row[ww][r][k][q];
      static_cast<R*>(a.prow)[(tile * kTR + r) * D + q] = sum;
    }
    lds_barrier();
    i0 += kTR;
  } while (i0 < rend);
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) static_cast<R*>(a.pcol)[(b * kTC + (w * C + c) * 64 + lane) * D + q] = g[c][q];
  double tot[4] = {-0.5 * a.inv_s2 * a_res2 - a_lphi, a.inv_sigma * (a.inv_s2 * a_res2 + a_rz), (double)miss,
                   (double)bad};
  block_sum_n(tot, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.ptile[b * 4 + k] = tot[k];
}

// One workgroup: the tile (or segment) totals in order, the -M/2 log sigma^2
// and -M/sigma terms (M: the pairs of the triangle less the missing ones), and
// the data checks (invalid deltas, and non-finite x counted by the tiles or by
// the packing kernel).
__global__ void __launch_bounds__(kFinalThreads) k_bmds_final(Args a) {
  __shared__ double sh[4 * kFinalThreads];
  double v[4] = {0, 0, 0, 0};   // the four totals
  for (int64_t t = threadIdx.x; t < a.nparts; t += kFinalThreads)
    for (int k = 0; k < 4; ++k) v[k] += a.ptile[t * 4 + k];
  for (int t = threadIdx.x; t < a.npack; t += kFinalThreads) v[3] += a.pbad[t];
  block_sum_n(v, sh);
  if (threadIdx.x == 0) {
    const double M = 0.5 * (double)a.n * (double)(a.n - 1) - v[2];
    const bool bad = v[3] > 0.0;
    a.out4[0] = bad ? NAN : -0.5 * M * log(a.sigma * a.sigma) + v[0];
    a.out4[1] = bad ? NAN : -M * a.inv_sigma + v[1];
    a.out4[2] = M;
    a.out4[3] = bad ? (double)HAWKES_EDATA : 0.0;
  }
}

// Per event: its row partials over the chunks of its band, then its column
// partials over the bands (tiles) or segments (strips) that reach its chunk.
// A workgroup takes 64 consecutive events, which share one band and one chunk,
// one event per lane, so each partial is read by a wave as one contiguous run;
// its kRedWavesB waves take every kRedWavesB-th chunk and band or segment, in
// order, and the waves' sums are added in wave order.
constexpr int kRedWavesB = 16;

template <int D, typename PT>
__global__ void __launch_bounds__(64 * kRedWavesB) k_bmds_reduce(Args a) {
  __shared__ double s_part[kRedWavesB][D][64];
  const PT* prow = static_cast<const PT*>(a.prow);
  const PT* pcol = static_cast<const PT*>(a.pcol);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n0 = blockIdx.x * 64;   // a multiple of kTR: the band's first row
  const int n = n0 + lane;
  const bool live = n < a.n;
  const bool bad = a.out4[3] != 0.0;
  double g[D];
#pragma unroll
  for (int q = 0; q < D; ++q) g[q] = 0.0;
  if (live && !bad) {
    const int I = n0 / kTR;
    const int64_t o = band_offset(I);
    for (int J = w; J <= I / 4; J += kRedWavesB)
#pragma unroll
      for (int q = 0; q < D; ++q) g[q] += (double)prow[((o + J) * kTR + lane) * D + q];
    const int J = n0 / kTC, c = n % kTC;
    if (a.seg_k > 0) {   // strips: the segments of chunk J
      const int64_t base = seg_base(J, a.seg_k, a.seg_m);
      const int cnt = a.seg_m - seg_m0(J, a.seg_k);
      for (int sg = w; sg < cnt; sg += kRedWavesB)
#pragma unroll
        for (int q = 0; q < D; ++q) g[q] += (double)pcol[((base + sg) * kTC + c) * D + q];
    } else {
      for (int Ib = 4 * J + w; Ib < a.nb; Ib += kRedWavesB)
#pragma unroll
        for (int q = 0; q < D; ++q) g[q] += (double)pcol[((band_offset(Ib) + J) * kTC + c) * D + q];
    }
  }
#pragma unroll
  for (int q = 0; q < D; ++q) s_part[w][q][lane] = g[q];
  __syncthreads();
  if (w != 0 || !live) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < kRedWavesB; ++ww) t += s_part[ww][q][lane];
    const int64_t e = (int64_t)n * D + q;
    a.grad_x[e] = bad ? NAN : (a.accumulate ? a.grad_x[e] + t : t);
  }
}

struct Pieces {
  size_t prow, pcol, ptile, xs, pbad, total;
};
static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
// Segments of the strips hold no more than the tiles (each is one or more
// tiles), so the tile-sized buffers serve both paths.
static Pieces pieces(int64_t n, int d, int64_t& ntiles, int& nb) {
  nb = (int)((n + kTR - 1) / kTR);
  ntiles = band_offset(nb);
  Pieces p;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  p.prow = take(sizeof(double) * (size_t)ntiles * kTR * d);
  p.pcol = take(sizeof(double) * (size_t)ntiles * kTC * d);
  p.ptile = take(sizeof(double) * (size_t)ntiles * 4);
  p.xs = take(sizeof(double) * (size_t)n * kXs);
  p.pbad = take(sizeof(double) * (size_t)((n + kPackThreads - 1) / kPackThreads));
  p.total = o;
  return p;
}

template <int D>
static void launch(const Args& a, int prec, hipStream_t s, int phase) {
  if (phase != 2) {
    const unsigned nt = (unsigned)a.ntiles;
    if (a.seg_k > 0) {
      const unsigned nseg = (unsigned)a.nparts;
      if (prec == HAWKES_MIXED && a.ntiles < kWideTiles) {
        k_bmds_pack<float, D><<<a.npack, kPackThreads, 0, s>>>(a);
        k_bmds_strips<D, true, 1, kTC / 64, kRingNarrow><<<nseg, kTC, 0, s>>>(a, static_cast<const float*>(a.xs), a.delta);
      } else if (prec == HAWKES_MIXED) {
        k_bmds_pack<float, D><<<a.npack, kPackThreads, 0, s>>>(a);
        k_bmds_strips<D, true, kStripColsMixed, kTC / (64 * kStripColsMixed), kRingMixed>
            <<<nseg, kTC / kStripColsMixed, 0, s>>>(a, static_cast<const float*>(a.xs), a.delta);
      } else {
        k_bmds_pack<double, D><<<a.npack, kPackThreads, 0, s>>>(a);
        k_bmds_strips<D, false, kStripColsFp64, kTC / (64 * kStripColsFp64), kRingFp64>
            <<<nseg, kTC / kStripColsFp64, 0, s>>>(a, static_cast<const double*>(a.xs), a.delta);
      }
    } else {   // float64 pairs, few tiles
      k_bmds_tiles<D, false, 1><<<nt, TileShape<1>::kLanes, 0, s>>>(a);
    }
    k_bmds_final<<<1, kFinalThreads, 0, s>>>(a);
  }
  if (phase != 1 && a.grad_x) {
    const unsigned nred = (unsigned)((a.n + 63) / 64);
    // the strips store float32 partials for float32 pairs
    if (a.seg_k > 0 && prec == HAWKES_MIXED) k_bmds_reduce<D, float><<<nred, 64 * kRedWavesB, 0, s>>>(a);
    else k_bmds_reduce<D, double><<<nred, 64 * kRedWavesB, 0, s>>>(a);
  }
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
  a.r2_mid = 16.0 * sigma * sigma;
  a.r2_mid32 = (float)(9.0 * sigma * sigma);
  a.pdf_c64 = -0.5 * a.inv_s2;
  a.pdf_k64 = 0.39894228040143267794 * a.inv_sigma;
  a.pdf_c32 = (float)(-0.5 * 1.4426950408889634074 * a.inv_s2);
  a.pdf_k32 = (float)std::log2(0.39894228040143267794 * a.inv_sigma);
  // many tiles, or float32 pairs: vertical strips of one chunk; otherwise
  // (float64 pairs, few tiles) one workgroup per tile, one column per lane
  if (a.ntiles >= kWideTiles || prec == HAWKES_MIXED) {
    const int K = a.ntiles < kWideTiles ? 1 : prec == HAWKES_MIXED ? kStripKMixed : kStripKFp64;
    a.seg_k = K;
    a.seg_m = (a.nb + K - 1) / K;
    a.ncb = (a.nb + 3) / 4;
    a.nparts = seg_base(a.ncb, K, a.seg_m);
    a.npack = (int)((n + kPackThreads - 1) / kPackThreads);
  } else {
    a.seg_k = 0;
    a.seg_m = 0;
    a.ncb = (a.nb + 3) / 4;
    a.nparts = a.ntiles;
    a.npack = 0;
  }
  a.xs = w + pc.xs;
  a.pbad = reinterpret_cast<double*>(w + pc.pbad);
  a.prow = w + pc.prow;
  a.pcol = w + pc.pcol;
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
