// gfx950 kernels of the Hawkes log-likelihood + gradient hot path.
//
// Notation (Sec. 2.1 of arXiv 2010.02994): for the ordered pair (i, j) with
// j earlier in time, r2 = |x_i - x_j|^2 and dt = t_i - t_j >= 0.
//   background term (symmetric)   e_bg = exp(-r2/(2 tau_x^2) - dt^2/(2 tau_t^2)),  dt != 0
//   excitation term (j -> i)      e_se = exp(-omega dt - r2/(2 h^2)),              dt > 0
// The weighted pair terms are mu_ij = c_bg e_bg and xi_ij = c_se e_se.
//
// Pass 1 accumulates, per event, the six unweighted sums
//   K = sum e_bg, R = sum e_bg r2, U = sum e_bg dt^2, J = sum e_se, V = sum e_se r2, W = sum e_se dt
// (K, R, U receive the pair from both endpoints; J, V, W only at the later one).
// Pass 2 accumulates the location gradient of App. A, scattering each
// unordered pair's coefficient into both endpoints.
//
// Mixed precision: coordinates are float32 offsets from the data center, the
// exponent is formed in base 2 with a constant shift S (terms carry a factor
// 2^S), exp is v_exp_f32, and per-tile float32 partials fold into float64.
// Rows whose rate sits below the shifted window are recomputed in float64 by
// the fix-up kernels (k_fix1, k_fix2), so no event loses range.
#pragma once
#include <type_traits>

#include "hawkes_common.hpp"

namespace hawkes {

template <int D, bool MIX> struct Traits;
template <int D> struct Traits<D, true> {
  using Real = float;
  using ColT = double;   // partial sums stored outside a wave
  static constexpr int RW = ((D + 2 + 3) / 4) * 4;  // record words: coords, t, aux, pad
  struct alignas(16) Rec { float v[RW]; };
};
template <int D> struct Traits<D, false> {
  using Real = double;
  using ColT = double;
  static constexpr int RW = ((D + 2 + 1) / 2) * 2;
  struct alignas(16) Rec { double v[RW]; };
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ float exp_pair(float z) { return __builtin_amdgcn_exp2f(z); }

#ifndef HK_FP64_UNROLL
#define HK_FP64_UNROLL 4   // column steps per loop trip in the float64 passes
#endif

__device__ __forceinline__ double block_max_256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Pointers taken from a request descriptor are generic; casting them to the
// global address space lets the compiler emit global (not flat) memory
// instructions with scalar base addresses.
#define HK_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ HK_GLOBAL T* glb(T* p) {
  return (HK_GLOBAL T*)p;
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Exact culling: every pair of the band's rows with this column tile lies
// further apart in time than kp.cull_dt, so both pair terms are exactly zero
// in this pass's arithmetic.  Records are time-sorted, so the band's first row
// (t_row0, read once per work item) and the tile's last column (read from the
// tile's records already staged in LDS) bound every pair's time difference.
// Mixed records hold times relative to their own tile's first event; there
// t_row0 is the band's first row relative to the column tile's first event.
template <int D, bool MIX, typename Real, typename Rec>
__device__ __forceinline__ bool tile_culled(Real t_row0, const Rec* tile_recs, int tile, const KParams& kp) {
  if (!kp.cull) return false;
  const int last = min(kp.n - 1, tile * kTile + kTile - 1) - tile * kTile;
  bool c;
  if constexpr (MIX) c = (float)t_row0 - (float)tile_recs[last].v[D] > kp.cull_dtf;
  else c = (double)t_row0 - (double)tile_recs[last].v[D] > kp.cull_dt;
  return uni(c ? 1 : 0) != 0;
}

// Mixed records: an event's time is stored relative to the first event of its
// own column tile of kTile events (so the float32 offsets span one tile's time
// range), and for each column tile the rows' times are re-expressed relative to
// that tile's first event in float64 and rounded once: a pair's time
// difference then carries an absolute rounding error of about 2^-24 times
// (|dt| + the tile's time span), whatever the length of the window.
__device__ __forceinline__ double tile_origin(const double* t, int tile) {
  return glb(t)[(int64_t)tile * kTile];
}

// Which request of a batched launch owns block `blk`: the last request whose
// first block (offsets are non-decreasing) is <= blk.  kind 0: pair-pass
// items, 1: per-event blocks, 2: pack blocks, 3: reduction blocks.
__device__ __forceinline__ int find_req(const ReqDesc* __restrict__ reqs, int nreq, int blk, int kind) {
  if (nreq == 1) return 0;
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int b = kind == 0 ? reqs[mid].blk_items
                : kind == 1 ? reqs[mid].blk_ev
                : kind == 2 ? reqs[mid].blk_pad
                            : reqs[mid].blk_red;
    if (b <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ prepare / pack

// One workgroup of 1024 threads per request: clears the status words, takes
// the float32 origin of the mixed path (spatial midpoint of the first and last
// events, temporal midpoint of the time range; any origin inside the data's
// extent keeps the offsets within the range), t_N, and writes the work-item
// table of the pair passes.  Items run band-major from the last (longest)
// band to the first.  Data validation happens in k_pack.
template <int D>
__device__ __forceinline__ void init_block(const ReqDesc& rq) {
  const auto x = glb(rq.x);
  const auto t = glb(rq.t);
  const int n = rq.kp.n, nb = rq.kp.nb, L = rq.kp.L, b_fine = rq.kp.b_fine;
  __shared__ int s_wsum[1024 / 64];
  const int tid = threadIdx.x;
  if (tid == 0) {
    glb(rq.status)[kStData] = 0;
    glb(rq.status)[kStZero] = 0;
    glb(rq.status)[kStFlagCount] = 0;
    glb(rq.dconst)[0] = t[n - 1];                       // t_N for sorted input
    for (int k = 0; k < D; ++k) glb(rq.dconst)[1 + k] = 0.5 * (x[k] + x[(int64_t)(n - 1) * D + k]);
    glb(rq.dconst)[1 + kMaxD] = 0.5 * (t[0] + t[n - 1]);
  }
  // the bands in rounds of 1024 positions (position p = band nb - 1 - p):
  // every thread counts one band's items, an exclusive scan over the round
  // (wave shuffles, then the earlier waves' totals) gives each band its first
  // item, and the waves then write the round's items, each band's by
  // consecutive lanes
  __shared__ int s_b[1024], s_base[1024], s_ch[1024];
  const int lane = tid & 63, wv = tid >> 6;
  int carry = 0;   // items of the earlier rounds
  for (int r0 = 0; r0 < nb; r0 += 1024) {
    const int pos = r0 + tid;
    int b = 0, ch = 0;
    if (pos < nb) {
      b = nb - 1 - pos;
      const int row_end = min(n, (b + 1) * kBandRows);
      const int nt = (row_end + kTile - 1) / kTile;
      const int Lb = item_tiles(b, b_fine, L);
      ch = (nt + Lb - 1) / Lb;
    }
    int incl = ch;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    if (lane == 63) s_wsum[wv] = incl;
    __syncthreads();
    int base = carry + incl - ch, total = 0;
    for (int w2 = 0; w2 < 1024 / 64; ++w2) {
      if (w2 < wv) base += s_wsum[w2];
      total += s_wsum[w2];
    }
    s_b[tid] = b;
    s_base[tid] = base;
    s_ch[tid] = ch;
    if (pos < nb) {
      glb(rq.band)[b].x = base;
      glb(rq.band)[b].y = ch;
    }
    __syncthreads();
    const int cnt = min(1024, nb - r0);
    for (int p = wv; p < cnt; p += 1024 / 64) {
      const int bp = s_b[p], bs = s_base[p], cp = s_ch[p];
      for (int c = lane; c < cp; c += 64) {
        glb(rq.items)[bs + c].x = bp;
        glb(rq.items)[bs + c].y = c;
      }
    }
    carry += total;
    __syncthreads();   // s_wsum and the round's tables are reused
  }
}

template <int D>
__global__ void __launch_bounds__(1024) k_init(const ReqDesc* __restrict__ reqs) {
  init_block<D>(reqs[blockIdx.x]);
}

// Single-request form: the descriptor arrives as a kernel argument, is
// written to device memory for the later kernels, and drives the set-up.
template <int D>
__global__ void __launch_bounds__(1024) k_init_one(ReqDesc d, ReqDesc* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = d;
  init_block<D>(d);
}

// Packed records and tie groups.  first[i] is the first index with t == t[i]
// (sorted input), so for j < i: t_j < t_i  <=>  j < first[i].  Padded rows get
// first = 0, which makes every pair with them inactive.
template <int D, bool MIX>
__global__ void __launch_bounds__(kEvBlock) k_pack(const ReqDesc* __restrict__ reqs, int nreq) {
  using Tr = Traits<D, MIX>;
  using Real = typename Tr::Real;
  const int r = find_req(reqs, nreq, blockIdx.x, 2);
  const ReqDesc& rq = reqs[r];
  const int i = (blockIdx.x - rq.blk_pad) * kEvBlock + threadIdx.x;
  const int n = rq.kp.n;
  if (i >= rq.kp.n_pad) return;
  const auto t = glb(rq.t);
  typename Tr::Rec rr;
#pragma unroll
  for (int k = 0; k < Tr::RW; ++k) rr.v[k] = Real(0);
  int f = 0;
  if (i < n) {
    const double ti = t[i];
    bool bad = !isfinite(ti) || ti < 0.0 || (i > 0 && !(ti >= t[i - 1]));
#pragma unroll
    for (int k = 0; k < D; ++k) bad = bad || !isfinite(glb(rq.x)[(int64_t)i * D + k]);
    if (bad) atomicOr(rq.status + kStData, 1);   // rare path: generic address is fine
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double v = glb(rq.x)[(int64_t)i * D + k];
      rr.v[k] = MIX ? Real((v - glb(rq.dconst)[1 + k]) * rq.kp.inv_tx) : Real(v);
    }
    // mixed: time relative to the first event of the event's column tile
    rr.v[D] = MIX ? Real((ti - t[(int64_t)(i / kTile) * kTile]) * rq.kp.inv_tt) : Real(ti);
    // first index with time ti: i itself unless the previous event ties
    // (then a lower_bound of ti in t[0..i], a chain of dependent loads that
    // only tied events pay)
    int lo = 0, hi = i;
    if (i == 0 || t[i - 1] < ti) lo = i;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (t[mid] < ti) lo = mid + 1; else hi = mid;
    }
    f = lo;
  }
  {
    const auto dst = glb(static_cast<typename Tr::Rec*>(rq.rec));
#pragma unroll
    for (int q = 0; q < Tr::RW; ++q) dst[i].v[q] = rr.v[q];
  }
  glb(rq.first)[i] = f;
  glb(static_cast<Real*>(rq.ps))[i] = Real(0);
}

// ------------------------------------------------------------ pair passes

// Stage one tile of 64 records into LDS (16-byte chunks).
template <typename Rec>
struct TileStage {
  static constexpr int kChunks = 64 * (int)sizeof(Rec) / 16;
  static constexpr int kPer = (kChunks + kThreads - 1) / kThreads;
  Chunk16 r[kPer];
  template <typename P>
  __device__ __forceinline__ void load(P src, int tile) {
    const HK_GLOBAL Chunk16* s = (const HK_GLOBAL Chunk16*)(src + (int64_t)tile * kTile);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int c = threadIdx.x + k * kThreads;
      if (c < kChunks) { r[k].a = s[c].a; r[k].b = s[c].b; r[k].c = s[c].c; r[k].d = s[c].d; }
    }
  }
  __device__ __forceinline__ void store(Rec* dst) {
    Chunk16* s = reinterpret_cast<Chunk16*>(dst);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int c = threadIdx.x + k * kThreads;
      if (c < kChunks) s[c] = r[k];
    }
  }
};

// Pass 1: rates and the moments the parameter gradient needs.
template <int D, bool MIX>
struct Pass1Rows {
  using Real = typename Traits<D, MIX>::Real;
  static constexpr int R = kRowsPerLane;
  Real x[R][D], t[R];   // mixed: t is relative to the current column tile's first event
  int first[R];
  Real a[R][6];        // per-tile partials (float32 in mixed, the running sums in float64)
  double acc[R][6];    // float64 running sums (mixed path only)
};

template <int D, bool MIX, bool MASK>
__device__ __forceinline__ void pass1_tile(Pass1Rows<D, MIX>& S, const typename Traits<D, MIX>::Rec* __restrict__ cols,
                                           typename Traits<D, MIX>::ColT* __restrict__ acc_w, int tile_base,
                                           const KParams& kp, const double* __restrict__ tab) {
  using Real = typename Traits<D, MIX>::Real;
  constexpr int R = kRowsPerLane;
  const int lane = threadIdx.x & 63;
  // base-2 (mixed) or natural (float64) exponent scales
  static_assert(!MIX, "the float32 passes use the lane-rotation kernels");
  const Real cb = Real(kp.alpha), ct = Real(kp.beta), cg = Real(kp.gamma), cw = Real(kp.omega);
#pragma unroll HK_FP64_UNROLL
  for (int k = 0; k < 64; ++k) {
    const int c = lane ^ k;
    const auto col = cols[c];
    Real cK, cR, cU;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Real r2 = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const Real dx = S.x[r][q] - col.v[q];
        r2 = dx * dx + r2;
      }
      const Real dt = S.t[r] - col.v[D];
      const Real dt2 = dt * dt;
      // exponents as one product plus a fused multiply-add each
      Real eb = exp_tab(-__builtin_fma(cb, r2, ct * dt2), tab);
      Real es = exp_tab(-__builtin_fma(cg, r2, cw * dt), tab);
      if (MASK) {
        const bool act = (tile_base + c) < S.first[r];
        eb = act ? eb : Real(0);
        es = act ? es : Real(0);
      }
      // raw r2, dt^2 and dt moments
      S.a[r][0] += eb;
      S.a[r][1] = eb * r2 + S.a[r][1];
      S.a[r][2] = eb * dt2 + S.a[r][2];
      S.a[r][3] += es;
      S.a[r][4] = es * r2 + S.a[r][4];
      S.a[r][5] = es * dt + S.a[r][5];
      // column contributions summed over this lane's rows
      cK = r == 0 ? eb : cK + eb;
      cR = r == 0 ? eb * r2 : eb * r2 + cR;
      cU = r == 0 ? eb * dt2 : eb * dt2 + cU;
    }
    atomicAdd(&acc_w[0 * 64 + c], cK);
    atomicAdd(&acc_w[1 * 64 + c], cR);
    atomicAdd(&acc_w[2 * 64 + c], cU);
  }
}

template <int D, bool MIX>
__global__ void __launch_bounds__(kThreads) k_pass1(const ReqDesc* __restrict__ reqs, int nreq) {
  using Rec = typename Traits<D, false>::Rec;
  using Real = double;
  using ColT = double;
  constexpr int R = kRowsPerLane;
  constexpr int NQ = 3;
  __shared__ Rec s_rec[2][kTile];
  __shared__ ColT s_acc[2][kWaves][NQ][kTile];
  __shared__ double s_exptab[kExpTab];   // 2^(j/kExpTab) for exp_tab
  fill_exp_table(s_exptab);
  const int rid = find_req(reqs, nreq, blockIdx.x, 0);
  const ReqDesc& rq = reqs[rid];
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const auto rec = glb(static_cast<const Rec*>(rq.rec));
  const auto first = glb(rq.first);
  const auto pcol = glb(static_cast<ColT*>(rq.pcol));
  const int item = blockIdx.x - rq.blk_items;
  const int band = uni(glb(rq.items)[item].x), chunk = uni(glb(rq.items)[item].y);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row_base = band * kBandRows;
  const int row_end = min(kp.n, row_base + kBandRows);
  const int nt_band = (row_end + kTile - 1) / kTile;
  const int Lb = item_tiles(band, kp.b_fine, kp.L);
  const int tile0 = chunk * Lb;
  const int tile1 = min(tile0 + Lb, nt_band);
  const bool partial_band = row_base + kBandRows > kp.n;
  const int first_min = uni(first[row_base]);
  const auto t_row0 = rec[row_base].v[D];   // the band's first row (culling)

  Pass1Rows<D, false> S;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gi = row_base + wave * 64 * R + r * 64 + lane;
    Rec rr;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Rec) / sizeof(rr.v[0])); ++q) rr.v[q] = rec[gi].v[q];
#pragma unroll
    for (int q = 0; q < D; ++q) S.x[r][q] = rr.v[q];
    S.t[r] = rr.v[D];
    S.first[r] = first[gi];
#pragma unroll
    for (int q = 0; q < 6; ++q) { S.a[r][q] = Real(0); S.acc[r][q] = 0.0; }
  }
  {
    ColT* z = &s_acc[0][0][0][0];
    for (int e = threadIdx.x; e < 2 * kWaves * NQ * kTile; e += kThreads) z[e] = ColT(0);
  }
  TileStage<Rec> stage;
  stage.load(rec, tile0);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int buf = (tile - tile0) & 1;
    stage.store(&s_rec[buf][0]);
    __syncthreads();
    if (tile + 1 < tile1) stage.load(rec, tile + 1);
    for (int e = threadIdx.x; tile > tile0 && e < NQ * kTile; e += kThreads) {
      // column sums of the previous tile: fixed-order sum over the waves
      const int q = e >> 6, c = e & 63;
      ColT s = ColT(0);
#pragma unroll
      for (int w = 0; w < kWaves; ++w) { s += s_acc[buf ^ 1][w][q][c]; s_acc[buf ^ 1][w][q][c] = ColT(0); }
      pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile - 1) * kTile + c] = s;
    }
    const bool full = !partial_band && (tile + 1) * kTile <= first_min;
    if (tile_culled<D, MIX>(t_row0, &s_rec[buf][0], tile, kp)) {
      // nothing to add: the tile's column sums stay zero
    } else if (full) {
      pass1_tile<D, MIX, false>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp, s_exptab);
    } else {
      pass1_tile<D, MIX, true>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp, s_exptab);
    }

  }
  __syncthreads();
  for (int e = threadIdx.x; e < NQ * kTile; e += kThreads) {
    const int buf = (tile1 - 1 - tile0) & 1;
    const int q = e >> 6, c = e & 63;
    ColT s = ColT(0);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += s_acc[buf][w][q][c];
    pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile1 - 1) * kTile + c] = s;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = wave * 64 * R + r * 64 + lane;
#pragma unroll
    for (int q = 0; q < 6; ++q) glb(static_cast<double*>(rq.prow))[((int64_t)item * 6 + q) * kBandRows + lr] = S.a[r][q];
  }
}

// Pass 2: location gradient.  For the pair (i later, j earlier)
//   c_ij = mu_ij (1/lambda_i + 1/lambda_j)/tau_x^2 + xi_ij/(lambda_i h^2)
// and d ell/d x_i += c_ij (x_j - x_i), d ell/d x_j += c_ij (x_i - x_j)   (App. A).
// Per event: pb = c_bg 2^-S/(lambda~ tau_x^2) in the record's aux slot (the
// column side), ps = c_se 2^-S/(lambda~ h^2) for the row side; both are 0 for
// rows the fix-up kernels handle.
template <int D, bool MIX>
struct Pass2Rows {
  using Real = typename Traits<D, MIX>::Real;
  static constexpr int R = kRowsPerLane;
  Real x[R][D], t[R], pb[R], ps[R];   // mixed: t is relative to the current column tile's first event
  int first[R];
  Real g[R][D];
  Real mom[2];        // mixed: per-tile sums of w r^2 and w dt^2 (w = background pair weight)
  double momd[2];     // their float64 running sums
  double acc[R][D];
};

template <int D, bool MIX, bool MASK>
__device__ __forceinline__ void pass2_tile(Pass2Rows<D, MIX>& S, const typename Traits<D, MIX>::Rec* __restrict__ cols,
                                           typename Traits<D, MIX>::ColT* __restrict__ acc_w, int tile_base,
                                           const KParams& kp, const double* __restrict__ tab) {
  using Real = typename Traits<D, MIX>::Real;
  constexpr int R = kRowsPerLane;
  const int lane = threadIdx.x & 63;
  static_assert(!MIX, "the float32 passes use the lane-rotation kernels");
  const Real cb = Real(kp.alpha), ct = Real(kp.beta), cg = Real(kp.gamma), cw = Real(kp.omega);
#pragma unroll HK_FP64_UNROLL
  for (int k = 0; k < 64; ++k) {
    const int c = lane ^ k;
    const auto col = cols[c];
    Real cgr[D];
#pragma unroll
    for (int q = 0; q < D; ++q) cgr[q] = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Real dx[D];
      Real r2 = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        dx[q] = S.x[r][q] - col.v[q];
        r2 = dx[q] * dx[q] + r2;
      }
      const Real dt = S.t[r] - col.v[D];
      // exponents as one product plus a fused multiply-add each
      Real eb = exp_tab(-__builtin_fma(cb, r2, ct * (dt * dt)), tab);
      Real es = exp_tab(-__builtin_fma(cg, r2, cw * dt), tab);
      if (MASK) {
        const bool act = (tile_base + c) < S.first[r];
        eb = act ? eb : Real(0);
        es = act ? es : Real(0);
      }
      const Real coef = eb * (S.pb[r] + col.v[D + 1]) + es * S.ps[r];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        S.g[r][q] = -coef * dx[q] + S.g[r][q];
        cgr[q] = coef * dx[q] + cgr[q];
      }
    }
#pragma unroll
    for (int q = 0; q < D; ++q) atomicAdd(&acc_w[q * 64 + c], cgr[q]);
  }
}

template <int D, bool MIX>
__global__ void __launch_bounds__(kThreads) k_pass2(const ReqDesc* __restrict__ reqs, int nreq) {
  using Rec = typename Traits<D, false>::Rec;
  using Real = double;
  using ColT = double;
  constexpr int R = kRowsPerLane;
  constexpr int NQ = D;
  __shared__ Rec s_rec[2][kTile];
  __shared__ ColT s_acc[2][kWaves][NQ][kTile];
  __shared__ double s_exptab[kExpTab];   // 2^(j/kExpTab) for exp_tab
  fill_exp_table(s_exptab);
  const int rid = find_req(reqs, nreq, blockIdx.x, 0);
  const ReqDesc& rq = reqs[rid];
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const auto rec = glb(static_cast<const Rec*>(rq.rec));
  const auto first = glb(rq.first);
  const auto pcol = glb(static_cast<ColT*>(rq.pcol));
  const int item = blockIdx.x - rq.blk_items;
  const int band = uni(glb(rq.items)[item].x), chunk = uni(glb(rq.items)[item].y);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row_base = band * kBandRows;
  const int row_end = min(kp.n, row_base + kBandRows);
  const int nt_band = (row_end + kTile - 1) / kTile;
  const int Lb = item_tiles(band, kp.b_fine, kp.L);
  const int tile0 = chunk * Lb;
  const int tile1 = min(tile0 + Lb, nt_band);
  const bool partial_band = row_base + kBandRows > kp.n;
  const int first_min = uni(first[row_base]);
  const auto t_row0 = rec[row_base].v[D];   // the band's first row (culling)

  Pass2Rows<D, false> S;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gi = row_base + wave * 64 * R + r * 64 + lane;
    Rec rr;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Rec) / sizeof(rr.v[0])); ++q) rr.v[q] = rec[gi].v[q];
#pragma unroll
    for (int q = 0; q < D; ++q) { S.x[r][q] = rr.v[q]; S.g[r][q] = Real(0);  }
    S.t[r] = rr.v[D];
    S.pb[r] = rr.v[D + 1];
    S.ps[r] = glb(static_cast<const Real*>(rq.ps))[gi];
    S.first[r] = first[gi];
  }
  {
    ColT* z = &s_acc[0][0][0][0];
    for (int e = threadIdx.x; e < 2 * kWaves * NQ * kTile; e += kThreads) z[e] = ColT(0);
  }
  TileStage<Rec> stage;
  stage.load(rec, tile0);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int buf = (tile - tile0) & 1;
    stage.store(&s_rec[buf][0]);
    __syncthreads();
    if (tile + 1 < tile1) stage.load(rec, tile + 1);
    for (int e = threadIdx.x; tile > tile0 && e < NQ * kTile; e += kThreads) {
      // column sums of the previous tile: fixed-order sum over the waves
      const int q = e >> 6, c = e & 63;
      ColT s = ColT(0);
#pragma unroll
      for (int w = 0; w < kWaves; ++w) { s += s_acc[buf ^ 1][w][q][c]; s_acc[buf ^ 1][w][q][c] = ColT(0); }
      pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile - 1) * kTile + c] = s;
    }
    const bool full = !partial_band && (tile + 1) * kTile <= first_min;
    if (tile_culled<D, MIX>(t_row0, &s_rec[buf][0], tile, kp)) {
      // nothing to add: the tile's column sums stay zero
    } else if (full) {
      pass2_tile<D, MIX, false>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp, s_exptab);
    } else {
      pass2_tile<D, MIX, true>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp, s_exptab);
    }

  }
  __syncthreads();
  for (int e = threadIdx.x; e < NQ * kTile; e += kThreads) {
    const int buf = (tile1 - 1 - tile0) & 1;
    const int q = e >> 6, c = e & 63;
    ColT s = ColT(0);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += s_acc[buf][w][q][c];
    pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile1 - 1) * kTile + c] = s;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = wave * 64 * R + r * 64 + lane;
#pragma unroll
    for (int q = 0; q < D; ++q) glb(static_cast<double*>(rq.prow))[((int64_t)item * D + q) * kBandRows + lr] = S.g[r][q];
  }
}

// ------------------------------------------------ mixed-precision pair passes
//
// The float32 passes keep the symmetric (column) sums out of LDS atomics:
// at step k of a 64-column tile, lane l pairs its rows with column (l + k) mod 64,
// and the column accumulators rotate one lane per step with a DPP wave_rol:1
// fused into the add (acc <- acc[lane + 1] + contribution), so after step k
// lane l holds the partial sum of column (l + k) mod 64.  The tile's records
// sit in LDS twice in a row, so the column read is lds[lane + k] with a
// constant offset.
//
// Float32 sums are micro-partials of at most 32 terms, folded into float64:
// every kColSteps = 32 / kRowsPerLane steps (16 steps x 2 rows = 32 terms) each lane adds
// its rotating column accumulator, converted to float64, to its column's slot
// of the wave's float64 LDS row with an LDS add (lanes hold distinct columns
// and a wave's LDS operations run in program order, so each slot receives its
// four adds in a fixed order), and restarts it at zero; the row sums are
// folded into their float64 accumulators every kRowFold = 32 steps.
// Everything stored outside the wave is float64.
constexpr int kColSteps = 32 / kRowsPerLane;
constexpr int kRowFold = 32;
static_assert(kColSteps * kRowsPerLane <= 32 && kRowFold <= 32 && kRowFold % kColSteps == 0 && 64 % kRowFold == 0,
              "float32 micro-partials hold at most 32 terms");

__device__ __forceinline__ float rol1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xf, 0xf, false));
}

template <int D, bool MASK, bool RU>
__device__ __forceinline__ void pass1_tile_mixed(Pass1Rows<D, true>& S, const typename Traits<D, true>::Rec* __restrict__ cols,
                                                 double* __restrict__ acc_w, int tile_base, const KParams& kp) {
  constexpr int R = kRowsPerLane;
  const int lane = threadIdx.x & 63;
  const float mA = kp.mA, mB = kp.mB, mG = kp.mG, mW = kp.mW, sh = kp.S;
  const typename Traits<D, true>::Rec* __restrict__ my = cols + lane;
  // The exponents of kRateExpSteps consecutive steps are formed first and
  // their exps issued back to back, so no exp result is consumed by the very
  // next instruction; the steps are then accumulated in order.
  constexpr int KS = kRateExpSteps;
  static_assert(kColSteps % KS == 0, "exp groups must not straddle a flush");
  constexpr int UO = HK_RATE_UNROLL >= kRowFold ? HK_RATE_UNROLL / kRowFold : 1;
  constexpr int UC = HK_RATE_UNROLL >= kRowFold ? kRowFold / kColSteps : 1;
#pragma unroll UO
  for (int k2 = 0; k2 < 64; k2 += kRowFold) {
#pragma unroll UC
  for (int kc = 0; kc < kRowFold; kc += kColSteps) {
    const int k1 = k2 + kc;
    float aK = 0.f, aR = 0.f, aU = 0.f;
#pragma unroll
    for (int kk = 0; kk < kColSteps; kk += KS) {
      const int k0 = k1 + kk;
      float r2v[KS][R], dtv[KS][R], ebv[KS][R], esv[KS][R];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const auto col = my[k0 + s];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float r2 = 0.f;
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const float dx = S.x[r][q] - col.v[q];
            r2 = q == 0 ? dx * dx : dx * dx + r2;
          }
          const float dt = S.t[r] - col.v[D];
          r2v[s][r] = r2;
          dtv[s][r] = dt;
          ebv[s][r] = __builtin_fmaf(-mB, dt * dt, __builtin_fmaf(-mA, r2, sh));
          esv[s][r] = __builtin_fmaf(-mW, dt, __builtin_fmaf(-mG, r2, sh));
        }
      }
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ebv[s][r] = __builtin_amdgcn_exp2f(ebv[s][r]);
          esv[s][r] = __builtin_amdgcn_exp2f(esv[s][r]);
        }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = k0 + s;
        float cK, cR, cU;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float r2 = r2v[s][r], dt = dtv[s][r], dt2 = dt * dt;
          float eb = ebv[s][r], es = esv[s][r];
          if (MASK) {
            const bool act = (tile_base + ((lane + k) & 63)) < S.first[r];
            eb = act ? eb : 0.f;
            es = act ? es : 0.f;
          }
          S.a[r][0] += eb;
          if (RU) {
            S.a[r][1] = eb * r2 + S.a[r][1];
            S.a[r][2] = eb * dt2 + S.a[r][2];
          }
          S.a[r][3] += es;
          S.a[r][4] = es * r2 + S.a[r][4];
          S.a[r][5] = es * dt + S.a[r][5];
          // column contributions summed over this lane's rows (no "+ 0": a
          // signed zero keeps the compiler from folding it)
          cK = r == 0 ? eb : cK + eb;
          if (RU) {
            cR = r == 0 ? eb * r2 : eb * r2 + cR;
            cU = r == 0 ? eb * dt2 : eb * dt2 + cU;
          }
        }
        aK = rol1(aK) + cK;
        if (RU) {
          aR = rol1(aR) + cR;
          aU = rol1(aU) + cU;
        }
      }
    }
    // column flush: this lane now holds column (lane + k1 + kColSteps - 1) mod 64
    const int c = (lane + k1 + kColSteps - 1) & 63;
    atomicAdd(&acc_w[0 * 64 + c], (double)aK);
    if (RU) { atomicAdd(&acc_w[1 * 64 + c], (double)aR); atomicAdd(&acc_w[2 * 64 + c], (double)aU); }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (!RU && (q == 1 || q == 2)) continue;
      S.acc[r][q] += (double)S.a[r][q];
      S.a[r][q] = 0.f;
    }
  }
}

// RU: also accumulate the background moments R = sum e r^2 and U = sum e dt^2
// (six row sums, three column sums).  Without RU (gradient calls) the rate
// pass keeps K, J, V, W (four row sums, one column sum) and the gradient pass
// forms the two moments' contributions to the parameter gradient instead.
template <int D, bool RU>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(rate_waves(D, RU)))) k_pass1_mixed(const ReqDesc* __restrict__ reqs, int nreq) {
  using Rec = typename Traits<D, true>::Rec;
  using Real = float;
  using ColT = double;
  constexpr int R = kRowsPerLane;
  constexpr int NQ = RU ? 3 : 1;   // column sums
  constexpr int QR = RU ? 6 : 4;   // row sums stored per item
  __shared__ Rec s_rec[2][2 * kTile];
  __shared__ double s_trow[R * kThreads];   // the rows' event times
  __shared__ ColT s_acc[2][kWaves][NQ][kTile];
  const int rid = find_req(reqs, nreq, blockIdx.x, 0);
  const ReqDesc& rq = reqs[rid];
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const auto rec = glb(static_cast<const Rec*>(rq.rec));
  const auto first = glb(rq.first);
  const auto pcol = glb(static_cast<ColT*>(rq.pcol));
  const int item = blockIdx.x - rq.blk_items;
  const int band = uni(glb(rq.items)[item].x), chunk = uni(glb(rq.items)[item].y);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row_base = band * kBandRows;
  const int row_end = min(kp.n, row_base + kBandRows);
  const int nt_band = (row_end + kTile - 1) / kTile;
  const int Lb = item_tiles(band, kp.b_fine, kp.L);
  const int tile0 = chunk * Lb;
  const int tile1 = min(tile0 + Lb, nt_band);
  const bool partial_band = row_base + kBandRows > kp.n;
  const int first_min = uni(first[row_base]);
  const double t_row0 = glb(rq.t)[row_base];   // the band's first row (culling)

  Pass1Rows<D, true> S;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gi = row_base + wave * 64 * R + r * 64 + lane;
    Rec rr;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Rec) / sizeof(rr.v[0])); ++q) rr.v[q] = rec[gi].v[q];
#pragma unroll
    for (int q = 0; q < D; ++q) S.x[r][q] = rr.v[q];
    s_trow[r * kThreads + threadIdx.x] = glb(rq.t)[gi < kp.n ? gi : kp.n - 1];   // own slots: no barrier
    S.first[r] = first[gi];
#pragma unroll
    for (int q = 0; q < 6; ++q) { S.a[r][q] = Real(0); S.acc[r][q] = 0.0; }
  }
  TileStage<Rec> stage;
  stage.load(rec, tile0);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int buf = (tile - tile0) & 1;
    stage.store(&s_rec[buf][0]);
    stage.store(&s_rec[buf][kTile]);
    __syncthreads();
    if (tile + 1 < tile1) stage.load(rec, tile + 1);
    for (int e = threadIdx.x; tile > tile0 && e < NQ * kTile; e += kThreads) {
      // column sums of the previous tile: fixed-order sum over the waves
      const int q = e >> 6, c = e & 63;
      ColT s = ColT(0);
#pragma unroll
      for (int w = 0; w < kWaves; ++w) { s += s_acc[buf ^ 1][w][q][c]; }
      pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile - 1) * kTile + c] = s;
    }
    const bool full = !partial_band && (tile + 1) * kTile <= first_min;
    // the wave's float64 column slots start at zero (a culled tile adds
    // exactly zero and leaves them so)
#pragma unroll
    for (int q = 0; q < NQ; ++q) s_acc[buf][wave][q][lane] = 0.0;
    // row times relative to this column tile's first event
    const double t_tile = tile_origin(rq.t, tile);
#pragma unroll
    for (int r = 0; r < R; ++r) S.t[r] = (float)((s_trow[r * kThreads + threadIdx.x] - t_tile) * kp.inv_tt);
    if (tile_culled<D, true>((float)((t_row0 - t_tile) * kp.inv_tt), &s_rec[buf][0], tile, kp)) {
    } else if (full) {
      pass1_tile_mixed<D, false, RU>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp);
    } else {
      pass1_tile_mixed<D, true, RU>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NQ * kTile; e += kThreads) {
    const int buf = (tile1 - 1 - tile0) & 1;
    const int q = e >> 6, c = e & 63;
    ColT s = ColT(0);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += s_acc[buf][w][q][c];
    pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile1 - 1) * kTile + c] = s;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = wave * 64 * R + r * 64 + lane;
#pragma unroll
    for (int q = 0; q < QR; ++q) {
      const int src = RU ? q : (q == 0 ? 0 : q + 2);   // without RU: K, J, V, W
      glb(static_cast<double*>(rq.prow))[((int64_t)item * QR + q) * kBandRows + lr] = S.acc[r][src];
    }
  }
}

template <int D, bool MASK>
__device__ __forceinline__ void pass2_tile_mixed(Pass2Rows<D, true>& S, const typename Traits<D, true>::Rec* __restrict__ cols,
                                                 double* __restrict__ acc_w, int tile_base, const KParams& kp) {
  constexpr int R = kRowsPerLane;
  const int lane = threadIdx.x & 63;
  const float mA = kp.mA, mB = kp.mB, mG = kp.mG, mW = kp.mW, sh = kp.S;
  const typename Traits<D, true>::Rec* __restrict__ my = cols + lane;
  // exponents of kGradExpSteps steps first, exps back to back, then the
  // steps in order (as in the rate pass)
  constexpr int KS = kGradExpSteps;
  static_assert(kColSteps % KS == 0, "exp groups must not straddle a flush");
  constexpr int UO = HK_GRAD_UNROLL >= kRowFold ? HK_GRAD_UNROLL / kRowFold : 1;
  constexpr int UC = HK_GRAD_UNROLL >= kRowFold ? kRowFold / kColSteps : 1;
#pragma unroll UO
  for (int k2 = 0; k2 < 64; k2 += kRowFold) {
#pragma unroll UC
  for (int kc = 0; kc < kRowFold; kc += kColSteps) {
    const int k1 = k2 + kc;
    float ag[D];
#pragma unroll
    for (int q = 0; q < D; ++q) ag[q] = 0.f;
#pragma unroll
    for (int kk = 0; kk < kColSteps; kk += KS) {
      const int k0 = k1 + kk;
      float dx[KS][R][D], r2[KS][R], dt[KS][R], eb[KS][R], es[KS][R], pbj[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const auto col = my[k0 + s];
        pbj[s] = col.v[D + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int q = 0; q < D; ++q) {
            dx[s][r][q] = S.x[r][q] - col.v[q];
            r2[s][r] = q == 0 ? dx[s][r][q] * dx[s][r][q] : dx[s][r][q] * dx[s][r][q] + r2[s][r];
          }
          dt[s][r] = S.t[r] - col.v[D];
          eb[s][r] = __builtin_fmaf(-mB, dt[s][r] * dt[s][r], __builtin_fmaf(-mA, r2[s][r], sh));
          es[s][r] = __builtin_fmaf(-mW, dt[s][r], __builtin_fmaf(-mG, r2[s][r], sh));
        }
      }
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          eb[s][r] = __builtin_amdgcn_exp2f(eb[s][r]);
          es[s][r] = __builtin_amdgcn_exp2f(es[s][r]);
        }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = k0 + s;
        float cgr[D];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float ebr = eb[s][r], esr = es[s][r];
          if (MASK) {
            const bool act = (tile_base + ((lane + k) & 63)) < S.first[r];
            ebr = act ? ebr : 0.f;
            esr = act ? esr : 0.f;
          }
          // background weight of the pair with both endpoints' 1/lambda; its
          // r^2 and dt^2 moments give the rate pass's R and U terms of the
          // tau_x and tau_t gradients
          const float wb = ebr * (S.pb[r] + pbj[s]);
          const float coef = esr * S.ps[r] + wb;
          S.mom[0] = wb * r2[s][r] + S.mom[0];
          S.mom[1] = wb * (dt[s][r] * dt[s][r]) + S.mom[1];
#pragma unroll
          for (int q = 0; q < D; ++q) {
            S.g[r][q] = -coef * dx[s][r][q] + S.g[r][q];
            cgr[q] = r == 0 ? coef * dx[s][r][q] : coef * dx[s][r][q] + cgr[q];
          }
        }
#pragma unroll
        for (int q = 0; q < D; ++q) ag[q] = rol1(ag[q]) + cgr[q];
      }
    }
    // column flush: this lane now holds column (lane + k1 + kColSteps - 1) mod 64
    const int c = (lane + k1 + kColSteps - 1) & 63;
#pragma unroll
    for (int q = 0; q < D; ++q) atomicAdd(&acc_w[q * 64 + c], (double)ag[q]);
    // the moments hold 2 rows x kColSteps terms: fold them at every flush
    S.momd[0] += (double)S.mom[0];
    S.momd[1] += (double)S.mom[1];
    S.mom[0] = S.mom[1] = 0.f;
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < D; ++q) { S.acc[r][q] += (double)S.g[r][q]; S.g[r][q] = 0.f; }
  }
}

template <int D>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(grad_waves(D)))) k_pass2_mixed(const ReqDesc* __restrict__ reqs, int nreq) {
  using Rec = typename Traits<D, true>::Rec;
  using Real = float;
  using ColT = double;
  constexpr int R = kRowsPerLane;
  constexpr int NQ = D;
  __shared__ Rec s_rec[2][2 * kTile];
  __shared__ double s_trow[R * kThreads];   // the rows' event times
  __shared__ ColT s_acc[2][kWaves][NQ][kTile];
  __shared__ double s_red[2 * kThreads];
  const int rid = find_req(reqs, nreq, blockIdx.x, 0);
  const ReqDesc& rq = reqs[rid];
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const auto rec = glb(static_cast<const Rec*>(rq.rec));
  const auto first = glb(rq.first);
  const auto pcol = glb(static_cast<ColT*>(rq.pcol));
  const int item = blockIdx.x - rq.blk_items;
  const int band = uni(glb(rq.items)[item].x), chunk = uni(glb(rq.items)[item].y);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row_base = band * kBandRows;
  const int row_end = min(kp.n, row_base + kBandRows);
  const int nt_band = (row_end + kTile - 1) / kTile;
  const int Lb = item_tiles(band, kp.b_fine, kp.L);
  const int tile0 = chunk * Lb;
  const int tile1 = min(tile0 + Lb, nt_band);
  const bool partial_band = row_base + kBandRows > kp.n;
  const int first_min = uni(first[row_base]);
  const double t_row0 = glb(rq.t)[row_base];   // the band's first row (culling)

  Pass2Rows<D, true> S;
  S.mom[0] = S.mom[1] = 0.f;
  S.momd[0] = S.momd[1] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gi = row_base + wave * 64 * R + r * 64 + lane;
    Rec rr;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(Rec) / sizeof(rr.v[0])); ++q) rr.v[q] = rec[gi].v[q];
#pragma unroll
    for (int q = 0; q < D; ++q) { S.x[r][q] = rr.v[q]; S.g[r][q] = Real(0); S.acc[r][q] = 0.0; }
    s_trow[r * kThreads + threadIdx.x] = glb(rq.t)[gi < kp.n ? gi : kp.n - 1];   // own slots: no barrier
    S.pb[r] = rr.v[D + 1];
    S.ps[r] = glb(static_cast<const Real*>(rq.ps))[gi];
    S.first[r] = first[gi];
  }
  TileStage<Rec> stage;
  stage.load(rec, tile0);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int buf = (tile - tile0) & 1;
    stage.store(&s_rec[buf][0]);
    stage.store(&s_rec[buf][kTile]);
    __syncthreads();
    if (tile + 1 < tile1) stage.load(rec, tile + 1);
    for (int e = threadIdx.x; tile > tile0 && e < NQ * kTile; e += kThreads) {
      // column sums of the previous tile: fixed-order sum over the waves
      const int q = e >> 6, c = e & 63;
      ColT s = ColT(0);
#pragma unroll
      for (int w = 0; w < kWaves; ++w) { s += s_acc[buf ^ 1][w][q][c]; }
      pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile - 1) * kTile + c] = s;
    }
    const bool full = !partial_band && (tile + 1) * kTile <= first_min;
    // the wave's float64 column slots start at zero (a culled tile adds
    // exactly zero and leaves them so)
#pragma unroll
    for (int q = 0; q < NQ; ++q) s_acc[buf][wave][q][lane] = 0.0;
    // row times relative to this column tile's first event
    const double t_tile = tile_origin(rq.t, tile);
#pragma unroll
    for (int r = 0; r < R; ++r) S.t[r] = (float)((s_trow[r * kThreads + threadIdx.x] - t_tile) * kp.inv_tt);
    if (tile_culled<D, true>((float)((t_row0 - t_tile) * kp.inv_tt), &s_rec[buf][0], tile, kp)) {
    } else if (full) {
      pass2_tile_mixed<D, false>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp);
    } else {
      pass2_tile_mixed<D, true>(S, s_rec[buf], &s_acc[buf][wave][0][0], tile * kTile, kp);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NQ * kTile; e += kThreads) {
    const int buf = (tile1 - 1 - tile0) & 1;
    const int q = e >> 6, c = e & 63;
    ColT s = ColT(0);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += s_acc[buf][w][q][c];
    pcol[((int64_t)band * NQ + q) * kp.n_pad + (tile1 - 1) * kTile + c] = s;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int lr = wave * 64 * R + r * 64 + lane;
#pragma unroll
    for (int q = 0; q < D; ++q)
      glb(static_cast<double*>(rq.prow))[((int64_t)item * D + q) * kBandRows + lr] = S.acc[r][q];
  }
  // the item's two moment sums, fixed-order over the workgroup
  double mom[2] = {S.momd[0], S.momd[1]};
  block_sum_n(mom, s_red);
  if (threadIdx.x == 0) {
    glb(rq.mompart)[(int64_t)item * 2 + 0] = mom[0];
    glb(rq.mompart)[(int64_t)item * 2 + 1] = mom[1];
  }
}

// ------------------------------------------------------------ reductions

// Per event: fixed-order sum of the row partials (this band's items) and the
// column partials (bands from this one to the last), conversion to the raw
// sums K, R, U, J, V, W (times exp(sigma)), the recompute flag, and the
// pass-2 factors (1/lambda scaled to the main pass's terms; 0 for flagged rows,
// whose pairs the float64 fix-ups take).  Pass 2 needs nothing later than this
// kernel, so it can run while the fix-ups and the finalize kernels do.
//
// A workgroup takes kRedEv consecutive events (one band, since kRedEv divides
// kBandRows), one per lane, in each of kRedWaves waves: wave w sums the items
// c = w, w + kRedWaves, ... and the bands I = b + w, b + w + kRedWaves, ..., so
// every load instruction reads one contiguous row of kRedEv float64 partials;
// the waves' sums meet in LDS and wave 0 adds them in wave order (a fixed
// order: results do not depend on timing).  Flagged rows of each workgroup are
// staged in index order for k_fix1.
constexpr int kRedThreads = 64 * kRedWaves;
static_assert(kRedEv == 64 && kBandRows % kRedEv == 0, "a reduction workgroup is one wave of events inside one band");

template <int D, bool MIX>
__global__ void __launch_bounds__(kRedThreads) k_reduce1(const ReqDesc* __restrict__ reqs, int nreq) {
  using ColT = double;   // partials are float64 in both precisions
  using Real = typename Traits<D, MIX>::Real;
  using Rec = typename Traits<D, MIX>::Rec;
  __shared__ double s_part[kRedWaves][6][kRedEv];
  const int rid = find_req(reqs, nreq, blockIdx.x, 3);
  const ReqDesc& rq = reqs[rid];
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const int lb = blockIdx.x - rq.blk_red;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = lb * kRedEv;
  const int i = i0 + lane;   // >= n only in the last band's padding (read, never written)
  const int b = i0 / kBandRows, lr = i % kBandRows;
  const IPair bi{glb(rq.band)[b].x, glb(rq.band)[b].y};
  const auto prow = glb(static_cast<const ColT*>(rq.prow));
  const auto pcol = glb(static_cast<const ColT*>(rq.pcol));
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (!MIX || kp.ru1) {
#pragma unroll 2
    for (int c = wave; c < bi.y; c += kRedWaves) {
      const auto p = prow + (int64_t)(bi.x + c) * 6 * kBandRows + lr;
#pragma unroll
      for (int q = 0; q < 6; ++q) s[q] += p[(int64_t)q * kBandRows];
    }
#pragma unroll 2
    for (int I = b + wave; I < kp.nb; I += kRedWaves) {
      const auto p = pcol + (int64_t)I * 3 * kp.n_pad + i;
#pragma unroll
      for (int q = 0; q < 3; ++q) s[q] += p[(int64_t)q * kp.n_pad];
    }
  } else {
    // rate pass without the background moments: rows K, J, V, W, column K
#pragma unroll 2
    for (int c = wave; c < bi.y; c += kRedWaves) {
      const auto p = prow + (int64_t)(bi.x + c) * 4 * kBandRows + lr;
      s[0] += p[0];
#pragma unroll
      for (int q = 1; q < 4; ++q) s[q + 2] += p[(int64_t)q * kBandRows];
    }
#pragma unroll 4
    for (int I = b + wave; I < kp.nb; I += kRedWaves) s[0] += pcol[(int64_t)I * kp.n_pad + i];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) s_part[wave][q][lane] = s[q];
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double v = s_part[0][q][lane];
#pragma unroll
    for (int w = 1; w < kRedWaves; ++w) v += s_part[w][q][lane];
    s[q] = v;
  }
  bool flag = false;
  if (i < kp.n) {
    if (MIX) {   // moments were accumulated in bandwidth units
      s[1] *= kp.tau_x * kp.tau_x;
      s[2] *= kp.tau_t * kp.tau_t;
      s[4] *= kp.tau_x * kp.tau_x;
      s[5] *= kp.tau_t;
    }
    const double lam = kp.cbg * s[0] + kp.cse * s[3];
    flag = !(lam >= kp.cmax * exp2(kp.flag_floor));
#pragma unroll
    for (int q = 0; q < 6; ++q) glb(rq.sums)[(int64_t)i * 6 + q] = s[q];
    glb(rq.sigma)[i] = kp.sigma_main;
    glb(rq.flags)[i] = flag ? 1 : 0;
    // mixed: coordinates are in units of tau_x, so one factor tau_x moves in
    const double il = flag ? 0.0 : 1.0 / lam;
    const double pb = MIX ? kp.cbg * kp.inv_tx * il : kp.cbg * kp.itx2 * il;
    const double ps = MIX ? kp.cse * kp.tau_x * kp.ih2 * il : kp.cse * kp.ih2 * il;
    glb(static_cast<Rec*>(rq.rec))[i].v[D + 1] = (Real)pb;
    glb(static_cast<Real*>(rq.ps))[i] = (Real)ps;
  }
  // stage this workgroup's flagged rows in index order (one wave ballot)
  const unsigned long long m = __ballot(flag);
  if (flag) glb(rq.bstage)[(int64_t)lb * kRedEv + __popcll(m & ((1ull << lane) - 1ull))] = i;
  if (lane == 0) glb(rq.bcount)[lb] = __popcll(m);
}

// Exact float64 recomputation of the six row sums of each flagged row.  The
// partners are split into kFixSeg segments; each (row, segment) task finds the
// segment's largest log pair term m_s, then sums exp(term - m_s) -- no term that
// matters can underflow.  k_final1 merges the segments in a fixed order.
// fixpart[(f * kFixSeg + s) * 8 + q]: q < 6 the unweighted sums times exp(-m_s), q = 6 m_s.
// The ordered list of flagged rows comes from k_reduce1's per-block counts
// and staged rows: every workgroup scans the counts (256 threads, each over a
// chunk of consecutive blocks) and finds its tasks' rows from the scan;
// workgroup 0 of each request also writes the list, each row's list position
// and the count, which the kernels after this one read.
template <int D>
__global__ void __launch_bounds__(256) k_fix1(const ReqDesc* __restrict__ reqs) {
  __shared__ double sh[6 * 256];
  __shared__ int s_scan[256];
  const ReqDesc& rq = reqs[blockIdx.y];
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const int tid = threadIdx.x;
  const int per = (kp.nsblk + 255) / 256;
  const int lo = min(kp.nsblk, tid * per), hi = min(kp.nsblk, lo + per);
  int own = 0;
  for (int b = lo; b < hi; ++b) own += glb(rq.bcount)[b];
  s_scan[tid] = own;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? s_scan[tid - off] : 0;
    __syncthreads();
    s_scan[tid] += v;
    __syncthreads();
  }
  const int cnt = s_scan[255];
  if (blockIdx.x == 0) {
    int pos = s_scan[tid] - own;
    for (int b = lo; b < hi; ++b) {
      const int c = glb(rq.bcount)[b];
      for (int k = 0; k < c; ++k) {
        const int i = glb(rq.bstage)[(int64_t)b * kRedEv + k];
        glb(rq.list)[pos] = i;
        glb(rq.listpos)[i] = pos;
        ++pos;
      }
    }
    if (tid == 0) glb(rq.status)[kStFlagCount] = cnt;
  }
  const auto x = glb(rq.x);
  const auto t = glb(rq.t);
  const int seg = (kp.n + kFixSeg - 1) / kFixSeg;
  for (int task = blockIdx.x; task < cnt * kFixSeg; task += gridDim.x) {
    const int f = task / kFixSeg, sg = task % kFixSeg;
    // row f of the list: the first chunk whose inclusive count exceeds f,
    // then the block inside it
    int c0 = 0, c1 = 255;
    while (c0 < c1) {
      const int mid = (c0 + c1) >> 1;
      if (s_scan[mid] > f) c1 = mid; else c0 = mid + 1;
    }
    int r = f - (c0 > 0 ? s_scan[c0 - 1] : 0);
    int b = c0 * per;
    for (int cb = glb(rq.bcount)[b]; r >= cb; cb = glb(rq.bcount)[b]) { r -= cb; ++b; }
    const int i = glb(rq.bstage)[(int64_t)b * kRedEv + r];
    const int j0 = sg * seg, j1 = min(kp.n, j0 + seg);
    double xi[D];
#pragma unroll
    for (int q = 0; q < D; ++q) xi[q] = x[(int64_t)i * D + q];
    const double ti = t[i];
    double m = -INFINITY;
    for (int j = j0 + threadIdx.x; j < j1; j += 256) {
      if (j == i) continue;
      double r2 = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) { const double dx = xi[q] - x[(int64_t)j * D + q]; r2 += dx * dx; }
      const double dt = ti - t[j];
      if (dt != 0.0) m = fmax(m, kp.log_cbg - kp.alpha * r2 - kp.beta * dt * dt);
      if (dt > 0.0) m = fmax(m, kp.log_cse - kp.omega * dt - kp.gamma * r2);
    }
    m = block_max_256(m, sh);
    const double msub = m > -INFINITY ? m : 0.0;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int j = j0 + threadIdx.x; j < j1; j += 256) {
      if (j == i) continue;
      double r2 = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) { const double dx = xi[q] - x[(int64_t)j * D + q]; r2 += dx * dx; }
      const double dt = ti - t[j];
      if (dt != 0.0) {
        const double e = exp(-kp.alpha * r2 - kp.beta * dt * dt - msub);
        a[0] += e; a[1] += e * r2; a[2] += e * dt * dt;
      }
      if (dt > 0.0) {
        const double e = exp(-kp.omega * dt - kp.gamma * r2 - msub);
        a[3] += e; a[4] += e * r2; a[5] += e * dt;
      }
    }
    block_sum_n(a, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < 6; ++q) glb(rq.fixpart)[((int64_t)f * kFixSeg + sg) * 8 + q] = a[q];
      glb(rq.fixpart)[((int64_t)f * kFixSeg + sg) * 8 + 6] = m;
    }
  }
}

__device__ __forceinline__ double std_normal_cdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }
__device__ __forceinline__ double std_normal_pdf(double z) { return 0.39894228040143267794 * exp(-0.5 * z * z); }

// Per event: lambda, log lambda, compensator, log-likelihood term and the six
// parameter-gradient terms; per-block fixed-order partials.
template <int D, bool MIX>
__global__ void __launch_bounds__(kEvBlock) k_final1(const ReqDesc* __restrict__ reqs, int nreq) {
  __shared__ double sh[8 * kEvBlock];
  const int rid = find_req(reqs, nreq, blockIdx.x, 1);
  const ReqDesc& rq = reqs[rid];
  if (glb(rq.status)[kStData] != 0) return;
  const KParams& kp = rq.kp;
  const int lb = blockIdx.x - rq.blk_ev;
  const int i = lb * kEvBlock + threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < kp.n) {
    double s[6];
    double sg;
    const bool fl = glb(rq.flags)[i] != 0;
    if (fl) {
      // merge the fix-up segments: common scale m = max_s m_s
      const auto fp = glb(rq.fixpart) + (int64_t)glb(rq.listpos)[i] * kFixSeg * 8;
      double m = -INFINITY;
      for (int g = 0; g < kFixSeg; ++g) m = fmax(m, fp[g * 8 + 6]);
      for (int q = 0; q < 6; ++q) s[q] = 0.0;
      if (m > -INFINITY) {
        for (int g = 0; g < kFixSeg; ++g) {
          const double mg = fp[g * 8 + 6];
          if (mg > -INFINITY) {
            const double w = exp(mg - m);
            for (int q = 0; q < 6; ++q) s[q] += fp[g * 8 + q] * w;
          }
        }
        sg = m;
      } else {
        sg = 0.0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) s[q] = glb(rq.sums)[(int64_t)i * 6 + q];
      sg = glb(rq.sigma)[i];
    }
    const double lt = kp.cbg * s[0] + kp.cse * s[3];   // lambda * exp(-sigma)
    const double L = log(lt) + sg;
    const double T = glb(rq.dconst)[0], ti = rq.t[i];
    const double a = (T - ti) / kp.tau_t, b = -ti / kp.tau_t;
    const double cdf_diff = std_normal_cdf(a) - std_normal_cdf(b);
    const double decay = exp(-kp.omega * (T - ti));
    const double omd = -expm1(-kp.omega * (T - ti));
    const double Lam = kp.mu0 * cdf_diff + kp.theta * omd;
    const double dtau = -kp.mu0 / (kp.tau_t * kp.tau_t) * ((T - ti) * std_normal_pdf(a) + ti * std_normal_pdf(b));
    const double il = 1.0 / lt;
    v[0] = L - Lam;
    v[1] = kp.cbg_unit * s[0] * il - cdf_diff;
    v[2] = kp.cbg * (s[1] / (kp.tau_x * kp.tau_x * kp.tau_x) - D * s[0] / kp.tau_x) * il;
    v[3] = kp.cbg * (s[2] / (kp.tau_t * kp.tau_t * kp.tau_t) - s[0] / kp.tau_t) * il - dtau;
    v[4] = kp.cse_unit * s[3] * il - omd;
    v[5] = kp.cse * (s[3] / kp.omega - s[5]) * il - kp.theta * (T - ti) * decay;
    v[6] = kp.cse * (s[4] / (kp.h * kp.h * kp.h) - D * s[3] / kp.h) * il;
    v[7] = lt > 0.0 ? 0.0 : 1.0;
    glb(rq.logl)[i] = L;
    if (rq.terms != nullptr) {
      // background rate per unit mu0, self-excitation rate per unit theta,
      // log lambda, and the probability that the event was triggered by an
      // earlier one (self-excitation share of the rate)
      const auto tp = glb(rq.terms) + (int64_t)i * 4;
      tp[0] = s[0] > 0.0 ? exp(log(kp.cbg_unit * s[0]) + sg) : 0.0;
      tp[1] = s[3] > 0.0 ? exp(log(kp.cse_unit * s[3]) + sg) : 0.0;
      tp[2] = L;
      tp[3] = kp.cse * s[3] * il;
    }
  }
  block_sum_n(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 8; ++q) glb(rq.bpart)[(int64_t)lb * 8 + q] = v[q];
}

// Sum the per-block partials in block order (one workgroup per request);
// out8 = [ell, 6 gradients, status].  Runs as the first blocks of k_fix2.
__device__ __forceinline__ void final2_block(const ReqDesc& rq, double* sh) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int bad = glb(rq.status)[kStData];
  if (bad == 0) {
    for (int b = threadIdx.x; b < rq.kp.nblk; b += 256)
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] += glb(rq.bpart)[(int64_t)b * 8 + q];
  }
  block_sum_n(v, sh);
  if (threadIdx.x == 0) {
    const auto out8 = glb(rq.out8);
    if (bad != 0) {
      for (int q = 0; q < 7; ++q) out8[q] = NAN;
      out8[7] = -3.0;   // HAWKES_EDATA
    } else if (v[7] > 0.0) {
      glb(rq.status)[kStZero] = 1;
      out8[0] = -INFINITY;
      for (int q = 1; q < 7; ++q) out8[q] = NAN;
      out8[7] = -4.0;
    } else {
      for (int q = 0; q < 7; ++q) out8[q] = v[q];
      out8[7] = 0.0;
    }
  }
}

// Location-gradient fix-up for flagged rows j: the j-side coefficient of
// every pair (j, i), c = mu_ij/(lambda_j tau_x^2) + [t_i < t_j] xi_ji/(lambda_j h^2),
// formed as exp(log-term - log lambda_j) in float64.
// Sweep B (one thread per event i): sum over flagged j of c (x_j - x_i).
template <int D>
__device__ __forceinline__ void fix2b_block(const ReqDesc* __restrict__ reqs, int nreq, int blk) {
  const int rid = find_req(reqs, nreq, blk, 1);
  const ReqDesc& rq = reqs[rid];
  const KParams& kp = rq.kp;
  const int i = (blk - rq.blk_ev) * kEvBlock + threadIdx.x;
  if (i >= kp.n || glb(rq.status)[kStData] != 0) return;
  const auto x = glb(rq.x);
  const auto t = glb(rq.t);
  const int cnt = glb(rq.status)[kStFlagCount];
  double g[D], xi[D];
#pragma unroll
  for (int q = 0; q < D; ++q) { g[q] = 0.0; xi[q] = x[(int64_t)i * D + q]; }
  const double ti = t[i];
  for (int f = 0; f < cnt; ++f) {
    const int j = glb(rq.list)[f];
    if (j == i) continue;
    double dx[D], r2 = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) { dx[q] = x[(int64_t)j * D + q] - xi[q]; r2 += dx[q] * dx[q]; }
    const double dt = t[j] - ti;   // > 0 when j is the later event
    const double Lj = glb(rq.logl)[j];
    if (Lj == -INFINITY) continue;   // lambda_j = 0: the call reports a zero rate
    double c = 0.0;
    if (dt != 0.0) c += exp(kp.log_cbg - kp.alpha * r2 - kp.beta * dt * dt - Lj) * kp.itx2;
    if (dt > 0.0) c += exp(kp.log_cse - kp.omega * dt - kp.gamma * r2 - Lj) * kp.ih2;
#pragma unroll
    for (int q = 0; q < D; ++q) g[q] += c * dx[q];
  }
#pragma unroll
  for (int q = 0; q < D; ++q) glb(rq.gfix)[(int64_t)i * D + q] = g[q];
}

// Sweep A (tasks = flagged row x partner segment): partial sums over the
// segment's events i of c (x_i - x_j) for flagged row j, merged by k_reduce2.
template <int D>
__device__ __forceinline__ void fix2a_block(const ReqDesc& rq, int bx, int nbx, double* sh) {
  if (uni(glb(rq.status)[kStData]) != 0) return;
  const KParams& kp = rq.kp;
  const auto x = glb(rq.x);
  const auto t = glb(rq.t);
  const int cnt = glb(rq.status)[kStFlagCount];
  const int seg = (kp.n + kFixSeg - 1) / kFixSeg;
  for (int task = bx; task < cnt * kFixSeg; task += nbx) {
    const int f = task / kFixSeg, sg = task % kFixSeg;
    const int j = glb(rq.list)[f];
    const int i0 = sg * seg, i1 = min(kp.n, i0 + seg);
    double xj[D];
#pragma unroll
    for (int q = 0; q < D; ++q) xj[q] = x[(int64_t)j * D + q];
    const double tj = t[j], Lj = glb(rq.logl)[j];
    if (Lj == -INFINITY) continue;   // lambda_j = 0: the call reports a zero rate
    double g[D];
#pragma unroll
    for (int q = 0; q < D; ++q) g[q] = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
      if (i == j) continue;
      double dx[D], r2 = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) { dx[q] = x[(int64_t)i * D + q] - xj[q]; r2 += dx[q] * dx[q]; }
      const double dt = tj - t[i];
      double c = 0.0;
      if (dt != 0.0) c += exp(kp.log_cbg - kp.alpha * r2 - kp.beta * dt * dt - Lj) * kp.itx2;
      if (dt > 0.0) c += exp(kp.log_cse - kp.omega * dt - kp.gamma * r2 - Lj) * kp.ih2;
#pragma unroll
      for (int q = 0; q < D; ++q) g[q] += c * dx[q];
    }
    block_sum_n(g, sh);
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < D; ++q) glb(rq.fixpart)[((int64_t)f * kFixSeg + sg) * 8 + q] = g[q];
  }
}

// The finalize reduction and both gradient fix-up sweeps in one launch
// (none reads what another writes): blocks [0, nreq) reduce each request's
// finalize partials, the next ev_blocks take sweep B, and kFixGrid blocks
// per request take sweep A.
template <int D>
__global__ void __launch_bounds__(kEvBlock) k_fix2(const ReqDesc* __restrict__ reqs, int nreq, int ev_blocks) {
  static_assert(kEvBlock == 256, "the finalize reduction uses 256 threads");
  __shared__ double sh[8 * kEvBlock];
  int b = blockIdx.x;
  if (b < nreq) {
    final2_block(reqs[b], sh);
    return;
  }
  b -= nreq;
  if (b < ev_blocks) {
    fix2b_block<D>(reqs, nreq, b);
    return;
  }
  b -= ev_blocks;
  fix2a_block<D>(reqs[b / kFixGrid], b % kFixGrid, kFixGrid, sh);
}

// grad_x = row partials + column partials + fix-up terms, in a fixed order
// (workgroups, waves and the LDS meeting as in k_reduce1).
template <int D, bool MIX>
__global__ void __launch_bounds__(kRedThreads) k_reduce2(const ReqDesc* __restrict__ reqs, int nreq) {
  using ColT = double;   // partials are float64 in both precisions
  __shared__ double s_part[kRedWaves][D][kRedEv];
  const int rid = find_req(reqs, nreq, blockIdx.x, 3);
  const ReqDesc& rq = reqs[rid];
  const KParams& kp = rq.kp;
  // the request's first workgroup completes out8 (and its host copy)
  const bool head = (int)blockIdx.x == rq.blk_red;
  if (uni(glb(rq.status)[kStData]) != 0) {
    if (head && rq.out_host && threadIdx.x < 8) rq.out_host[threadIdx.x] = glb(rq.out8)[threadIdx.x];
    return;
  }
  if (MIX && !kp.ru1 && head) {
    // the background moments' terms of d ell/d tau_x and d ell/d tau_t, from
    // the gradient pass's item sums in item order: sum over pairs of
    // w r'^2 = sum_n c_bg R_n / (tau_x^3 lambda_n) and w dt'^2 tau_x / tau_t =
    // sum_n c_bg U_n / (tau_t^3 lambda_n) over the unflagged rows (flagged
    // rows carry their exact R and U from the fix-up instead)
    __shared__ double s_mom[kRedThreads];
    double m0 = 0.0, m1 = 0.0;
    for (int it = threadIdx.x; it < kp.items; it += kRedThreads) {
      m0 += glb(rq.mompart)[(int64_t)it * 2 + 0];
      m1 += glb(rq.mompart)[(int64_t)it * 2 + 1];
    }
    s_mom[threadIdx.x] = m0;
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) s_mom[threadIdx.x] += s_mom[threadIdx.x + h];
      __syncthreads();
    }
    m0 = s_mom[0];
    __syncthreads();
    s_mom[threadIdx.x] = m1;
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) s_mom[threadIdx.x] += s_mom[threadIdx.x + h];
      __syncthreads();
    }
    m1 = s_mom[0];
    if (threadIdx.x == 0 && glb(rq.out8)[7] == 0.0) {
      glb(rq.out8)[2] += m0;
      glb(rq.out8)[3] += m1 * kp.tau_x / kp.tau_t;
    }
  }
  if (head && rq.out_host && threadIdx.x == 0)   // the thread that added the moment terms
#pragma unroll
    for (int q = 0; q < 8; ++q) rq.out_host[q] = glb(rq.out8)[q];
  if (rq.grad_x == nullptr) return;
  const auto grad_x = glb(rq.grad_x);
  const int lb = blockIdx.x - rq.blk_red;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = lb * kRedEv;
  const int i = i0 + lane;   // >= n only in the last band's padding (read, never written)
  if (uni(glb(rq.status)[kStZero]) != 0) {
    if (wave == 0 && i < kp.n)
#pragma unroll
      for (int q = 0; q < D; ++q) grad_x[(int64_t)i * D + q] = NAN;
    return;
  }
  const int b = i0 / kBandRows, lr = i % kBandRows;
  const IPair bi{glb(rq.band)[b].x, glb(rq.band)[b].y};
  const auto prow = glb(static_cast<const ColT*>(rq.prow));
  const auto pcol = glb(static_cast<const ColT*>(rq.pcol));
  double s[D];
#pragma unroll
  for (int q = 0; q < D; ++q) s[q] = 0.0;
#pragma unroll 2
  for (int c = wave; c < bi.y; c += kRedWaves) {
    const auto p = prow + (int64_t)(bi.x + c) * D * kBandRows + lr;
#pragma unroll
    for (int q = 0; q < D; ++q) s[q] += p[(int64_t)q * kBandRows];
  }
#pragma unroll 2
  for (int I = b + wave; I < kp.nb; I += kRedWaves) {
    const auto p = pcol + (int64_t)I * D * kp.n_pad + i;
#pragma unroll
    for (int q = 0; q < D; ++q) s[q] += p[(int64_t)q * kp.n_pad];
  }
#pragma unroll
  for (int q = 0; q < D; ++q) s_part[wave][q][lane] = s[q];
  __syncthreads();
  if (wave != 0 || i >= kp.n) return;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    double v = s_part[0][q][lane];
#pragma unroll
    for (int w = 1; w < kRedWaves; ++w) v += s_part[w][q][lane];
    s[q] = v + glb(rq.gfix)[(int64_t)i * D + q];
  }
  if (glb(rq.flags)[i] != 0) {
    const auto fp = glb(rq.fixpart) + (int64_t)glb(rq.listpos)[i] * kFixSeg * 8;
    for (int g = 0; g < kFixSeg; ++g)
#pragma unroll
      for (int q = 0; q < D; ++q) s[q] += fp[g * 8 + q];
  }
#pragma unroll
  for (int q = 0; q < D; ++q) grad_x[(int64_t)i * D + q] = s[q];
}


}  // namespace hawkes
