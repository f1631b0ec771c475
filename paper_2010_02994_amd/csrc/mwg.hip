// libhawkes: Metropolis-within-Gibbs moves of event locations and reweighted
// log-likelihoods, both O(N) given cached per-event terms (arXiv 2010.02994,
// Sec. 3: block-wise Metropolis updates of individual location variables;
// rates and compensator of Sec. 2.1).
//
// Cached state, n x 4 float64 per event (written by hawkes_event_terms):
//   a_i  background rate at event i per unit mu0   (sum over j of the background pair term)
//   b_i  self-excitation rate per unit theta        (sum over earlier j)
//   L_i  log lambda_i, lambda_i = mu0 a_i + theta b_i
//   p_i  theta b_i / lambda_i
// Moving the locations of a block of events changes row i's rate only through
// its pairs with the moved events, so Delta ell = sum_i log(lambda_i'/lambda_i)
// costs O(N * block) plus one full O(N) row per moved event.  The compensator
// does not depend on locations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/hawkes.h"
#include "hawkes_common.hpp"
#include "hawkes_internal.hpp"

namespace hawkes {
namespace mwg {

constexpr int kBlock = 256;
constexpr double kGuard = 0x1p-16; // incremental update kept only above this share of its terms
constexpr int kSeg = 32;          // partner segments per exactly recomputed row (workspace per event)
constexpr int kMaxSeg = 512;      // at most, when few rows are listed
constexpr int kExactGrid = 512;   // workgroups of the exact-row kernel (grid-stride over tasks)
constexpr int kListThreads = 1024;

struct Model {
  double mu0, theta;
  double cbg_unit, cse_unit;  // pair weights per unit mu0 / theta
  double alpha, beta, gamma;  // 1/(2 tau_x^2), 1/(2 tau_t^2), 1/(2 h^2)
  double omega;
};

struct Step {
  Model m;
  double* x;            // n x D, moved rows overwritten on accept
  const double* t;
  int n, nmove, nrb;    // events, moved events, row blocks
  double* terms;        // n x 4 cached state
  const int64_t* idx;   // nmove moved events, strictly increasing
  const double* xnew;   // nmove x D proposed locations
  const double* thresh; // accept iff Delta ell > *thresh
  double* out3;         // [Delta ell, accepted, status]
  // workspace
  double* new_a;        // n each
  double* new_b;
  double* dlog;         // incremental rows: log-rate change; listed rows: old log-rate
  int* flag;            // 0 incremental, 1 recompute exactly, 2 moved
  double* bpart;        // nrb: per row block, sum of dlog over its incremental rows
  int* bcount;          // nrb: rows of the block needing an exact recompute
  int* stage;           // nrb x kBlock: those rows in index order
  int* list;            // n: all of them in index order
  double* part;         // n x kSeg x 2: segment sums (a, b) of the listed rows
  int* state;           // [accepted, list length]
};

// Contributions of event j to row i: background per unit mu0 (excluded at equal
// times) and self-excitation per unit theta (only from strictly earlier j).
template <int D>
__device__ __forceinline__ void pair_ab(const Model& m, const double* xi, double ti, const double* xj, double tj,
                                        double& a, double& b, const double* __restrict__ tab) {
  double r2 = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const double dx = xi[q] - xj[q];
    r2 = fma(dx, dx, r2);
  }
  const double dt = ti - tj;
  a = dt != 0.0 ? m.cbg_unit * exp_tab(-m.alpha * r2 - m.beta * dt * dt, tab) : 0.0;
  b = dt > 0.0 ? m.cse_unit * exp_tab(-m.omega * dt - m.gamma * r2, tab) : 0.0;
}

// Position of event j in the moved list, or -1 (binary search; the list is
// read within its bounds whatever it holds).
__device__ __forceinline__ int find_moved(const int64_t* idx, int nmove, int j) {
  int lo = 0, hi = nmove - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int64_t v = idx[mid];
    if (v == j) return mid;
    if (v < j) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// Sum over the workgroup in a fixed order: a butterfly within each wave (every
// lane ends with its wave's total; each step adds the same two values on both
// lanes of a pair), then the wave totals in wave order.  Every thread calls it
// and gets the same value; its barriers also order earlier LDS writes.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();   // sh may be written again right after
  return r;
}

// Rows not moved: the change of (a_i, b_i) from the moved events' old and new
// places, and its log-rate change, summed per block in a fixed order.  When the
// change cancels most of the rate or of either part of it (the new value is
// below 2^-16 of the terms it was formed from, so its rounding error could
// exceed ~2^-37 of it) the row is listed for an exact recompute instead, so
// float64 cancellation neither decides a move nor corrupts the cached parts.
// Moved rows are listed too.  A workgroup covers kBlock rows with RL adjacent
// lanes per row: each lane takes every RL-th moved event, and butterfly steps
// combine the RL sums in a fixed order (the same on every lane), so a block of
// many moved events is not one long chain per row.  Few moved events take one
// lane per row (smaller workgroups start and finish sooner).
constexpr int kRowLanesMany = 4;
constexpr int kManyMoved = 8;   // moved events from which four lanes per row pay

template <int D, int RL>
__global__ void __launch_bounds__(RL * kBlock) k_mwg_rows(Step s) {
  __shared__ double s_old[kBlock][D];
  __shared__ double s_new[kBlock][D];
  __shared__ double s_t[kBlock];
  __shared__ int s_j[kBlock];
  __shared__ double s_dl[kBlock];
  __shared__ double sh[RL * kBlock];
  __shared__ int s_wcnt[(RL * kBlock) / 64];
  __shared__ double s_exptab[kExpTab];   // 2^(j/kExpTab) for exp_tab (read after the loop's barrier)
  fill_exp_table(s_exptab);
  const int tid = threadIdx.x;
  const int rl = tid / RL, sub = tid % RL;
  const int i = blockIdx.x * kBlock + rl;
  const bool row = i < s.n;
  double xi[D], ti = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) xi[q] = row ? s.x[(int64_t)i * D + q] : 0.0;
  if (row) ti = s.t[i];
  double da = 0.0, db = 0.0, oa = 0.0, ob = 0.0;
  int moved = 0;
  for (int c0 = 0; c0 < s.nmove; c0 += kBlock) {
    const int cn = min(kBlock, s.nmove - c0);
    __syncthreads();
    if (tid < cn) {
      const int64_t j = s.idx[c0 + tid];
      const bool ok = j >= 0 && j < s.n;
      s_j[tid] = ok ? (int)j : -1;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        s_old[tid][q] = ok ? s.x[j * D + q] : 0.0;
        s_new[tid][q] = s.xnew[(int64_t)(c0 + tid) * D + q];
      }
      s_t[tid] = ok ? s.t[j] : 0.0;
    }
    __syncthreads();
    if (row) {
      for (int k = sub; k < cn; k += RL) {
        const int j = s_j[k];
        if (j < 0) continue;
        if (j == i) {
          moved = 1;
          continue;
        }
        double a0, b0, a1, b1;
        pair_ab<D>(s.m, xi, ti, s_old[k], s_t[k], a0, b0, s_exptab);
        pair_ab<D>(s.m, xi, ti, s_new[k], s_t[k], a1, b1, s_exptab);
        da += a1 - a0;
        db += b1 - b0;
        oa += a0;
        ob += b0;
      }
    }
  }
  // the lanes of a row are adjacent lanes of one wave, all present
#pragma unroll
  for (int o = 1; o < RL; o <<= 1) {
    da += __shfl_xor(da, o);
    db += __shfl_xor(db, o);
    oa += __shfl_xor(oa, o);
    ob += __shfl_xor(ob, o);
    moved |= __shfl_xor(moved, o);
  }
  int fl = 0;
  double dl = 0.0;
  if (row) {
    if (moved) {
      fl = 2;
    } else {
      const double a = s.terms[(int64_t)i * 4 + 0], b = s.terms[(int64_t)i * 4 + 1];
      const double na = a + da, nb = b + db;
      const double lam = s.m.mu0 * a + s.m.theta * b;
      const double lam1 = s.m.mu0 * na + s.m.theta * nb;
      const double formed_from = lam + s.m.mu0 * oa + s.m.theta * ob;
      const double fa = a + oa, fb = b + ob;   // magnitudes each part was formed from
      const bool kept = lam1 > kGuard * formed_from && !(fa > 0.0 && !(na > kGuard * fa)) &&
                        !(fb > 0.0 && !(nb > kGuard * fb));
      fl = kept ? 0 : 1;
      if (sub == 0) {
        s.new_a[i] = na;
        s.new_b[i] = nb;
      }
      if (fl == 0) dl = log1p((s.m.mu0 * da + s.m.theta * db) / lam);
    }
    if (sub == 0) {
      s.flag[i] = fl;
      // listed rows: their old log-rate, for the exact change formed later
      s.dlog[i] = fl == 0 ? dl : s.terms[(int64_t)i * 4 + 2];
    }
  }
  // block sum of the rows' log-rate changes over the row order (the first
  // kBlock threads hold the rows, the rest zeros, so the tree is the one of a
  // kBlock-thread sum)
  if (sub == 0) s_dl[rl] = dl;
  __syncthreads();
  const double bs = block_sum(tid < kBlock ? s_dl[tid] : 0.0, sh);
  // stage the rows needing an exact recompute, in index order (one lane per row votes)
  const bool listed = row && sub == 0 && fl != 0;
  const unsigned long long msk = __ballot(listed);
  const int lane = tid & 63, w = tid >> 6;
  if (lane == 0) s_wcnt[w] = __popcll(msk);
  __syncthreads();
  int before = 0, total = 0;
  for (int ww = 0; ww < (RL * kBlock) / 64; ++ww) {
    if (ww < w) before += s_wcnt[ww];
    total += s_wcnt[ww];
  }
  if (listed) s.stage[(int64_t)blockIdx.x * kBlock + before + __popcll(msk & ((1ull << lane) - 1ull))] = i;
  if (tid == 0) {
    s.bcount[blockIdx.x] = total;
    s.bpart[blockIdx.x] = bs;
  }
}

// Partner segments per listed row: kSeg, or more when few rows are listed so
// that the tasks still spread over the grid (never more partials than the
// workspace holds: kSeg per event).
__device__ __forceinline__ int segs_for(int cnt, int n) {
  int segs = kSeg;
  while (segs < kMaxSeg && (int64_t)cnt * segs * 2 <= kExactGrid && (int64_t)cnt * segs * 2 <= (int64_t)n * kSeg)
    segs *= 2;
  return segs;
}

// Exact rows, split into (row, partner segment) tasks over a fixed grid: sums
// of the row's pair terms against one segment of partners, every event at its
// proposed place; a moved row sits at its proposed location.  The listed rows
// in index order come from k_mwg_rows' per-block counts and staged rows: every
// workgroup scans the counts (each thread over a chunk of consecutive blocks)
// and finds its tasks' rows from the scan; workgroup 0 also writes the list
// and its length, which the later kernels read.
template <int D>
__global__ void __launch_bounds__(kBlock) k_mwg_exact(Step s) {
  __shared__ double sh[2 * kBlock];
  __shared__ int s_scan[kBlock];
  __shared__ int s_wtot[kBlock / 64];
  __shared__ double s_exptab[kExpTab];   // 2^(j/kExpTab) for exp_tab (read after the scan's barriers)
  fill_exp_table(s_exptab);
  const int tid = threadIdx.x;
  const int per = (s.nrb + kBlock - 1) / kBlock;
  const int lo = min(s.nrb, tid * per), hi = min(s.nrb, lo + per);
  int own = 0;
  for (int b = lo; b < hi; ++b) own += s.bcount[b];
  // inclusive scan of the counts: within each wave by shuffles, then the
  // totals of the earlier waves (two barriers instead of sixteen)
  {
    const int lane = tid & 63, wv = tid >> 6;
    int incl = own;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    if (lane == 63) s_wtot[wv] = incl;
    __syncthreads();
    for (int w2 = 0; w2 < wv; ++w2) incl += s_wtot[w2];
    s_scan[tid] = incl;
    __syncthreads();
  }
  const int cnt = s_scan[kBlock - 1];
  if (blockIdx.x == 0) {
    int pos = s_scan[tid] - own;
    for (int b = lo; b < hi; ++b) {
      const int c = s.bcount[b];
      for (int k = 0; k < c; ++k) s.list[pos++] = s.stage[(int64_t)b * kBlock + k];
    }
    if (tid == 0) s.state[1] = cnt;
  }
  const int segs = segs_for(cnt, s.n);
  const int seg = (s.n + segs - 1) / segs;
  for (int64_t task = blockIdx.x; task < (int64_t)cnt * segs; task += gridDim.x) {
    const int e = (int)(task / segs), sg = (int)(task % segs);
    // listed row e: the first chunk whose inclusive count exceeds e, then the
    // block inside it
    int c0 = 0, c1 = kBlock - 1;
    while (c0 < c1) {
      const int mid = (c0 + c1) >> 1;
      if (s_scan[mid] > e) c1 = mid; else c0 = mid + 1;
    }
    int rr = e - (c0 > 0 ? s_scan[c0 - 1] : 0);
    int rb = c0 * per;
    for (int cb = s.bcount[rb]; rr >= cb; cb = s.bcount[rb]) { rr -= cb; ++rb; }
    const int r = s.stage[(int64_t)rb * kBlock + rr];
    const int rpos = s.flag[r] == 2 ? find_moved(s.idx, s.nmove, r) : -1;
    double xr[D];
#pragma unroll
    for (int q = 0; q < D; ++q) xr[q] = rpos >= 0 ? s.xnew[(int64_t)rpos * D + q] : s.x[(int64_t)r * D + q];
    const double tr = s.t[r];
    const int j0 = sg * seg, j1 = min(s.n, j0 + seg);
    double a = 0.0, b = 0.0;
    for (int j = j0 + threadIdx.x; j < j1; j += kBlock) {
      if (j == r) continue;
      // k_mwg_rows flagged the moved rows with 2: only they search the list
      const int pos = s.flag[j] == 2 ? find_moved(s.idx, s.nmove, j) : -1;
      double xj[D];
#pragma unroll
      for (int q = 0; q < D; ++q) xj[q] = pos >= 0 ? s.xnew[(int64_t)pos * D + q] : s.x[(int64_t)j * D + q];
      double pa, pb;
      pair_ab<D>(s.m, xr, tr, xj, s.t[j], pa, pb, s_exptab);
      a += pa;
      b += pb;
    }
    double ab[2] = {a, b};
    block_sum_n(ab, sh);
    if (threadIdx.x == 0) {
      s.part[((int64_t)e * segs + sg) * 2 + 0] = ab[0];
      s.part[((int64_t)e * segs + sg) * 2 + 1] = ab[1];
    }
  }
}

// Decision and update in one launch.  Every workgroup checks the moved block,
// merges the listed rows' segments and sums the log-rate changes in the same
// fixed order, so all of them reach the same total and the same decision;
// each then updates its own rows on accept, and workgroup 0 reports.  The
// listed rows' old log-rates come from k_mwg_rows' copy (a workgroup updating
// its rows' cached terms must not change what another one reads).  (A
// device-wide fence in every workgroup of the exact kernel, to decide in its
// last workgroup instead, would write back the L2 of each die, which costs
// more than a launch.)
template <int D>
__global__ void __launch_bounds__(kBlock) k_mwg_settle(Step s) {
  __shared__ double sh[kBlock];
  __shared__ double s_na[kBlock], s_nb[kBlock], s_dl[kBlock];
  __shared__ int s_own[kBlock];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int base = blockIdx.x * kBlock;
  s_own[tid] = 0;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = tid; k < s.nmove; k += kBlock) {
    const int64_t j = s.idx[k];
    bool bad = j < 0 || j >= s.n || (k > 0 && s.idx[k - 1] >= j);
#pragma unroll
    for (int q = 0; q < D; ++q) bad = bad || !isfinite(s.xnew[(int64_t)k * D + q]);
    if (bad) atomicOr(&s_bad, 1);
  }
  const int cnt = s.state[1];
  const int segs = segs_for(cnt, s.n);
  // G lanes per listed row (segs / 4, at most a wave): they add strided
  // segments, a butterfly within the group combines them (the same fixed
  // order every time), and the group's first lane keeps the row's log-rate
  // change in its running sum.  Many listed rows (G small) run side by side.
  const int G = min(64, segs / 4);
  const int grp = tid / G, gl = tid % G;
  double acc = 0.0;
  for (int e = grp; e < cnt; e += kBlock / G) {
    double a = 0.0, b = 0.0;
    for (int sg = gl; sg < segs; sg += G) {
      a += s.part[((int64_t)e * segs + sg) * 2 + 0];
      b += s.part[((int64_t)e * segs + sg) * 2 + 1];
    }
    for (int o = G / 2; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      b += __shfl_xor(b, o);
    }
    if (gl == 0) {
      const int r = s.list[e];
      const double dl = log(s.m.mu0 * a + s.m.theta * b) - s.dlog[r];
      acc += dl;
      if (r >= base && r < base + kBlock) {
        s_na[r - base] = a;
        s_nb[r - base] = b;
        s_dl[r - base] = dl;
        s_own[r - base] = 1;
      }
    }
  }
  for (int b = tid; b < s.nrb; b += kBlock) acc += s.bpart[b];
  const double tot = block_sum(acc, sh);   // also orders the LDS writes above
  const bool bad = s_bad != 0;
  const bool accept = !bad && tot > *s.thresh;
  if (blockIdx.x == 0 && tid == 0) {
    s.out3[0] = bad ? NAN : tot;
    s.out3[1] = accept ? 1.0 : 0.0;
    s.out3[2] = bad ? (double)HAWKES_EDATA : 0.0;
    s.state[0] = accept ? 1 : 0;
  }
  if (!accept) return;
  const int i = base + tid;
  if (i < s.nmove) {
    const int64_t j = s.idx[i];
#pragma unroll
    for (int q = 0; q < D; ++q) s.x[j * D + q] = s.xnew[(int64_t)i * D + q];
  }
  if (i >= s.n) return;
  double* tp = s.terms + (int64_t)i * 4;
  const bool own = s_own[tid] != 0;
  const double na = own ? s_na[tid] : s.new_a[i], nb = own ? s_nb[tid] : s.new_b[i];
  if (s.flag[i] == 0 && na == tp[0] && nb == tp[1]) return;
  const double lam1 = s.m.mu0 * na + s.m.theta * nb;
  tp[0] = na;
  tp[1] = nb;
  tp[2] = tp[2] + (own ? s_dl[tid] : s.dlog[i]);
  tp[3] = s.m.theta * nb / lam1;
}

// Log-likelihood and its derivatives in mu0 and theta at new weights, every
// other parameter as when the terms were computed (one workgroup):
//   ell = sum_i log(mu0 a_i + theta b_i) - sum_i (mu0 C_i + theta E_i)
// with C_i the background's time integral and E_i = 1 - exp(-omega (T - t_i)).
__global__ void __launch_bounds__(kListThreads) k_reweight(const double* t, int n, Model m, double tau_t,
                                                             const double* terms, double* out3) {
  __shared__ double sh[3 * kListThreads];
  const double T = t[n - 1];
  double ll = 0.0, gm = 0.0, gt = 0.0;
  for (int i = threadIdx.x; i < n; i += kListThreads) {
    const double a = terms[(int64_t)i * 4 + 0], b = terms[(int64_t)i * 4 + 1];
    const double lam = m.mu0 * a + m.theta * b;
    const double ti = t[i];
    const double za = (T - ti) / tau_t, zb = -ti / tau_t;
    const double C = 0.5 * erfc(-za * 0.70710678118654752440) - 0.5 * erfc(-zb * 0.70710678118654752440);
    const double E = -expm1(-m.omega * (T - ti));
    ll += log(lam) - m.mu0 * C - m.theta * E;
    gm += a / lam - C;
    gt += b / lam - E;
  }
  double v[3] = {ll, gm, gt};
  block_sum_n(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) out3[k] = v[k];
}

static Model make_model(const hawkes_params_t* p, int d) {
  const double two_pi = 6.283185307179586476925286766559;
  Model m;
  m.mu0 = p->mu;
  m.theta = p->theta;
  m.cbg_unit = std::pow(two_pi, -0.5 * (d + 1)) * std::pow(p->h, -d) / p->tau;
  m.cse_unit = p->omega * std::pow(two_pi, -0.5 * d) * std::pow(p->xi, -d);
  m.alpha = 0.5 / (p->h * p->h);
  m.beta = 0.5 / (p->tau * p->tau);
  m.gamma = 0.5 / (p->xi * p->xi);
  m.omega = p->omega;
  return m;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Workspace pieces for n events, in order.
struct Pieces {
  size_t new_a, new_b, dlog, flag, bpart, bcount, stage, list, part, state, total;
};
static Pieces pieces(int64_t n) {
  const size_t nrb = (size_t)((n + kBlock - 1) / kBlock);
  Pieces p;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  p.new_a = take(sizeof(double) * (size_t)n);
  p.new_b = take(sizeof(double) * (size_t)n);
  p.dlog = take(sizeof(double) * (size_t)n);
  p.flag = take(sizeof(int) * (size_t)n);
  p.bpart = take(sizeof(double) * nrb);
  p.bcount = take(sizeof(int) * nrb);
  p.stage = take(sizeof(int) * nrb * kBlock);
  p.list = take(sizeof(int) * (size_t)n);
  p.part = take(sizeof(double) * 2 * kSeg * (size_t)n);
  p.state = take(sizeof(int) * 16);
  p.total = o;
  return p;
}

template <int D>
static void launch(const Step& s, hipStream_t st) {
  if (s.nmove >= kManyMoved)
    k_mwg_rows<D, kRowLanesMany><<<s.nrb, kRowLanesMany * kBlock, 0, st>>>(s);
  else
    k_mwg_rows<D, 1><<<s.nrb, kBlock, 0, st>>>(s);
  k_mwg_exact<D><<<kExactGrid, kBlock, 0, st>>>(s);
  k_mwg_settle<D><<<s.nrb, kBlock, 0, st>>>(s);
}

}  // namespace mwg
}  // namespace hawkes

extern "C" {

size_t hawkes_mwg_workspace_bytes(int64_t n) {
  if (n < 2 || n > (int64_t(1) << 30)) return 0;
  return hawkes::mwg::pieces(n).total;
}

int hawkes_mwg_step(double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, double* terms,
                    const int64_t* idx, const double* x_new, int64_t nmove, const double* log_thresh, void* ws,
                    size_t ws_bytes, void* stream, double* out3) {
  using namespace hawkes::mwg;
  if (!x || !t || !p || !terms || !idx || !x_new || !log_thresh || !ws || !out3) return HAWKES_EINVAL;
  if (d < 1 || d > hawkes::kMaxD || nmove < 1 || nmove > n) return HAWKES_EINVAL;
  const size_t need = hawkes_mwg_workspace_bytes(n);
  if (need == 0 || ws_bytes < need) return HAWKES_EINVAL;
  if (!hawkes::valid_params(p)) return HAWKES_EPARAM;
  const Pieces pc = pieces(n);
  char* w = static_cast<char*>(ws);
  Step s;
  s.m = make_model(p, d);
  s.x = x;
  s.t = t;
  s.n = (int)n;
  s.nmove = (int)nmove;
  s.nrb = (int)((n + kBlock - 1) / kBlock);
  s.terms = terms;
  s.idx = idx;
  s.xnew = x_new;
  s.thresh = log_thresh;
  s.out3 = out3;
  s.new_a = reinterpret_cast<double*>(w + pc.new_a);
  s.new_b = reinterpret_cast<double*>(w + pc.new_b);
  s.dlog = reinterpret_cast<double*>(w + pc.dlog);
  s.flag = reinterpret_cast<int*>(w + pc.flag);
  s.bpart = reinterpret_cast<double*>(w + pc.bpart);
  s.bcount = reinterpret_cast<int*>(w + pc.bcount);
  s.stage = reinterpret_cast<int*>(w + pc.stage);
  s.list = reinterpret_cast<int*>(w + pc.list);
  s.part = reinterpret_cast<double*>(w + pc.part);
  s.state = reinterpret_cast<int*>(w + pc.state);
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  switch (d) {
    case 1: launch<1>(s, st); break;
    case 2: launch<2>(s, st); break;
    case 3: launch<3>(s, st); break;
    case 4: launch<4>(s, st); break;
    case 5: launch<5>(s, st); break;
    case 6: launch<6>(s, st); break;
    case 7: launch<7>(s, st); break;
    case 8: launch<8>(s, st); break;
  }
  return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

int hawkes_loglik_reweight(const double* t, int64_t n, int d, const hawkes_params_t* p, const double* terms,
                           void* stream, double* out3) {
  using namespace hawkes::mwg;
  if (!t || !p || !terms || !out3 || n < 2 || n > (int64_t(1) << 30) || d < 1 || d > hawkes::kMaxD)
    return HAWKES_EINVAL;
  if (!hawkes::valid_params(p)) return HAWKES_EPARAM;
  (void)hipGetLastError();
  k_reweight<<<1, kListThreads, 0, static_cast<hipStream_t>(stream)>>>(t, (int)n, make_model(p, d), p->tau, terms,
                                                                          out3);
  return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // extern "C"
