// libhawkes: C ABI, workspace layout and launch sequence of the gfx950 Hawkes
// log-likelihood + gradient (arXiv 2010.02994, Sec. 2.1 and App. A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/hawkes.h"
#include "hawkes_common.hpp"
#include "hawkes_internal.hpp"
#include "hawkes_kernels.hpp"

namespace hawkes {

constexpr double kShiftMixed = 120.0;       // base-2 shift of the mixed pass's terms
constexpr double kFloorMixed = -60.0;       // flag when lambda * 2^S < cmax * 2^-60
constexpr double kFloorFp64 = -900.0;       // flag when lambda < cmax * 2^-900
constexpr int kTargetItems = 10240;   // about six rounds of the chip's concurrent pair-pass workgroups
constexpr int kNumStages = 9;

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// The pair passes dispatch bands from the last to the first, so the first
// bands' items run last.  Split into one-tile items, they end the launch with
// short workgroups, so the chip drains in about a tile's time instead of an
// item's.  The split covers the first bands whose tiles total at most
// kTailTiles (about one round of the chip's concurrent workgroups), in
// launches of at least 8 kTailTiles tiles (N >~ 36,000), where that tail is a
// small share of the work; smaller launches keep their measured item sizes.
#ifndef HK_TAIL_TILES
#define HK_TAIL_TILES 1280
#endif
constexpr int64_t kTailTiles = HK_TAIL_TILES;
static int fine_bands(int64_t n, int nb, int L) {
  if (L <= 1) return 0;
  int64_t all = 0;
  for (int b = 0; b < nb; ++b) all += (std::min<int64_t>(n, (int64_t)(b + 1) * kBandRows) + kTile - 1) / kTile;
  if (all < 8 * kTailTiles) return 0;
  int64_t tiles = 0;
  int b = 0;
  for (; b < nb; ++b) {
    const int64_t nt = (std::min<int64_t>(n, (int64_t)(b + 1) * kBandRows) + kTile - 1) / kTile;
    if (tiles + nt > kTailTiles) break;
    tiles += nt;
  }
  return b;
}

static int tiles_per_item(int64_t n) {
  if (const char* e = std::getenv("HAWKES_TILES_PER_ITEM")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  const int nb = (int)((n + kBandRows - 1) / kBandRows);
  int64_t tiles = 0;
  for (int b = 0; b < nb; ++b) tiles += (std::min<int64_t>(n, (int64_t)(b + 1) * kBandRows) + kTile - 1) / kTile;
  // about kTargetItems work items (several rounds of the chip's workgroups,
  // so the last round's idle tail is a small share; at N = 50,000 four tiles
  // per item measured fastest against 3, 5, 6, 8 and 16); at small N, where
  // that would leave one tile per item, up to four tiles per item (fewer row
  // partials for the reductions to read; measured best at N = 4,000-10,000)
  const int64_t fill = (tiles + kTargetItems - 1) / kTargetItems;
  const int64_t small = std::min<int64_t>(4, (tiles + 159) / 160);
  return (int)std::max<int64_t>(1, std::max(fill, small));
}

bool make_layout(int64_t n, int d, int prec, Layout& Lo) {
  const int base = prec & ~HAWKES_CULL;
  if (n < 2 || n > (int64_t(1) << 30) || d < 1 || d > kMaxD || (base != HAWKES_FP64 && base != HAWKES_MIXED))
    return false;
  Lo.n = n;
  Lo.d = d;
  Lo.mixed = base == HAWKES_MIXED;
  Lo.cull = (prec & HAWKES_CULL) != 0;
  Lo.nb = (int)((n + kBandRows - 1) / kBandRows);
  Lo.n_pad = Lo.nb * kBandRows;
  Lo.L = tiles_per_item(n);
  Lo.b_fine = fine_bands(n, Lo.nb, Lo.L);
  Lo.items = 0;
  for (int b = 0; b < Lo.nb; ++b) {
    const int64_t nt = (std::min<int64_t>(n, (int64_t)(b + 1) * kBandRows) + kTile - 1) / kTile;
    const int Lb = item_tiles(b, Lo.b_fine, Lo.L);
    Lo.items += (int)((nt + Lb - 1) / Lb);
  }
  Lo.nblk = (int)((n + kEvBlock - 1) / kEvBlock);
  Lo.nsblk = (int)((n + kRedEv - 1) / kRedEv);
  const size_t real = Lo.mixed ? 4 : 8;
  const int rw = Lo.mixed ? ((d + 2 + 3) / 4) * 4 : ((d + 2 + 1) / 2) * 2;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  Lo.off_desc = take(sizeof(ReqDesc));
  Lo.off_status = take(sizeof(int) * kStSlots);
  Lo.off_dconst = take(sizeof(double) * 16);
  Lo.off_out8 = take(sizeof(double) * 8);
  Lo.off_items = take(sizeof(IPair) * (size_t)Lo.items);
  Lo.off_band = take(sizeof(IPair) * (size_t)Lo.nb);
  Lo.off_rec = take(real * rw * (size_t)Lo.n_pad);
  Lo.off_first = take(sizeof(int) * (size_t)Lo.n_pad);
  Lo.off_ps = take(real * (size_t)Lo.n_pad);
  // row and column partial sums are float64 in both precisions
  Lo.off_prow = take(sizeof(double) * (size_t)Lo.items * std::max(6, d) * kBandRows);
  Lo.off_pcol = take(sizeof(double) * (size_t)Lo.nb * std::max(3, d) * Lo.n_pad);
  Lo.off_sums = take(sizeof(double) * 6 * (size_t)n);
  Lo.off_sigma = take(sizeof(double) * (size_t)n);
  Lo.off_flags = take(sizeof(int) * (size_t)n);
  Lo.off_list = take(sizeof(int) * (size_t)n);
  Lo.off_listpos = take(sizeof(int) * (size_t)n);
  Lo.off_bcount = take(sizeof(int) * (size_t)Lo.nsblk);
  Lo.off_bstage = take(sizeof(int) * (size_t)Lo.nsblk * kRedEv);
  Lo.off_logl = take(sizeof(double) * (size_t)n);
  Lo.off_bpart = take(sizeof(double) * 8 * (size_t)Lo.nblk);
  Lo.off_gfix = take(sizeof(double) * (size_t)d * n);
  Lo.off_fixpart = take(sizeof(double) * 8 * kFixSeg * (size_t)n);
  Lo.off_mompart = take(sizeof(double) * 2 * (size_t)Lo.items);
  Lo.total = o;
  return true;
}

bool valid_params(const hawkes_params_t* p) {
  const double v[6] = {p->mu, p->h, p->tau, p->theta, p->omega, p->xi};
  for (double a : v)
    if (!std::isfinite(a)) return false;
  if (!(p->h > 0) || !(p->tau > 0) || !(p->omega > 0) || !(p->xi > 0)) return false;
  if (p->mu < 0 || p->theta < 0 || (p->mu == 0 && p->theta == 0)) return false;
  return true;
}

// Base-2 shift of the mixed pass.  In bandwidth units every accumulated
// product is bounded: 2^(S-a r2) r2 <= 2^S 2/(e a ln 2) for a = mA or mG, and
// 2^(S-w dt) dt <= 2^S/(e w ln 2); a float32 sum holds at most 32 such terms
// (the micro-partials of the pair passes; everything beyond is float64).  S
// keeps every float32 sum below 2^127 with margin, and is at most 120.
static double shift_for(const KParams& k) {
  const double ln2 = std::log(2.0), e = std::exp(1.0);
  const double bound_r = 2.0 / (e * std::min((double)k.mA, (double)k.mG) * ln2);
  const double bound_t = 2.0 / (e * (double)k.mB * ln2);
  const double bound_w = 1.0 / (e * (double)k.mW * ln2);
  const double m = std::max({1.0, bound_r, bound_t, bound_w});
  // headroom: 2^127 max float, minus log2 of the largest float32 term count
  const double terms = std::ceil(std::log2(32.0));
  return std::floor(std::min(kShiftMixed, 126.0 - terms - std::log2(m)));
}

KParams make_kparams(const Layout& Lo, const hawkes_params_t* p) {
  KParams k;
  std::memset(&k, 0, sizeof(k));
  const int D = Lo.d;
  const double two_pi = 6.283185307179586476925286766559;
  const double log2e = 1.4426950408889634073599246810019;
  k.n = (int)Lo.n;
  k.n_pad = Lo.n_pad;
  k.nb = Lo.nb;
  k.L = Lo.L;
  k.b_fine = Lo.b_fine;
  k.items = Lo.items;
  k.d = D;
  k.nblk = Lo.nblk;
  k.nsblk = Lo.nsblk;
  k.mu0 = p->mu;
  k.tau_x = p->h;
  k.tau_t = p->tau;
  k.theta = p->theta;
  k.omega = p->omega;
  k.h = p->xi;
  k.cbg_unit = std::pow(two_pi, -0.5 * (D + 1)) * std::pow(k.tau_x, -D) / k.tau_t;
  k.cse_unit = k.omega * std::pow(two_pi, -0.5 * D) * std::pow(k.h, -D);
  k.cbg = k.mu0 * k.cbg_unit;
  k.cse = k.theta * k.cse_unit;
  k.log_cbg = k.cbg > 0 ? std::log(k.cbg) : -INFINITY;
  k.log_cse = k.cse > 0 ? std::log(k.cse) : -INFINITY;
  k.cmax = std::max(k.cbg, k.cse);
  k.alpha = 0.5 / (k.tau_x * k.tau_x);
  k.beta = 0.5 / (k.tau_t * k.tau_t);
  k.gamma = 0.5 / (k.h * k.h);
  k.itx2 = 1.0 / (k.tau_x * k.tau_x);
  k.ih2 = 1.0 / (k.h * k.h);
  k.mA = (float)(0.5 * log2e);
  k.mB = (float)(0.5 * log2e);
  k.mG = (float)(0.5 * log2e * (k.tau_x / k.h) * (k.tau_x / k.h));
  k.mW = (float)(log2e * k.omega * k.tau_t);
  k.inv_tx = 1.0 / k.tau_x;
  k.inv_tt = 1.0 / k.tau_t;
  k.mixed = Lo.mixed;
  const double S = Lo.mixed ? shift_for(k) : 0.0;
  k.S = (float)S;
  k.sigma_main = -S * std::log(2.0);
  k.flag_floor = Lo.mixed ? kFloorMixed : kFloorFp64;
  // Culling distances, ignoring the spatial parts of the exponents (which
  // only lower them).  Mixed: both base-2 exponents S - mB dt^2 and S - mW dt
  // (dt in units of tau_t) below -160, where exp2 is 0 to any rounding.
  // Float64: both natural exponents -beta dt^2 and -omega dt below -750,
  // where exp is 0.
  k.cull = Lo.cull;
  k.ru1 = 1;
  if (Lo.mixed) {
    const double lim = S + 160.0;
    k.cull_dtf = (float)std::max(std::sqrt(lim / (double)k.mB), lim / (double)k.mW);
    k.cull_dt = (double)k.cull_dtf * k.tau_t;
  } else {
    k.cull_dt = std::max(std::sqrt(750.0 / k.beta), 750.0 / k.omega);
    k.cull_dtf = (float)(k.cull_dt / k.tau_t);
  }
  return k;
}

template <typename T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Per-request descriptor: constants, inputs and outputs, workspace pieces.
ReqDesc make_desc(const Layout& Lo, const KParams& kp, const double* x, const double* t, void* ws, double* out8,
                  double* grad_x) {
  ReqDesc r;
  std::memset(&r, 0, sizeof(r));
  r.kp = kp;
  r.x = x;
  r.t = t;
  r.grad_x = grad_x;
  r.out8 = out8;
  r.status = at<int>(ws, Lo.off_status);
  r.dconst = at<double>(ws, Lo.off_dconst);
  r.items = at<IPair>(ws, Lo.off_items);
  r.band = at<IPair>(ws, Lo.off_band);
  r.rec = at<void>(ws, Lo.off_rec);
  r.first = at<int>(ws, Lo.off_first);
  r.ps = at<void>(ws, Lo.off_ps);
  r.prow = at<void>(ws, Lo.off_prow);
  r.pcol = at<void>(ws, Lo.off_pcol);
  r.sums = at<double>(ws, Lo.off_sums);
  r.sigma = at<double>(ws, Lo.off_sigma);
  r.flags = at<int>(ws, Lo.off_flags);
  r.list = at<int>(ws, Lo.off_list);
  r.listpos = at<int>(ws, Lo.off_listpos);
  r.bcount = at<int>(ws, Lo.off_bcount);
  r.bstage = at<int>(ws, Lo.off_bstage);
  r.logl = at<double>(ws, Lo.off_logl);
  r.bpart = at<double>(ws, Lo.off_bpart);
  r.gfix = at<double>(ws, Lo.off_gfix);
  r.fixpart = at<double>(ws, Lo.off_fixpart);
  r.mompart = at<double>(ws, Lo.off_mompart);
  // mixed gradient calls form the background moments' gradient terms in the
  // gradient pass; every other call accumulates them in the rate pass
  r.kp.ru1 = (Lo.mixed && grad_x != nullptr) ? 0 : 1;
  return r;
}

// Optional per-stage timing (hawkes_grad_timed): events recorded before each
// launch on the call's stream.
struct StageTimer {
  hipEvent_t ev[kNumStages + 1];
  int used = 0;
};
static thread_local StageTimer* g_timer = nullptr;
// Set while a call must create nothing (hawkes_grad_noalloc): only a side
// stream already in the pool may be used, else the call runs on one stream.
static thread_local bool g_no_create = false;
void set_no_create(bool on) { g_no_create = on; }

static inline void mark(hipStream_t s, int stage) {
  if (g_timer) {
    (void)hipEventRecord(g_timer->ev[stage], s);
    g_timer->used = stage + 1;
  }
}

// A side stream and two events.  In a gradient call the fix-up and finalize
// kernels (fix1, final1, fix2) run on the side
// stream while pass 2 runs on the caller's stream: pass 2 reads nothing they
// write, and k_reduce2, which reads both, waits for the side chain.
// Forks are held exclusively while a call enqueues (an event re-recorded by
// another thread between record and wait would order the wrong work) and
// returned afterwards; the stream work they ordered needs nothing more.  One
// pool per device, grown on demand, kept for the life of the process.
class ForkPool {
 public:
  // allow_create = false (the caller's stream is being captured into a
  // graph, where creating a stream or event is not permitted): only a pooled
  // fork is handed out, else none.
  Fork* take(int dev, bool allow_create) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto& v = free_[dev];
      if (!v.empty()) {
        Fork* f = v.back();
        v.pop_back();
        return f;
      }
    }
    if (!allow_create) return nullptr;
    Fork f{};
    const bool s_ok = hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) == hipSuccess;
    // the two events only order the streams on the device (nothing on the
    // host waits for them), so they record without the system-scope fence
    constexpr unsigned kFlags = hipEventDisableTiming | hipEventDisableSystemFence;
    const bool r_ok = s_ok && hipEventCreateWithFlags(&f.ready, kFlags) == hipSuccess;
    const bool d_ok = r_ok && hipEventCreateWithFlags(&f.done, kFlags) == hipSuccess;
    if (!d_ok) {   // caller falls back to one stream
      if (r_ok) (void)hipEventDestroy(f.ready);
      if (s_ok) (void)hipStreamDestroy(f.side);
      (void)hipGetLastError();
      return nullptr;
    }
    return new Fork(f);
  }
  void give(int dev, Fork* f) {
    std::lock_guard<std::mutex> lk(mu_);
    free_[dev].push_back(f);
  }

 private:
  std::mutex mu_;
  std::map<int, std::vector<Fork*>> free_;
};
static ForkPool& fork_pool() {
  static ForkPool* p = new ForkPool();   // never destroyed: streams outlive static destructors
  return *p;
}
Fork* fork_take(int dev, bool allow_create) { return fork_pool().take(dev, allow_create); }
void fork_give(int dev, Fork* f) { fork_pool().give(dev, f); }

// Host-pinned result buffers of eight doubles, mapped into the device's
// address space (coherent: the device's stores bypass its caches), pooled
// for the life of the process.  The last kernel of a synchronous gradient
// call writes out8 there, so the call reads its scalars after the stream
// synchronization with no device-to-host copy.  A buffer is held by one call
// at a time.
struct Pinned {
  double* host = nullptr;
  double* dev = nullptr;
};
class PinnedPool {
 public:
  Pinned take(bool allow_create) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!free_.empty()) {
        const Pinned p = free_.back();
        free_.pop_back();
        return p;
      }
    }
    Pinned p;
    if (!allow_create) return p;
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, 8 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable) !=
        hipSuccess) {
      (void)hipGetLastError();
      return p;
    }
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || d == nullptr) {
      (void)hipGetLastError();
      (void)hipHostFree(h);
      return p;
    }
    p.host = static_cast<double*>(h);
    p.dev = static_cast<double*>(d);
    return p;
  }
  void give(const Pinned& p) {
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(p);
  }

 private:
  std::mutex mu_;
  std::vector<Pinned> free_;
};
static PinnedPool& pinned_pool() {
  static PinnedPool* p = new PinnedPool();   // never destroyed, like the side streams
  return *p;
}

// The phases over every request of a batch (all with the same D and
// precision).  reqs: device array of descriptors; totals: grid sizes.
// fk == nullptr: everything in order on s (used when stages are timed).
// one != nullptr: a single request whose descriptor the first kernel writes
// to reqs[0].
template <int D, bool MIX>
static bool launch_phases(const ReqDesc* reqs, int nreq, const BatchGrid& g, bool grad, hipStream_t s,
                          const Fork* fk, const ReqDesc* one) {
  bool ok = true;
  mark(s, 0);
  if (one) k_init_one<D><<<1, 1024, 0, s>>>(*one, const_cast<ReqDesc*>(reqs));
  else k_init<D><<<nreq, 1024, 0, s>>>(reqs);
  mark(s, 1);
  k_pack<D, MIX><<<g.pad_blocks, kEvBlock, 0, s>>>(reqs, nreq);
  mark(s, 2);
  if constexpr (MIX) {
    if (grad) k_pass1_mixed<D, false><<<g.items, kThreads, 0, s>>>(reqs, nreq);
    else k_pass1_mixed<D, true><<<g.items, kThreads, 0, s>>>(reqs, nreq);
  } else {
    k_pass1<D, MIX><<<g.items, kThreads, 0, s>>>(reqs, nreq);
  }
  mark(s, 3);
  k_reduce1<D, MIX><<<g.red_blocks, kRedThreads, 0, s>>>(reqs, nreq);
  mark(s, 4);
  const bool fork = grad && fk != nullptr;
  hipStream_t a = s;   // stream of the fix-up and finalize chain
  if (fork) {
    ok = ok && hipEventRecord(fk->ready, s) == hipSuccess;
    ok = ok && hipStreamWaitEvent(fk->side, fk->ready, 0) == hipSuccess;
    a = fk->side;
  }
  k_fix1<D><<<dim3(kFixGrid, nreq), 256, 0, a>>>(reqs);
  mark(a, 5);
  k_final1<D, MIX><<<g.ev_blocks, kEvBlock, 0, a>>>(reqs, nreq);
  mark(a, 6);
  if (!grad) {
    mark(a, 7);
    k_fix2<D><<<nreq, kEvBlock, 0, a>>>(reqs, nreq, 0);   // the finalize reduction alone
    mark(a, 8);
    return ok;
  }
  // finalize reduction + both gradient fix-up sweeps
  const int fix2_blocks = nreq + g.ev_blocks + kFixGrid * nreq;
  if (fork) {
    k_fix2<D><<<fix2_blocks, kEvBlock, 0, a>>>(reqs, nreq, g.ev_blocks);
    ok = ok && hipEventRecord(fk->done, a) == hipSuccess;
  }
  if constexpr (MIX) k_pass2_mixed<D><<<g.items, kThreads, 0, s>>>(reqs, nreq);
  else k_pass2<D, MIX><<<g.items, kThreads, 0, s>>>(reqs, nreq);
  mark(s, 7);
  if (fork) ok = ok && hipStreamWaitEvent(s, fk->done, 0) == hipSuccess;
  else k_fix2<D><<<fix2_blocks, kEvBlock, 0, s>>>(reqs, nreq, g.ev_blocks);
  mark(s, 8);
  k_reduce2<D, MIX><<<g.red_blocks, kRedThreads, 0, s>>>(reqs, nreq);
  mark(s, 9);
  return ok;
}

template <bool MIX>
static bool dispatch_d(int d, const ReqDesc* reqs, int nreq, const BatchGrid& g, bool grad, hipStream_t s,
                       const Fork* fk, const ReqDesc* one) {
  switch (d) {
    case 1: return launch_phases<1, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 2: return launch_phases<2, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 3: return launch_phases<3, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 4: return launch_phases<4, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 5: return launch_phases<5, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 6: return launch_phases<6, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 7: return launch_phases<7, MIX>(reqs, nreq, g, grad, s, fk, one);
    case 8: return launch_phases<8, MIX>(reqs, nreq, g, grad, s, fk, one);
  }
  return false;
}

// Enqueue a batch whose descriptors already sit in device memory (block
// offsets filled in), or, with one != nullptr, a single request whose
// descriptor the first kernel copies to dev_reqs[0].  Gradient batches fork
// onto a side stream unless the stages are being timed.  Returns
// HAWKES_EDEVICE if a launch failed.
int launch_batch(int d, int mixed, const ReqDesc* dev_reqs, int nreq, const BatchGrid& g, bool grad,
                 hipStream_t s, const ReqDesc* one) {
  (void)hipGetLastError();
  int dev = -1;
  Fork* fk = nullptr;
  if (grad && g_timer == nullptr && hipGetDevice(&dev) == hipSuccess) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    fk = fork_pool().take(dev, !capturing && !g_no_create);
  }
  const bool ok = mixed ? dispatch_d<true>(d, dev_reqs, nreq, g, grad, s, fk, one)
                        : dispatch_d<false>(d, dev_reqs, nreq, g, grad, s, fk, one);
  if (fk) fork_pool().give(dev, fk);
  return ok && hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

// Fill the block offsets of descriptors [0, nreq) and return the grid sizes.
BatchGrid assign_blocks(ReqDesc* descs, int nreq) {
  BatchGrid g{0, 0, 0, 0};
  for (int r = 0; r < nreq; ++r) {
    descs[r].blk_items = g.items;
    descs[r].blk_ev = g.ev_blocks;
    descs[r].blk_pad = g.pad_blocks;
    descs[r].blk_red = g.red_blocks;
    g.items += descs[r].kp.items;
    g.ev_blocks += descs[r].kp.nblk;
    g.pad_blocks += descs[r].kp.n_pad / kEvBlock;
    g.red_blocks += descs[r].kp.nsblk;
  }
  return g;
}

// Host-side checks shared by every entry point.
static int check_args(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec,
                      void* ws, size_t ws_bytes, Layout& Lo) {
  if (!x || !t || !p || !ws) return HAWKES_EINVAL;
  if (!make_layout(n, d, prec, Lo)) return HAWKES_EINVAL;
  if (ws_bytes < Lo.total) return HAWKES_EINVAL;
  if (!valid_params(p)) return HAWKES_EPARAM;
  return HAWKES_OK;
}

int run_async(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec, void* ws,
              size_t ws_bytes, void* stream, double* out8, double* grad_x, double* terms, double* out_host) {
  Layout Lo;
  const int st = check_args(x, t, n, d, p, prec, ws, ws_bytes, Lo);
  if (st != HAWKES_OK) return st;
  if (!out8) return HAWKES_EINVAL;
  const KParams kp = make_kparams(Lo, p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  ReqDesc desc = make_desc(Lo, kp, x, t, ws, out8, grad_x);
  desc.terms = terms;
  desc.out_host = grad_x ? out_host : nullptr;   // written by k_reduce2, which only gradient calls run
  const BatchGrid g = assign_blocks(&desc, 1);
  ReqDesc* dev = at<ReqDesc>(ws, Lo.off_desc);
  return launch_batch(d, Lo.mixed, dev, 1, g, grad_x != nullptr, s, &desc);
}

int run_sync(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec, void* ws,
             size_t ws_bytes, void* stream, double* loglik, double* grad_x, double* grad_params, double* terms) {
  Layout Lo;
  if (!ws || !make_layout(n, d, prec, Lo)) return HAWKES_EINVAL;
  double* out8 = at<double>(ws, Lo.off_out8);
  // gradient calls take the scalars from a pinned buffer that their last
  // kernel writes (none is created while allocation is barred)
  const Pinned pin = grad_x ? pinned_pool().take(!g_no_create) : Pinned{};
  if (pin.host)
    for (int q = 0; q < 8; ++q) pin.host[q] = NAN;   // a status the kernel did not write reads as a device error
  int st = run_async(x, t, n, d, p, prec, ws, ws_bytes, stream, out8, grad_x, terms, pin.dev);
  if (st != HAWKES_OK) {
    // argument errors come before any launch; after a failed launch some of
    // the call's kernels may be queued, so the buffer is not reused
    if (pin.host && st != HAWKES_EDEVICE) pinned_pool().give(pin);
    return st;
  }
  double h[8];
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pin.host) {
    if (hipStreamSynchronize(s) != hipSuccess) return HAWKES_EDEVICE;   // buffer not reused either
    for (int q = 0; q < 8; ++q) h[q] = static_cast<volatile double*>(pin.host)[q];
    pinned_pool().give(pin);
    if (std::isnan(h[7])) return HAWKES_EDEVICE;
  } else {
    if (hipMemcpyAsync(h, out8, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return HAWKES_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return HAWKES_EDEVICE;
  }
  st = (int)h[7];
  if (st == HAWKES_EDATA) return st;
  if (loglik) *loglik = h[0];
  if (grad_params)
    for (int k = 0; k < 6; ++k) grad_params[k] = h[1 + k];
  return st;
}

}  // namespace hawkes

extern "C" {

size_t hawkes_workspace_bytes(int64_t n, int d, int prec) {
  hawkes::Layout Lo;
  return hawkes::make_layout(n, d, prec, Lo) ? Lo.total : 0;
}

int hawkes_loglik(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec, void* ws,
                  size_t ws_bytes, void* stream, double* loglik) {
  if (!loglik) return HAWKES_EINVAL;
  return hawkes::run_sync(x, t, n, d, p, prec, ws, ws_bytes, stream, loglik, nullptr, nullptr);
}

int hawkes_grad(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec, void* ws,
                size_t ws_bytes, void* stream, double* loglik, double* grad_x, double* grad_params) {
  if (!grad_x) return HAWKES_EINVAL;
  return hawkes::run_sync(x, t, n, d, p, prec, ws, ws_bytes, stream, loglik, grad_x, grad_params);
}

int hawkes_event_terms(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec,
                       void* ws, size_t ws_bytes, void* stream, double* terms, double* loglik) {
  if (!terms) return HAWKES_EINVAL;
  return hawkes::run_sync(x, t, n, d, p, prec, ws, ws_bytes, stream, loglik, nullptr, nullptr, terms);
}

int hawkes_grad_async(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec,
                      void* ws, size_t ws_bytes, void* stream, double* out8, double* grad_x) {
  return hawkes::run_async(x, t, n, d, p, prec, ws, ws_bytes, stream, out8, grad_x);
}

const char* hawkes_strerror(int status) {
  switch (status) {
    case HAWKES_OK: return "ok";
    case HAWKES_EINVAL: return "invalid argument (n < 2, d outside [1,8], null pointer or workspace too small)";
    case HAWKES_EPARAM: return "parameter non-finite or outside its domain";
    case HAWKES_EDATA: return "data invalid (times unsorted, negative or non-finite; locations non-finite)";
    case HAWKES_EZERORATE: return "some event has zero rate: log-likelihood is -inf";
    case HAWKES_ENOMEM: return "request footprint exceeds the memory budget";
    case HAWKES_EDEVICE: return "HIP runtime error";
    case HAWKES_ESTATE: return "unknown ticket or dataset, or server shutting down";
    case HAWKES_ETIMEOUT: return "wait timed out";
    case HAWKES_EPENDING: return "request pending";
    default: return "unknown status";
  }
}

const char* hawkes_version(void) { return "0.1.0"; }

int hawkes_diagnostics(const void* ws, size_t ws_bytes, int64_t n, int d, int prec, const hawkes_params_t* p,
                       void* stream, int32_t* flags, hawkes_diag_t* out) {
  hawkes::Layout Lo;
  if (!ws || !p || !out || !hawkes::make_layout(n, d, prec, Lo) || ws_bytes < Lo.total) return HAWKES_EINVAL;
  if (!hawkes::valid_params(p)) return HAWKES_EPARAM;
  const hawkes::KParams kp = hawkes::make_kparams(Lo, p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const char* base = static_cast<const char*>(ws);
  int count = 0;
  if (hipMemcpyAsync(&count, base + Lo.off_status + sizeof(int) * hawkes::kStFlagCount, sizeof(int),
                     hipMemcpyDeviceToHost, s) != hipSuccess)
    return HAWKES_EDEVICE;
  if (flags && hipMemcpyAsync(flags, base + Lo.off_flags, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                              s) != hipSuccess)
    return HAWKES_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return HAWKES_EDEVICE;
  out->flagged_rows = count;
  out->shift_log2 = (double)kp.S;
  out->floor_log2 = kp.flag_floor;
  out->cmax = kp.cmax;
  return HAWKES_OK;
}

int hawkes_grad_timed(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec,
                      void* ws, size_t ws_bytes, void* stream, double* loglik, double* grad_x, double* grad_params,
                      float* stage_ms) {
  if (!stage_ms) return HAWKES_EINVAL;
  // events are created once per thread and device and reused
  static thread_local hawkes::StageTimer tm_cache[16];
  static thread_local bool tm_ready[16] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return HAWKES_EDEVICE;
  hawkes::StageTimer& tm = tm_cache[dev];
  if (!tm_ready[dev]) {
    for (int k = 0; k <= hawkes::kNumStages; ++k)
      if (hipEventCreate(&tm.ev[k]) != hipSuccess) return HAWKES_EDEVICE;
    tm_ready[dev] = true;
  }
  tm.used = 0;
  hawkes::g_timer = &tm;
  const int st = hawkes::run_sync(x, t, n, d, p, prec, ws, ws_bytes, stream, loglik, grad_x, grad_params);
  hawkes::g_timer = nullptr;
  for (int k = 0; k < hawkes::kNumStages; ++k) stage_ms[k] = 0.f;
  if (st == HAWKES_OK || st == HAWKES_EZERORATE) {
    (void)hipEventSynchronize(tm.ev[tm.used - 1]);
    for (int k = 0; k + 1 < tm.used; ++k) (void)hipEventElapsedTime(&stage_ms[k], tm.ev[k], tm.ev[k + 1]);
  }
  return st;
}

}  // extern "C"
