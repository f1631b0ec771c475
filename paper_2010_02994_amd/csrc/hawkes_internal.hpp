// Internal interface between the evaluation entry points and the serving
// runtime of libhawkes (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/hawkes.h"
#include "hawkes_common.hpp"

namespace hawkes {

struct Layout {
  int64_t n = 0;
  int d = 0, mixed = 0, cull = 0;
  int nb = 0, n_pad = 0, L = 1, b_fine = 0, items = 0, nblk = 0, nsblk = 0;
  size_t off_desc, off_status, off_dconst, off_out8, off_items, off_band, off_rec, off_first, off_ps, off_prow,
      off_pcol, off_sums, off_sigma, off_flags, off_list, off_listpos, off_bcount, off_bstage, off_logl, off_bpart,
      off_gfix, off_fixpart, off_mompart, total;
};

struct BatchGrid {
  int items;       // blocks of a pair-pass launch
  int ev_blocks;   // blocks of a per-event launch
  int pad_blocks;  // blocks of the pack launch
  int red_blocks;  // blocks of a reduction launch
};

bool make_layout(int64_t n, int d, int prec, Layout& Lo);
bool valid_params(const hawkes_params_t* p);
KParams make_kparams(const Layout& Lo, const hawkes_params_t* p);
ReqDesc make_desc(const Layout& Lo, const KParams& kp, const double* x, const double* t, void* ws, double* out8,
                  double* grad_x);
BatchGrid assign_blocks(ReqDesc* descs, int nreq);
int launch_batch(int d, int mixed, const ReqDesc* dev_reqs, int nreq, const BatchGrid& g, bool grad, hipStream_t s,
                 const ReqDesc* one = nullptr);
// Enqueue one full evaluation (validation, rate pass, finalize and, when
// grad_x is not null, the gradient pass) with no host synchronization.
// out_host (gradient calls only; may be null): device-visible pinned memory
// that the last kernel also writes out8 to.
int run_async(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec, void* ws,
              size_t ws_bytes, void* stream, double* out8, double* grad_x, double* terms = nullptr,
              double* out_host = nullptr);
// run_async, then the scalars to the host (stream synchronized).
int run_sync(const double* x, const double* t, int64_t n, int d, const hawkes_params_t* p, int prec, void* ws,
             size_t ws_bytes, void* stream, double* loglik, double* grad_x, double* grad_params,
             double* terms = nullptr);
// While on (per host thread), gradient calls create no side stream or event:
// they use one already pooled, or run every kernel on the caller's stream.
void set_no_create(bool on);
// A side stream and two events, from a per-device pool kept for the life of
// the process.  A fork is held exclusively while a call enqueues and given
// back afterwards.  allow_create = false (the stream is being captured into a
// graph): only a pooled fork is handed out, else nullptr.
struct Fork {
  hipStream_t side;
  hipEvent_t ready, done;
};
Fork* fork_take(int dev, bool allow_create);
void fork_give(int dev, Fork* f);

// Enqueue one Bayesian MDS evaluation; accumulate: grad_x += its location
// gradient instead of grad_x = it.  phase 0: everything on s; phase 1: the
// pair pass and the scalars only; phase 2: only the per-event gradient
// reduction (after phase 1's work, with the same arguments).
int bmds_enqueue(const double* x, const double* delta, int64_t n, int d, double sigma, int prec, void* ws,
                 size_t ws_bytes, hipStream_t s, double* out4, double* grad_x, bool accumulate, int phase = 0);

}  // namespace hawkes
