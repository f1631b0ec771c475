// Shared definitions of the gfx950 Hawkes library (device and host side).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hawkes {

// Pair-pass geometry: waves per workgroup and rows per lane (a band has
// 64 * kWaves * kRowsPerLane rows).  Overridable at build time for tuning.
#ifndef HK_WAVES
#define HK_WAVES 4
#endif
#ifndef HK_ROWS_PER_LANE
#define HK_ROWS_PER_LANE 2
#endif
#ifndef HK_RATE_WAVES_PER_EU
#define HK_RATE_WAVES_PER_EU 4
#endif
#ifndef HK_GRAD_WAVES_PER_EU
#define HK_GRAD_WAVES_PER_EU 5
#endif
#ifndef HK_RATE_EXP_STEPS
#define HK_RATE_EXP_STEPS 1
#endif
#ifndef HK_GRAD_EXP_STEPS
#define HK_GRAD_EXP_STEPS 1
#endif
// Column steps of a tile's 64-step sweep unrolled per loop trip in the mixed
// rate and gradient passes (32: one trip per float32 row fold).
#ifndef HK_RATE_UNROLL
#define HK_RATE_UNROLL 32
#endif
#ifndef HK_GRAD_UNROLL
#define HK_GRAD_UNROLL 32
#endif
constexpr int kWaves = HK_WAVES;        // waves per workgroup
constexpr int kThreads = 64 * kWaves;   // workgroup size
constexpr int kRowsPerLane = HK_ROWS_PER_LANE;  // rows each lane owns in the pair passes
constexpr int kBandRows = kThreads * kRowsPerLane;  // rows per band (512)
constexpr int kTile = 64;               // columns per tile (one wave width)
constexpr int kMaxD = 8;
constexpr int kFixGrid = 256;            // workgroups per request in the fix-up kernels
constexpr int kFixSeg = 16;             // partner segments per flagged row in the fix-up kernels
constexpr int kEvBlock = 256;           // events per block of the per-event kernels
constexpr int kRedEv = 64;              // events per workgroup of the partial-sum reductions
constexpr int kRedWaves = 16;           // waves per reduction workgroup (each sums a stride of partials)
// float32 pair passes: steps whose exps are issued together (rate, gradient)
// Waves per SIMD the mixed passes are compiled for: the register budget
// (512 / waves per lane) must hold the rows' state, which grows with D, or
// the kernel spills to scratch.  The set values apply at D <= 2; wider
// records take fewer waves.
constexpr int rate_waves(int d, bool ru) { return ru && d >= 2 ? 4 : HK_RATE_WAVES_PER_EU; }
constexpr int grad_waves(int d) { return d <= 2 ? HK_GRAD_WAVES_PER_EU : d <= 4 ? 5 : d <= 6 ? 4 : 3; }
// Column tiles of a work item of band `band`.
__host__ __device__ inline int item_tiles(int band, int b_fine, int L) { return band < b_fine ? 1 : L; }

constexpr int kRateExpSteps = HK_RATE_EXP_STEPS;
constexpr int kGradExpSteps = HK_GRAD_EXP_STEPS;

// Plain pairs and 16-byte chunks (the HIP vector types cannot be used through
// address-space-qualified pointers).
struct IPair { int x, y; };
struct alignas(16) Chunk16 { unsigned a, b, c, d; };

// Sums NV values over the workgroup (blockDim.x a power of two; sh holds
// NV * blockDim.x elements) with one fixed-shape tree per value, so the
// result does not depend on timing; every thread receives the totals.
template <typename T, int NV>
__device__ __forceinline__ void block_sum_n(T (&v)[NV], T* sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
#pragma unroll
  for (int q = 0; q < NV; ++q) sh[q * nt + tid] = v[q];
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) sh[q * nt + tid] += sh[q * nt + tid + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = sh[q * nt];
  __syncthreads();
}

// Status words kept in each request's workspace.
enum StatusSlot { kStData = 0, kStZero = 1, kStFlagCount = 2, kStSlots = 16 };

// Constants of one evaluation (host-computed from the parameters and sizes).
struct KParams {
  int n;          // events
  int n_pad;      // NB * kBandRows
  int nb;         // row bands
  int L;          // column tiles per work item (bands below b_fine: one)
  int b_fine;     // bands dispatched last, split into one-tile items
  int items;      // work items of a pair pass
  int d;
  int nblk;       // ceil(n / kEvBlock)
  int nsblk;      // ceil(n / kRedEv): reduction workgroups (flagged-row staging blocks)
  int mixed;
  // model parameters (paper symbols)
  double mu0, tau_x, tau_t, theta, omega, h;
  double cbg, cse;            // weighted pair constants
  double cbg_unit, cse_unit;  // per unit mu0, per unit theta
  double log_cbg, log_cse;    // natural logs (-inf when the weight is 0)
  double cmax;                // max(cbg, cse)
  // float64 path: natural-exponent scales
  double alpha, beta, gamma;  // 1/(2 tau_x^2), 1/(2 tau_t^2), 1/(2 h^2)
  double itx2, ih2;           // 1/tau_x^2, 1/h^2
  // mixed path: base-2 exponent scales and the constant shift S
  // The mixed path stores coordinates in units of tau_x and times in units of
  // tau_t; in those units the base-2 exponents are
  //   background  S - mA r2 - mB dt^2,   excitation  S - mG r2 - mW dt
  // with mA = mB = log2(e)/2, mG = log2(e)/2 (tau_x/h)^2, mW = log2(e) omega tau_t.
  float mA, mB, mG, mW, S;
  double inv_tx, inv_tt;      // 1/tau_x, 1/tau_t (packing scales)
  double sigma_main;          // natural log of the scale the main pass sums carry (-S ln 2, or 0)
  double flag_floor;          // a row is recomputed when lambda~ < cmax * 2^flag_floor
  // exact culling (optional): a column tile whose every pair is further apart
  // in time than cull_dt (in the records' time units) adds exactly zero
  int cull;
  int ru1;                    // the rate pass accumulates the background moments R, U (else the gradient pass
                              // forms their parameter-gradient terms; mixed gradient calls)
  float cull_dtf;             // mixed records: bandwidth units of tau_t
  double cull_dt;             // float64 records: time units
};

// One request of a launch: its constants, its inputs and outputs, the pieces
// of its workspace, and where its blocks start in each batched grid.
struct ReqDesc {
  KParams kp;
  const double* x;
  const double* t;
  double* grad_x;   // null: rate pass and finalize only
  double* out8;     // [loglik, 6 parameter gradients, status]
  int* status;
  double* dconst;
  IPair* items;
  IPair* band;
  void* rec;
  int* first;
  void* ps;
  void* prow;       // row partials: float (mixed) or double
  void* pcol;
  double* sums;
  double* sigma;
  int* flags;
  int* list;
  int* listpos;
  int* bcount;
  int* bstage;
  double* logl;
  double* bpart;
  double* gfix;
  double* fixpart;
  double* terms;    // optional, n x 4: per-event terms written by k_final1 (null: none)
  double* mompart;  // items x 2: per-item moment sums of the mixed gradient pass
  double* out_host; // optional host-pinned copy of out8, written by the gradient call's last kernel (null: none)
  int blk_items;    // first block of this request in a pair-pass launch
  int blk_ev;       // first block in a per-event launch (kEvBlock events per block)
  int blk_pad;      // first block in the pack launch (n_pad / kEvBlock blocks)
  int blk_red;      // first block in a reduction launch (kRedEv events per block)
};

// Float64 exp of the pair passes and the Metropolis kernels, by Tang's table-driven method (P. T. P. Tang,
// ACM Trans. Math. Softw. 15(2), 1989) with 2^8 table entries tab[j] = 2^(j/256)
// held in LDS: z = (256 m + j) ln2/256 + r with |r| <= ln2/512, and
// exp(z) = 2^m tab[j] (1 + p(r)), p the Taylor polynomial of expm1 of degree 4,
// truncated below 4e-17 relative.  The reduction subtracts k ln2/256 in two
// fused steps (ln2/256 split into a double and its remainder), so r is exact
// to ~1e-18.  ldexp rounds once, also into the subnormal range.  Arguments are
// first clamped at -1100: exp is 0 below -746, ldexp returns exactly 0 for
// such scales, and the clamp keeps k in range (and maps -inf to 0).
constexpr int kExpBits = 8;
constexpr int kExpTab = 1 << kExpBits;
__device__ __forceinline__ double exp_tab(double z, const double* __restrict__ tab) {
  constexpr double kInvStep = 369.3299304675746;        // 256 / ln2
  constexpr double kStepHi = 0x1.62e42fefa39efp-9;       // ln2 / 256, rounded
  constexpr double kStepLo = 0x1.abc9e3b39803fp-64;      // ln2 / 256 - kStepHi
  z = __builtin_fmax(z, -1100.0);
  // k = z 2^8/ln2 rounded to an integer by adding 1.5 * 2^52 (the sum's unit
  // in the last place is 1, so the low word of its bits is k in two's
  // complement; exact for |k| < 2^31, and |k| < 410,000 after the clamp)
  constexpr double kRound = 0x1.8p52;
  const double kb = __builtin_fma(z, kInvStep, kRound);
  const int k = __double2loint(kb);
  const double kf = kb - kRound;
  double r = __builtin_fma(-kf, kStepHi, z);
  r = __builtin_fma(-kf, kStepLo, r);
  double p = __builtin_fma(r, 1.0 / 24.0, 1.0 / 6.0);
  p = __builtin_fma(r, p, 0.5);
  p = __builtin_fma(r, p, 1.0);
  p = r * p;
  const double tj = tab[k & (kExpTab - 1)];
  return __builtin_ldexp(__builtin_fma(tj, p, tj), k >> kExpBits);
}

// Fills the table of exp_tab; the caller synchronizes the workgroup before
// the first use.
__device__ __forceinline__ void fill_exp_table(double* tab) {
  for (int j = threadIdx.x; j < kExpTab; j += blockDim.x) tab[j] = exp2((double)j / kExpTab);
}

}  // namespace hawkes
