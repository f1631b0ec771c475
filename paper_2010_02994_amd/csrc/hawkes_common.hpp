// Shared definitions of the gfx950 Hawkes library (device and host side).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hawkes {

constexpr int kWaves = 4;               // waves per workgroup
constexpr int kThreads = 64 * kWaves;   // workgroup size
constexpr int kRowsPerLane = 2;         // rows each lane owns in the pair passes
constexpr int kBandRows = kThreads * kRowsPerLane;  // rows per band (512)
constexpr int kTile = 64;               // columns per tile (one wave width)
constexpr int kMaxD = 8;

// Status words kept in the workspace.
enum StatusSlot { kStData = 0, kStZero = 1, kStFlagCount = 2, kStSlots = 16 };

// Host-computed constants of one evaluation, passed to kernels by value.
struct KParams {
  int n;          // events
  int n_pad;      // NB * kBandRows
  int nb;         // row bands
  int L;          // column tiles per work item
  int items;      // work items of a pair pass
  int d;
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
  float Ab, Bt, Gs, Ws, S;    // log2(e)/(2 tau_x^2), log2(e)/(2 tau_t^2), log2(e)/(2 h^2), log2(e) omega, S
  double sigma_main;          // natural log of the scale the main pass sums carry (-S ln 2, or 0)
  double flag_floor;          // a row is recomputed when lambda~ < cmax * 2^flag_floor
  int mixed;
};

}  // namespace hawkes
