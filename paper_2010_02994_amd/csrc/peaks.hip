// Peak-rate microbenchmarks for the VALU roofline denominators on gfx950.
//
// Each kernel runs CH independent dependency chains per lane of one VALU
// instruction kind, so the issue rate (not latency) is measured.  Launches use
// 256 CUs x 8 waves so every SIMD holds two waves.  Results are lane-ops per
// second; dividing by (CUs x 2.4 GHz) gives lane-ops per CU per clock.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CH 8
#define ITERS 4096

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { \
  std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); std::exit(1);} } while (0)

template <int KIND>
__global__ void __launch_bounds__(256) k_peak(float* out, double* out64, float seed, unsigned long long* clk) {
  const unsigned long long c0 = __builtin_amdgcn_s_memtime();
  const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
  float a[CH]; double d[CH]; int iv[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) { a[c] = seed + 0.001f * (threadIdx.x + c); d[c] = a[c]; iv[c] = threadIdx.x + c; }
  const float b = 0.999f, cst = 1e-3f;
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if constexpr (KIND == 0) {            // v_exp_f32
        asm volatile("v_exp_f32 %0, -%0" : "+v"(a[c]));
      } else if constexpr (KIND == 1) {     // v_fma_f32
        asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[c]) : "v"(b), "v"(cst));
      } else if constexpr (KIND == 2) {     // v_fma_f64
        asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[c]) : "v"((double)b), "v"((double)cst));
      } else if constexpr (KIND == 3) {     // v_add_f64
        asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[c]) : "v"((double)cst));
      } else if constexpr (KIND == 4) {     // v_cvt_f32_i32
        asm volatile("v_cvt_f32_i32 %0, %1" : "=v"(a[c]) : "v"(iv[c]));
        asm volatile("v_cvt_i32_f32 %0, %1" : "=v"(iv[c]) : "v"(a[c]));
      } else if constexpr (KIND == 5) {     // v_cvt_f64_f32 + v_cvt_f32_f64
        asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d[c]) : "v"(a[c]));
        asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(a[c]) : "v"(d[c]));
      } else if constexpr (KIND == 6) {     // 1 exp + 3 fma_f32 per step (co-issue probe)
        asm volatile("v_exp_f32 %0, -%0" : "+v"(a[c]));
        asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(iv[c]) : "v"(b), "v"(cst));
        asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(iv[c]) : "v"(b), "v"(cst));
        asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(iv[c]) : "v"(b), "v"(cst));
      } else if constexpr (KIND == 7) {     // v_sub_u32
        asm volatile("v_sub_u32 %0, %0, %1" : "+v"(iv[c]) : "v"(7));
      } else if constexpr (KIND == 8) {     // v_add_f32
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[c]) : "v"(cst));
      } else if constexpr (KIND == 9) {     // v_exp_f64 is absent: v_ldexp_f64
        asm volatile("v_ldexp_f64 %0, %0, %1" : "+v"(d[c]) : "v"(0));
      }
    }
  }
  float s = 0.f; double s64 = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) { s += a[c] + (float)iv[c]; s64 += d[c]; }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
  out64[blockIdx.x * blockDim.x + threadIdx.x] = s64;
  const unsigned long long c1 = __builtin_amdgcn_s_memtime();
  const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) { clk[2 * blockIdx.x] = c1 - c0; clk[2 * blockIdx.x + 1] = r1 - r0; }
}

template <int KIND>
static double run(const char* name, int ops_per_chain_step, int grid, float* o, double* o64) {
  unsigned long long* clk; CHECK(hipMalloc(&clk, sizeof(unsigned long long) * 2 * grid));
  hipEvent_t e0, e1; CHECK(hipEventCreate(&e0)); CHECK(hipEventCreate(&e1));
  k_peak<KIND><<<grid, 256>>>(o, o64, 0.5f, clk);               // warm-up
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  const int reps = 5;
  for (int r = 0; r < reps; ++r) k_peak<KIND><<<grid, 256>>>(o, o64, 0.5f, clk);
  CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
  float ms = 0.f; CHECK(hipEventElapsedTime(&ms, e0, e1));
  double lane_ops = (double)reps * grid * 256.0 * ITERS * CH * ops_per_chain_step;
  double rate = lane_ops / (ms * 1e-3);
  unsigned long long* h = (unsigned long long*)std::malloc(sizeof(unsigned long long) * 2 * grid);
  CHECK(hipMemcpy(h, clk, sizeof(unsigned long long) * 2 * grid, hipMemcpyDeviceToHost));
  double cyc = 0, rt = 0;
  for (int b = 0; b < grid; ++b) { cyc += (double)h[2 * b]; rt += (double)h[2 * b + 1]; }
  const double ghz = cyc / rt * 0.1;   // s_memrealtime ticks at 100 MHz
  std::free(h); CHECK(hipFree(clk));
  std::printf("{\"op\": \"%s\", \"lane_ops_per_s\": %.4e, \"per_cu_per_clk_at_2p4GHz\": %.2f, \"shader_ghz\": %.3f, \"per_cu_per_clk_measured\": %.2f, \"ms\": %.3f}\n",
              name, rate, rate / (256.0 * 2.4e9), ghz, rate / (256.0 * ghz * 1e9), ms / reps);
  CHECK(hipEventDestroy(e0)); CHECK(hipEventDestroy(e1));
  return rate;
}

// LDS accumulate throughput: one wave instruction per step, 64 distinct
// addresses (XOR schedule).  KIND 0: ds_add_f32, 1: ds_add_f64,
// 2: read-modify-write of a float4 (ds_read_b128, 3 adds, ds_write_b128).
template <int KIND>
__global__ void __launch_bounds__(256) k_lds(float* out, float val, int iters) {
  __shared__ float sf[4][256];
  __shared__ double sd[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 4 * 256; i += 256) (&sf[0][0])[i] = 0.f;
  for (int i = threadIdx.x; i < 4 * 64; i += 256) (&sd[0][0])[i] = 0.0;
  __syncthreads();
  const float v = val + 1e-3f * lane;
  for (int it = 0; it < iters; ++it) {
#pragma unroll 8
    for (int k = 0; k < 64; ++k) {
      const int c = lane ^ k;
      if constexpr (KIND == 0) atomicAdd(&sf[w][c], v);
      else if constexpr (KIND == 1) atomicAdd(&sd[w][c], (double)v);
      else {
        float4* p = reinterpret_cast<float4*>(&sf[w][0]) + c;
        float4 q = *p; q.x += v; q.y += v; q.z += v; *p = q;
      }
    }
  }
  __syncthreads();
  out[blockIdx.x * 256 + threadIdx.x] = sf[w][lane] + (float)sd[w][lane];
}

template <int KIND>
static void lds_run(const char* name, float* o, int grid) {
  hipEvent_t a, b; CHECK(hipEventCreate(&a)); CHECK(hipEventCreate(&b));
  const int iters = 100;
  k_lds<KIND><<<grid, 256>>>(o, 1.f, 5);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(a));
  k_lds<KIND><<<grid, 256>>>(o, 1.f, iters);
  CHECK(hipEventRecord(b)); CHECK(hipEventSynchronize(b));
  float ms = 0.f; CHECK(hipEventElapsedTime(&ms, a, b));
  const double wave_steps_per_cu = (double)grid * 4 * iters * 64 / 256.0;
  std::printf("{\"op\": \"%s\", \"ns_per_wave_instruction_per_cu\": %.3f}\n", name, ms * 1e6 / wave_steps_per_cu);
  CHECK(hipEventDestroy(a)); CHECK(hipEventDestroy(b));
}

// Plain streaming copy of a known byte count: the reference against which the
// FETCH_SIZE / WRITE_SIZE hardware counters are scaled.
__global__ void __launch_bounds__(256) k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n4) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

static int copy_mode(size_t mib) {
  const size_t bytes = mib << 20, n4 = bytes / 16;
  float4 *a, *b;
  CHECK(hipMalloc(&a, bytes)); CHECK(hipMalloc(&b, bytes));
  CHECK(hipMemset(a, 0, bytes));
  hipEvent_t e0, e1; CHECK(hipEventCreate(&e0)); CHECK(hipEventCreate(&e1));
  for (int r = 0; r < 3; ++r) {
    CHECK(hipEventRecord(e0));
    k_copy<<<4096, 256>>>(a, b, n4);
    CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
    float ms = 0.f; CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::printf("{\"op\": \"copy\", \"bytes_read\": %zu, \"bytes_written\": %zu, \"ms\": %.4f, \"GB_per_s\": %.1f}\n",
                bytes, bytes, ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
  }
  CHECK(hipFree(a)); CHECK(hipFree(b));
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "copy") == 0) return copy_mode(argc > 2 ? (size_t)std::atoll(argv[2]) : 256);
  hipDeviceProp_t p; CHECK(hipGetDeviceProperties(&p, 0));
  std::printf("{\"device\": \"%s\", \"gcn\": \"%s\", \"cus\": %d, \"clock_khz\": %d}\n",
              p.name, p.gcnArchName, p.multiProcessorCount, p.clockRate);
  const int grid = p.multiProcessorCount * 8;
  float* o; double* o64;
  CHECK(hipMalloc(&o, sizeof(float) * grid * 256)); CHECK(hipMalloc(&o64, sizeof(double) * grid * 256));
  run<0>("v_exp_f32", 1, grid, o, o64);
  run<1>("v_fma_f32", 1, grid, o, o64);
  run<8>("v_add_f32", 1, grid, o, o64);
  run<2>("v_fma_f64", 1, grid, o, o64);
  run<3>("v_add_f64", 1, grid, o, o64);
  run<9>("v_ldexp_f64", 1, grid, o, o64);
  run<4>("v_cvt_f32_i32+v_cvt_i32_f32", 2, grid, o, o64);
  run<5>("v_cvt_f64_f32+v_cvt_f32_f64", 2, grid, o, o64);
  run<7>("v_sub_u32", 1, grid, o, o64);
  run<6>("exp+3fma (instructions)", 4, grid, o, o64);
  lds_run<0>("ds_add_f32", o, grid);
  lds_run<1>("ds_add_f64", o, grid);
  lds_run<2>("ds_read_b128+3 v_add_f32+ds_write_b128", o, grid);
  CHECK(hipFree(o)); CHECK(hipFree(o64));
  return 0;
}
