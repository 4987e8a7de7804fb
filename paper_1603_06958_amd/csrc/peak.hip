// Integer-VALU ceiling of the LCS recurrence's instruction mix on gfx950.
//
// The bit-parallel LCS step costs three 32-bit VALU instructions per 32 DP
// cells (FAMSA, Methods, "Pairwise similarities calculation": w cells per
// machine word, O(|A||B|/w) per pair): v_and_b32 (U = V & M),
// v_addc_co_u32 (V + U with the carry chained through the dwords of a row)
// and v_bitop3_b32 (S | (V & ~M)).  This kernel runs long chains of exactly
// those instructions on every CU, with the masks in registers instead of LDS
// and nothing else in the loop, so its rate is the ceiling the LCS kernels
// are measured against.  Each workgroup's first wave also reads the shader
// clock counter (s_memtime) and the constant-rate counter (s_memrealtime)
// around its loop, which gives the clock the chip ran at under this load.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "runtime.h"

namespace famsa {
namespace {

constexpr int kPeakW = 8;       // dwords per lane (one 256-bit row vector)
constexpr int kPeakUnroll = 8;  // column steps per loop iteration

// Variant 0: the recurrence itself, W dwords per step, four mask sets
// rotating through the unrolled steps.
__device__ __forceinline__ void mix_step(uint32_t (&V)[kPeakW], const uint32_t (&M)[kPeakW]) {
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kPeakW; ++w) {
    const uint32_t U = V[w] & M[w];
    uint32_t co;
    const uint32_t S = __builtin_addc(V[w], U, c, &co);
    c = co;
    V[w] = __builtin_amdgcn_bitop3_b32(S, V[w], M[w], 0xF4);
  }
}

__global__ __launch_bounds__(256) void valu_peak_kernel(uint32_t variant, uint32_t iters, uint32_t seed,
                                                        uint32_t* __restrict__ sink,
                                                        uint64_t* __restrict__ clocks) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t V[kPeakW], M0[kPeakW], M1[kPeakW], M2[kPeakW], M3[kPeakW];
#pragma unroll
  for (int w = 0; w < kPeakW; ++w) {
    const uint32_t x = (t + 1u) * 2654435761u ^ (seed + 97u * (uint32_t)w);
    V[w] = 0xFFFFFFFFu ^ (x & 0x00FF00FFu);
    M0[w] = x * 2246822519u;
    M1[w] = x * 3266489917u;
    M2[w] = x * 668265263u;
    M3[w] = x * 374761393u;
  }
  uint64_t t0 = 0, r0 = 0;
  if (threadIdx.x == 0) {
    t0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  if (variant == 0) {
    for (uint32_t i = 0; i < iters; ++i) {
      mix_step(V, M0);
      mix_step(V, M1);
      mix_step(V, M2);
      mix_step(V, M3);
      mix_step(V, M1);
      mix_step(V, M0);
      mix_step(V, M3);
      mix_step(V, M2);
    }
  } else if (variant == 1) {  // v_and_b32 only, eight independent chains
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
      for (int u = 0; u < 3 * kPeakUnroll; ++u) {
#pragma unroll
        for (int w = 0; w < kPeakW; ++w) asm volatile("v_and_b32 %0, %0, %1" : "+v"(V[w]) : "v"(M0[w]));
      }
    }
  } else if (variant == 2) {  // v_addc_co_u32 only, one carry chain through the eight dwords
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
      for (int u = 0; u < 3 * kPeakUnroll; ++u) {
        asm volatile(
            "v_add_co_u32 %0, vcc, %0, %8\n\t"
            "v_addc_co_u32 %1, vcc, %1, %9, vcc\n\t"
            "v_addc_co_u32 %2, vcc, %2, %10, vcc\n\t"
            "v_addc_co_u32 %3, vcc, %3, %11, vcc\n\t"
            "v_addc_co_u32 %4, vcc, %4, %12, vcc\n\t"
            "v_addc_co_u32 %5, vcc, %5, %13, vcc\n\t"
            "v_addc_co_u32 %6, vcc, %6, %14, vcc\n\t"
            "v_addc_co_u32 %7, vcc, %7, %15, vcc"
            : "+v"(V[0]), "+v"(V[1]), "+v"(V[2]), "+v"(V[3]), "+v"(V[4]), "+v"(V[5]), "+v"(V[6]), "+v"(V[7])
            : "v"(M0[0]), "v"(M0[1]), "v"(M0[2]), "v"(M0[3]), "v"(M0[4]), "v"(M0[5]), "v"(M0[6]), "v"(M0[7])
            : "vcc");
      }
    }
  } else {  // v_bitop3_b32 only, eight independent chains
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
      for (int u = 0; u < 3 * kPeakUnroll; ++u) {
#pragma unroll
        for (int w = 0; w < kPeakW; ++w)
          asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xf4" : "+v"(V[w]) : "v"(M0[w]), "v"(M1[w]));
      }
    }
  }
  if (threadIdx.x == 0) {
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    clocks[2 * blockIdx.x + 0] = t1 - t0;
    clocks[2 * blockIdx.x + 1] = r1 - r0;
  }
  uint32_t acc = 0;
#pragma unroll
  for (int w = 0; w < kPeakW; ++w) acc ^= V[w];
  sink[t] = acc;  // keeps every chain live
}

}  // namespace
}  // namespace famsa

using namespace famsa;

extern "C" int famsa_valu_peak(int device, uint32_t variant, uint32_t blocks_per_cu, uint32_t iters,
                               famsa_valu_peak_result* out) {
  clear_error();
  if (!out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  if (variant > 3) return set_error(FAMSA_LCS_EINVAL, "variant %u: 0..3", variant);
  if (blocks_per_cu < 1 || blocks_per_cu > 32) return set_error(FAMSA_LCS_EINVAL, "blocks_per_cu %u: 1..32", blocks_per_cu);
  if (iters < 1 || iters > (1u << 24)) return set_error(FAMSA_LCS_EINVAL, "iters %u: 1..2^24", iters);
  FAMSA_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  FAMSA_HIP(hipGetDeviceProperties(&prop, device));
  int wall_khz = 0;
  FAMSA_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device));
  const uint32_t cus = (uint32_t)prop.multiProcessorCount;
  const uint32_t blocks = cus * blocks_per_cu;
  DevMem sink, clocks;
  int rc = sink.alloc((size_t)blocks * 256 * 4);
  if (rc) return rc;
  if ((rc = clocks.alloc((size_t)blocks * 16))) return rc;
  hipStream_t s = nullptr;
  FAMSA_HIP(hipStreamCreate(&s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int err = 0;
  float ms = 0.f;
  auto launch = [&](uint32_t it) {
    hipLaunchKernelGGL(valu_peak_kernel, dim3(blocks), dim3(256), 0, s, variant, it, 12345u, sink.as<uint32_t>(),
                       clocks.as<uint64_t>());
    return hipGetLastError();
  };
  std::vector<uint64_t> h(2 * (size_t)blocks);
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) err = 1;
  if (!err && launch(iters < 64 ? iters : 64) != hipSuccess) err = 2;  // warm-up
  if (!err && hipEventRecord(e0, s) != hipSuccess) err = 3;
  if (!err && launch(iters) != hipSuccess) err = 4;
  if (!err && hipEventRecord(e1, s) != hipSuccess) err = 5;
  if (!err && hipEventSynchronize(e1) != hipSuccess) err = 6;
  if (!err && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) err = 7;
  if (!err && hipMemcpy(h.data(), clocks.p, h.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) err = 8;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  if (err) return set_error(FAMSA_LCS_EDEVICE, "peak kernel failed (step %d)", err);
  // the clock of each workgroup's loop: counter ticks over constant-rate ticks
  double ghz = 0.0, cyc = 0.0;
  for (uint32_t b = 0; b < blocks; ++b) {
    const double t = (double)h[2 * b], r = (double)h[2 * b + 1];
    if (r > 0) ghz += t / (r / ((double)wall_khz * 1e3)) / 1e9;
    cyc += t;
  }
  ghz /= blocks;
  const double per_lane = (double)iters * kPeakUnroll * kPeakW * (variant == 0 ? 3.0 : 3.0);
  const double lane_ops = per_lane * (double)blocks * 256.0;
  out->ms = ms;
  out->lane_ops = lane_ops;
  out->ops_per_s = lane_ops / (ms * 1e-3);
  out->clock_ghz = ghz;
  out->cus = cus;
  out->mean_loop_cycles = cyc / blocks;
  out->lane_ops_per_clk_per_cu = ghz > 0 ? out->ops_per_s / (ghz * 1e9 * cus) : 0.0;
  return 0;
}
