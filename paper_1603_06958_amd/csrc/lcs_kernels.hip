// HIP kernels for the all-pairs LCS similarity stage on gfx950 (CDNA4).
//
// The quantity is LCS_len(A, B), computed by the bit-parallel method the
// paper uses for its first stage (Methods, "Pairwise similarities
// calculation": the DP matrix is evaluated w cells at a time, O(|A||B|/w)
// per pair).  The recurrence used here is the one of the bit-vector family
// the paper cites (Hyyro 2004; also Crochemore et al. 2001):
//
//   V = all ones (|A| bits, bit p <-> A[p]);
//   for each symbol b of B:  U = V & PM[b];  V = (V + U) | (V & ~PM[b]);
//   LCS_len(A, B) = number of zero bits of V.
//
// It is exact: every kernel below returns the DP value bit for bit.
//
// Three kernels:
//  * build_masks   -- PM[c][w] for every sequence (one thread per dword).
//  * lcs_fast<cls> -- one wavefront handles 64 rows (one per lane) against a
//    single column sequence, so the column symbol is wave-uniform: it is
//    fetched with scalar loads, and each lane reads its row's mask dwords
//    for that symbol from LDS with 128-bit reads (lane-interleaved layout,
//    conflict free).  Per 32 cells a lane spends three VALU instructions:
//    v_and_b32 (U), v_addc_co_u32 (carry chain through the dwords) and
//    v_bitop3_b32 (the three-input S | (V & ~M), a gfx950 instruction).
//    Persistent workgroups pull work items from an atomic queue.
//  * lcs_plain     -- the baseline: one pair per lane, 64-bit words, masks
//    read from global memory, no LDS and no queue.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lcs_common.h"

namespace famsa {

// ------------------------------------------------------------ mask build

__global__ __launch_bounds__(256) void build_masks_kernel(
    const uint8_t* __restrict__ codes, const uint64_t* __restrict__ dev_off, const uint32_t* __restrict__ len,
    const uint64_t* __restrict__ mask_off, const uint64_t* __restrict__ wprefix, uint32_t nseq,
    uint64_t total_words, uint32_t sigma, uint32_t* __restrict__ masks) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_words) return;
  // last sequence whose first word index is <= g (empty sequences own no words)
  uint32_t lo = 0, hi = nseq;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (wprefix[mid] <= g) lo = mid; else hi = mid;
  }
  const uint32_t s = lo;
  const uint32_t w = (uint32_t)(g - wprefix[s]);
  const uint32_t Ws = (uint32_t)(wprefix[s + 1] - wprefix[s]);
  const uint32_t L = len[s];
  const uint32_t nvalid = min(32u, L - 32u * w);
  const uint4* src = reinterpret_cast<const uint4*>(codes + dev_off[s] + 32ull * w);  // 32-byte aligned, padded
  const uint4 q0 = src[0], q1 = src[1];
  const uint32_t d[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
  uint32_t sym[32];
#pragma unroll
  for (int p = 0; p < 32; ++p) sym[p] = (p < (int)nvalid) ? ((d[p >> 2] >> (8 * (p & 3))) & 0xFFu) : 0xFFFFFFFFu;
  uint32_t* dst = masks + mask_off[s] + w;
  for (uint32_t c = 0; c < sigma; ++c) {
    uint32_t m = 0;
#pragma unroll
    for (int p = 0; p < 32; ++p) m |= (sym[p] == c ? 1u : 0u) << p;
    dst[(uint64_t)c * Ws] = m;
  }
}

__global__ void step_begin_kernel(StepCtl* ctl) {
  if (threadIdx.x == 0) {
    ctl->step = ctl->next_step;
    ctl->next_step = ctl->next_step + ctl->stride;
#pragma unroll
    for (int i = 0; i < 4; ++i) ctl->cursor[i] = 0;
  }
}

// ------------------------------------------------------------ fast kernel

// LDS table of one 64-row group for W dwords per lane: symbol c occupies
// W*64 dwords at c*W*64; inside it, dword quad q of lane l is at q*256 + 4l
// (read with one 128-bit access), a trailing pair at Q*256 + 2l, a trailing
// single dword at Q*256 + (pair ? 128 : 0) + l.  Consecutive lanes read
// consecutive 16-, 8- or 4-byte words, so a wave's read is conflict free.
__device__ __forceinline__ uint32_t lds_index(uint32_t W, uint32_t w, uint32_t lane) {
  const uint32_t Q = W >> 2, R = W & 3, q = w >> 2;
  if (q < Q) return q * 256u + lane * 4u + (w & 3u);
  const uint32_t r = w & 3u;
  if (R >= 2 && r < 2) return Q * 256u + lane * 2u + r;
  return Q * 256u + (R >= 2 ? 128u : 0u) + lane;
}

// One symbol of the column: advance the 32*W-bit vector V of this lane's row.
template <int W>
__device__ __forceinline__ void lcs_step(uint32_t (&V)[W], const uint32_t* __restrict__ tab, uint32_t lane) {
  constexpr int Q = W / 4, R = W % 4;
  uint32_t M[W];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint4 x = *reinterpret_cast<const uint4*>(tab + q * 256 + lane * 4);
    M[4 * q + 0] = x.x;
    M[4 * q + 1] = x.y;
    M[4 * q + 2] = x.z;
    M[4 * q + 3] = x.w;
  }
  if constexpr (R >= 2) {
    const uint2 x = *reinterpret_cast<const uint2*>(tab + Q * 256 + lane * 2);
    M[4 * Q + 0] = x.x;
    M[4 * Q + 1] = x.y;
  }
  if constexpr (R & 1) M[W - 1] = tab[Q * 256 + (R >= 2 ? 128 : 0) + lane];
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t U = V[w] & M[w];
    uint32_t co;
    const uint32_t S = __builtin_addc(V[w], U, c, &co);
    c = co;  // carry out of the top dword is dropped: it leaves the row
    V[w] = __builtin_amdgcn_bitop3_b32(S, V[w], M[w], 0xF4);  // S | (V & ~M)
  }
}

template <int W>
__device__ __forceinline__ void lcs_step4(uint32_t (&V)[W], const uint32_t* __restrict__ lds, uint32_t lane,
                                          uint32_t word) {
  constexpr uint32_t kSym = W * 64;
  lcs_step<W>(V, lds + (word & 0xFFu) * kSym, lane);
  lcs_step<W>(V, lds + ((word >> 8) & 0xFFu) * kSym, lane);
  lcs_step<W>(V, lds + ((word >> 16) & 0xFFu) * kSym, lane);
  lcs_step<W>(V, lds + (word >> 24) * kSym, lane);
}

struct LaneCtx {
  uint64_t out_off;
  uint32_t pos, orig;
};

// All columns of one work item for a group with W dwords per lane.  Waves
// take columns from a shared LDS counter so they stay balanced.
template <int W>
__device__ __forceinline__ void run_item(const uint8_t* __restrict__ codes, const uint64_t* __restrict__ dev_off,
                                         const uint32_t* __restrict__ len, const uint32_t* __restrict__ colmap,
                                         const uint64_t* __restrict__ rowbase, const GroupDesc& g, uint32_t c1,
                                         const uint32_t* __restrict__ lds, uint32_t* s_col, const LaneCtx& lc,
                                         int32_t* __restrict__ out) {
  constexpr uint32_t kSym = W * 64;
  const uint32_t lane = threadIdx.x & 63u;
  for (;;) {
    uint32_t col = 0;
    if (lane == 0) col = atomicAdd(s_col, 1u);
    col = __builtin_amdgcn_readfirstlane(col);
    if (col >= c1) break;
    const uint32_t b = g.colmap_base == kNoMap ? col : colmap[g.colmap_base + col];
    const uint64_t rb = g.rowbase_base == kNoMap ? 0ull : rowbase[g.rowbase_base + b];
    const uint32_t s = g.fam_base + b;
    const uint32_t n = len[s];
    const uint4* B = reinterpret_cast<const uint4*>(codes + dev_off[s]);
    uint32_t V[W];
#pragma unroll
    for (int w = 0; w < W; ++w) V[w] = 0xFFFFFFFFu;
    const uint32_t nch = n >> 4;
    for (uint32_t ch = 0; ch < nch; ++ch) {
      const uint4 q = B[ch];
      lcs_step4<W>(V, lds, lane, q.x);
      lcs_step4<W>(V, lds, lane, q.y);
      lcs_step4<W>(V, lds, lane, q.z);
      lcs_step4<W>(V, lds, lane, q.w);
    }
    const uint32_t rem = n & 15u;
    if (rem) {
      const uint4 q = B[nch];  // inside the 32-byte padding of the sequence
      for (uint32_t t = 0; t < rem; ++t) {
        const uint32_t word = t < 4 ? q.x : (t < 8 ? q.y : (t < 12 ? q.z : q.w));
        const uint32_t sym = (word >> (8u * (t & 3u))) & 0xFFu;
        lcs_step<W>(V, lds + sym * kSym, lane);
      }
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) cnt += __builtin_popcount(~V[w]);
    if (col > lc.pos) {
      const uint64_t o = lc.orig < b ? lc.out_off + (b - lc.orig - 1u) : rb + (lc.orig - b - 1u);
      out[o] = (int32_t)cnt;
    }
  }
}

template <int W, int WHI>
__device__ __forceinline__ void dispatch_w(uint32_t w, const uint8_t* __restrict__ codes,
                                           const uint64_t* __restrict__ dev_off, const uint32_t* __restrict__ len,
                                           const uint32_t* __restrict__ colmap, const uint64_t* __restrict__ rowbase,
                                           const GroupDesc& g, uint32_t c1, const uint32_t* __restrict__ lds,
                                           uint32_t* s_col, const LaneCtx& lc, int32_t* __restrict__ out) {
  if constexpr (W <= WHI) {
    if (w == W) {
      run_item<W>(codes, dev_off, len, colmap, rowbase, g, c1, lds, s_col, lc, out);
      return;
    }
    dispatch_w<W + 1, WHI>(w, codes, dev_off, len, colmap, rowbase, g, c1, lds, s_col, lc, out);
  }
}

template <int CLS>
__global__ __launch_bounds__(1024) void lcs_fast_kernel(
    const uint8_t* __restrict__ codes, const uint64_t* __restrict__ dev_off, const uint32_t* __restrict__ len,
    const uint64_t* __restrict__ mask_off, const uint32_t* __restrict__ masks,
    const GroupDesc* __restrict__ groups, const LaneDesc* __restrict__ lanes, const ItemDesc* __restrict__ items,
    const uint32_t* __restrict__ colmap, const uint64_t* __restrict__ rowbase, const StepRange* __restrict__ ranges,
    StepCtl* __restrict__ ctl, int32_t* __restrict__ out, uint32_t sigma) {
  constexpr int WLO = CLS == 0 ? 1 : kClassWMax[CLS - 1] + 1;
  constexpr int WHI = kClassWMax[CLS];
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_col;
  const uint32_t step = ctl->step;
  const uint32_t begin = ranges[step].begin[CLS];
  const uint32_t end = ranges[step].end[CLS];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t nwaves = blockDim.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_item = begin + atomicAdd(&ctl->cursor[CLS], 1u);
    __syncthreads();
    const uint32_t it = s_item;
    if (it >= end) break;  // same value in every thread
    const ItemDesc item = items[it];
    const GroupDesc g = groups[item.group];
    LaneCtx lc{0ull, 0xFFFFFFFFu, 0u};  // pos = max: an empty lane never stores
    uint32_t seq = 0;
    if (lane < g.nrows) {
      const LaneDesc d = lanes[g.lane_first + lane];
      lc.out_off = d.out_off;
      lc.pos = d.pos;
      lc.orig = d.orig;
      seq = d.seq;
    }
    {  // stage the group's masks in LDS (zero past each row's end)
      const uint32_t W = g.W;
      const uint32_t Ws = lane < g.nrows ? (len[seq] + 31u) >> 5 : 0u;
      const uint64_t mo = lane < g.nrows ? mask_off[seq] : 0ull;
      const uint32_t n = sigma * W;
      for (uint32_t e = wave; e < n; e += nwaves) {
        const uint32_t c = e / W, w = e - c * W;
        const uint32_t v = (w < Ws) ? masks[mo + (uint64_t)c * Ws + w] : 0u;
        lds[c * W * 64u + lds_index(W, w, lane)] = v;
      }
    }
    if (threadIdx.x == 0) s_col = item.c0;
    __syncthreads();
    dispatch_w<WLO, WHI>(g.W, codes, dev_off, len, colmap, rowbase, g, item.c1, lds, &s_col, lc, out);
    __syncthreads();  // LDS and s_item are reused by the next item
  }
}

// ------------------------------------------------------------ plain kernel

// One pair per lane, V in 64-bit words.  W64 > 0: V lives in registers and
// rows have at most W64 words; W64 == 0: V lives in `work` (w64_max words per
// thread, strided across threads), any length.
template <int W64>
__global__ __launch_bounds__(256) void lcs_plain_kernel(
    const uint8_t* __restrict__ codes, const uint64_t* __restrict__ dev_off, const uint32_t* __restrict__ len,
    const uint64_t* __restrict__ mask_off, const uint32_t* __restrict__ masks, const PlainRow* __restrict__ rows,
    const uint32_t* __restrict__ colmap, const uint64_t* __restrict__ rowbase, const StepRange* __restrict__ ranges,
    const StepCtl* __restrict__ ctl, int32_t* __restrict__ out, uint64_t* __restrict__ work) {
  const uint32_t step = ctl->step;
  const uint32_t rb = ranges[step].begin[3], re = ranges[step].end[3];
  const uint64_t total = ranges[step].plain_pairs;
  const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t p = tid; p < total; p += nthreads) {
    uint32_t lo = rb, hi = re;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (rows[mid].pair_first <= p) lo = mid; else hi = mid;
    }
    const PlainRow row = rows[lo];
    const uint32_t col = row.pos + 1u + (uint32_t)(p - row.pair_first);
    const uint32_t b = row.colmap_base == kNoMap ? col : colmap[row.colmap_base + col];
    const uint32_t sa = row.seq, sb = row.fam_base + b;
    const uint32_t m = len[sa], n = len[sb];
    const uint32_t W32 = (m + 31u) >> 5, Wd = (m + 63u) >> 6;
    const uint32_t* pm = masks + mask_off[sa];
    const uint8_t* B = codes + dev_off[sb];
    uint32_t cnt = 0;
    if constexpr (W64 > 0) {
      uint64_t V[W64];
#pragma unroll
      for (int w = 0; w < W64; ++w) V[w] = ~0ull;
      for (uint32_t t = 0; t < n; ++t) {
        const uint32_t* pc = pm + (uint32_t)B[t] * W32;
        unsigned long long carry = 0;
#pragma unroll
        for (int w = 0; w < W64; ++w) {
          if ((uint32_t)w < Wd) {
            const uint64_t lo32 = pc[2 * w];
            const uint64_t hi32 = (2u * w + 1u < W32) ? pc[2 * w + 1] : 0u;
            const uint64_t M = lo32 | (hi32 << 32);
            const uint64_t U = V[w] & M;
            unsigned long long co;
            const uint64_t S = __builtin_addcll(V[w], U, carry, &co);
            carry = co;
            V[w] = S | (V[w] & ~M);
          }
        }
      }
#pragma unroll
      for (int w = 0; w < W64; ++w)
        if ((uint32_t)w < Wd) cnt += __builtin_popcountll(~V[w]);
    } else {
      uint64_t* V = work + tid;
      for (uint32_t w = 0; w < Wd; ++w) V[(uint64_t)w * nthreads] = ~0ull;
      for (uint32_t t = 0; t < n; ++t) {
        const uint32_t* pc = pm + (uint32_t)B[t] * W32;
        unsigned long long carry = 0;
        for (uint32_t w = 0; w < Wd; ++w) {
          const uint64_t lo32 = pc[2 * w];
          const uint64_t hi32 = (2u * w + 1u < W32) ? pc[2 * w + 1] : 0u;
          const uint64_t M = lo32 | (hi32 << 32);
          const uint64_t v = V[(uint64_t)w * nthreads];
          unsigned long long co;
          const uint64_t S = __builtin_addcll(v, v & M, carry, &co);
          carry = co;
          V[(uint64_t)w * nthreads] = S | (v & ~M);
        }
      }
      for (uint32_t w = 0; w < Wd; ++w) cnt += __builtin_popcountll(~V[(uint64_t)w * nthreads]);
    }
    const uint64_t o = row.orig < b ? row.out_off + (b - row.orig - 1u)
                                    : rowbase[row.rowbase_base + b] + (row.orig - b - 1u);
    out[o] = (int32_t)cnt;
  }
}

// ------------------------------------------------------------ launchers

static inline int hip_ok(hipError_t e) { return e == hipSuccess ? 0 : (int)e; }

size_t g_max_lds = kMaxLds;

int launch_build_masks(const DeviceBatch& b, const uint64_t* d_wprefix, uint32_t nseq, uint64_t total_words,
                       uint32_t sigma, uint32_t* d_masks, void* stream) {
  if (total_words == 0) return 0;
  const uint64_t blocks = (total_words + 255) / 256;
  hipLaunchKernelGGL(build_masks_kernel, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, b.codes,
                     b.dev_off, b.len, b.mask_off, d_wprefix, nseq, total_words, sigma, d_masks);
  return hip_ok(hipGetLastError());
}

int launch_step_begin(StepCtl* ctl, void* stream) {
  hipLaunchKernelGGL(step_begin_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, ctl);
  return hip_ok(hipGetLastError());
}

size_t fast_lds_bytes(uint32_t sigma, uint32_t wmax) { return (size_t)sigma * wmax * 64u * 4u; }

template <int CLS>
static const void* fast_fn() {
  return reinterpret_cast<const void*>(&lcs_fast_kernel<CLS>);
}

static const void* fast_kernel_ptr(int cls) {
  switch (cls) {
    case 0: return fast_fn<0>();
    case 1: return fast_fn<1>();
    default: return fast_fn<2>();
  }
}

// Allow the class's dynamic LDS and report how many workgroups of `waves`
// waves fit on one CU.  Call before any launch (and before graph capture).
int fast_prepare(int cls, uint32_t sigma, uint32_t wmax, uint32_t waves, int* blocks_per_cu) {
  const size_t lds = fast_lds_bytes(sigma, wmax);
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, fast_kernel_ptr(cls));
  if (e != hipSuccess) return (int)e;
  if (fa.sharedSizeBytes > kLdsReserve || lds + kLdsReserve > g_max_lds) return (int)hipErrorInvalidValue;
  e = hipFuncSetAttribute(fast_kernel_ptr(cls), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(g_max_lds - fa.sharedSizeBytes));
  if (e != hipSuccess) return (int)e;
  int nb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fast_kernel_ptr(cls), (int)(waves * 64), lds);
  if (e != hipSuccess) return (int)e;
  if (blocks_per_cu) *blocks_per_cu = nb;
  return 0;
}

int launch_fast(int cls, const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t sigma,
                uint32_t wmax, uint32_t blocks, uint32_t waves, void* stream) {
  const size_t lds = fast_lds_bytes(sigma, wmax);
  const dim3 grid(blocks), block(waves * 64);
#define FAMSA_FAST(C)                                                                                            \
  hipLaunchKernelGGL(lcs_fast_kernel<C>, grid, block, lds, (hipStream_t)stream, b.codes, b.dev_off, b.len,        \
                     b.mask_off, b.masks, w.groups, w.lanes, w.items, w.colmap, w.rowbase, w.ranges, ctl, out, sigma)
  switch (cls) {
    case 0: FAMSA_FAST(0); break;
    case 1: FAMSA_FAST(1); break;
    default: FAMSA_FAST(2); break;
  }
#undef FAMSA_FAST
  return hip_ok(hipGetLastError());
}

uint32_t plain_register_w64_limit() { return 40; }

int launch_plain(const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t w64_max,
                 uint32_t blocks, uint64_t* d_work, void* stream) {
  const dim3 grid(blocks), block(kPlainBlock);
  hipStream_t s = (hipStream_t)stream;
#define FAMSA_PLAIN(WW)                                                                                        \
  hipLaunchKernelGGL(lcs_plain_kernel<WW>, grid, block, 0, s, b.codes, b.dev_off, b.len, b.mask_off, b.masks, \
                     w.prows, w.colmap, w.rowbase, w.ranges, ctl, out, d_work)
  if (w64_max <= 2) FAMSA_PLAIN(2);
  else if (w64_max <= 4) FAMSA_PLAIN(4);
  else if (w64_max <= 8) FAMSA_PLAIN(8);
  else if (w64_max <= 16) FAMSA_PLAIN(16);
  else if (w64_max <= 40) FAMSA_PLAIN(40);
  else {
    if (!d_work) return (int)hipErrorInvalidValue;
    FAMSA_PLAIN(0);
  }
#undef FAMSA_PLAIN
  return hip_ok(hipGetLastError());
}

}  // namespace famsa
