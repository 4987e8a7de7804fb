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
//    single column sequence, so the column symbol is wave-uniform; each lane
//    reads its row's mask dwords for that symbol from LDS with 128-bit reads
//    (lane-interleaved layout, conflict free), at an address formed by one
//    SDWA add from the pre-scaled symbol.  Per 32 cells a lane spends three
//    VALU instructions:
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

// LDS table of one 64-row group: for every dword quad q of the rows' masks
// (W dwords per lane, Q = ceil(W/4) quads, the last one zero padded) and
// every symbol c, the 64 lanes' 16-byte quads lie side by side:
//   byte offset = q * SIG * 1024 + c * 1024 + lane * 16.
// A wave's 128-bit read of one (q, c) plane is 1 KB of consecutive bytes,
// conflict free, and the symbol's part c * 1024 does not depend on W, so the
// column streams store it pre-scaled and one SDWA v_add forms the address.
// When W is not a multiple of 4 the last quad is read only as far as W
// reaches (a 32-, 64- or 96-bit read at a 16-byte lane stride): lanes 16
// apart then meet in the same banks, and such a read takes as many LDS
// cycles as a full quad, no more.
template <int SIG>
__device__ __forceinline__ uint32_t lds_byte(uint32_t q, uint32_t c, uint32_t lane) {
  return q * (SIG * 1024u) + c * 1024u + lane * 16u;
}

// One column symbol: advance this lane's 32*W-bit vector V.  `p` is the
// lane's address in the symbol's plane of quad 0.
template <int W, int SIG>
__device__ __forceinline__ void lcs_step(uint32_t (&V)[W], const char* __restrict__ p) {
  constexpr int Q = (W + 3) / 4;
  uint32_t M[4 * Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint4 x = *reinterpret_cast<const uint4*>(p + q * (SIG * 1024));
    M[4 * q + 0] = x.x;
    M[4 * q + 1] = x.y;
    M[4 * q + 2] = x.z;
    M[4 * q + 3] = x.w;
  }
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t U = V[w] & M[w];
    uint32_t co;
    const uint32_t S = __builtin_addc(V[w], U, c, &co);
    c = co;  // the carry out of the top dword leaves the row
    V[w] = __builtin_amdgcn_bitop3_b32(S, V[w], M[w], 0xF4);  // S | (V & ~M)
  }
}

struct LaneCtx {
  uint64_t out_off;
  uint32_t pos, orig, len;
};

// The value a tile holds for a pair with LCS `lcs` of sequences of lengths
// la and lb: the LCS, the indel distance la + lb - 2 LCS, or the similarity
// LCS / indel^2 (Methods, "Pairwise similarities calculation") as the float
// rounding of the correctly rounded double, +infinity for indel 0.
__device__ __forceinline__ int32_t tile_value(uint32_t values, uint32_t lcs, uint32_t la, uint32_t lb) {
  if (values == FAMSA_LCS_VALUES_LCS) return (int32_t)lcs;
  const int32_t d = (int32_t)(la + lb) - 2 * (int32_t)lcs;
  if (values == FAMSA_LCS_VALUES_INDEL) return d;
  const double dd = (double)d * (double)d;  // exact: d <= 131070
  const float f = d == 0 ? __builtin_inff() : (float)((double)lcs / dd);
  return __float_as_int(f);
}

// All columns of one work item for a group with W dwords per lane.  Waves
// take columns from a shared LDS counter so they stay balanced.  The column
// stream is read with vector loads at a wave-uniform address (kept in VGPRs,
// counted by vmcnt, so waiting for it never waits for the LDS reads), one
// 8-symbol chunk ahead of use.
template <int W, int SIG>
__device__ __forceinline__ void run_item(const DeviceBatch& bt, const uint32_t* __restrict__ colmap,
                                         const uint64_t* __restrict__ rowbase, const GroupDesc& g, uint32_t c1,
                                         const char* __restrict__ lds, uint32_t* s_col, const LaneCtx& lc,
                                         int32_t* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63u;
  const char* lbase = lds + lane * 16u;
  uint32_t vzero;  // a zero the compiler must treat as per-lane: keeps the stream loads in VGPRs
  asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
  for (;;) {
    uint32_t col = 0;
    if (lane == 0) col = atomicAdd(s_col, 1u);
    col = __builtin_amdgcn_readfirstlane(col);
    if (col >= c1) break;
    uint32_t b = col;
    uint64_t rb = 0;
    if (g.colmap_base != kNoMap) {
      if (col < g.nmap) {
        b = colmap[g.colmap_base + col];
        rb = rowbase[g.rowbase_base + col];
      } else {
        b = col + g.shift;  // above every row of the group
      }
    }
    const uint32_t s = g.fam_base + b;
    const uint32_t n = bt.len[s];
    const uint4* B = reinterpret_cast<const uint4*>(bt.sym + bt.sym_off[s]) + vzero;
    uint32_t V[W];
#pragma unroll
    for (int w = 0; w < W; ++w) V[w] = 0xFFFFFFFFu;
    const uint32_t nch = n >> 3;
    uint4 nxt = B[0];
    for (uint32_t ch = 0; ch < nch; ++ch) {
      const uint4 q = nxt;
      nxt = B[ch + 1];  // the spare chunk makes this read safe on the last chunk
      lcs_step<W, SIG>(V, lbase + (q.x & 0xFFFFu));
      lcs_step<W, SIG>(V, lbase + (q.x >> 16));
      lcs_step<W, SIG>(V, lbase + (q.y & 0xFFFFu));
      lcs_step<W, SIG>(V, lbase + (q.y >> 16));
      lcs_step<W, SIG>(V, lbase + (q.z & 0xFFFFu));
      lcs_step<W, SIG>(V, lbase + (q.z >> 16));
      lcs_step<W, SIG>(V, lbase + (q.w & 0xFFFFu));
      lcs_step<W, SIG>(V, lbase + (q.w >> 16));
    }
    const uint32_t rem = n & 7u;
    if (rem) {
      const uint32_t qw[4] = {nxt.x, nxt.y, nxt.z, nxt.w};
#pragma unroll
      for (uint32_t t = 0; t < 7; ++t) {
        if (t < rem) lcs_step<W, SIG>(V, lbase + ((qw[t >> 1] >> (16u * (t & 1u))) & 0xFFFFu));
      }
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) cnt += __builtin_popcount(~V[w]);
    if (col > lc.pos) {
      const uint64_t o = lc.orig < b ? lc.out_off + (b - lc.orig - 1u) : rb + (lc.orig - b - 1u);
      out[o] = tile_value(bt.values, cnt, lc.len, n);
    }
  }
}

template <int W, int WHI, int SIG>
__device__ __forceinline__ void dispatch_w(uint32_t w, const DeviceBatch& bt, const uint32_t* __restrict__ colmap,
                                           const uint64_t* __restrict__ rowbase, const GroupDesc& g, uint32_t c1,
                                           const char* __restrict__ lds, uint32_t* s_col, const LaneCtx& lc,
                                           int32_t* __restrict__ out) {
  if constexpr (W <= WHI) {
    if (w == W) {
      run_item<W, SIG>(bt, colmap, rowbase, g, c1, lds, s_col, lc, out);
      return;
    }
    dispatch_w<W + 1, WHI, SIG>(w, bt, colmap, rowbase, g, c1, lds, s_col, lc, out);
  }
}

template <int CLS, int SIG>
__global__ __launch_bounds__(1024) void lcs_fast_kernel(
    DeviceBatch bt, const GroupDesc* __restrict__ groups, const LaneDesc* __restrict__ lanes,
    const ItemDesc* __restrict__ items, const uint32_t* __restrict__ colmap, const uint64_t* __restrict__ rowbase,
    const StepRange* __restrict__ ranges, StepCtl* __restrict__ ctl, int32_t* __restrict__ out, uint32_t sigma) {
  constexpr int WLO = CLS == 0 ? 1 : 4 * kClassQMax[CLS > 0 ? CLS - 1 : 0] + 1;
  constexpr int WHI = 4 * kClassQMax[CLS];
  extern __shared__ uint4 lds4[];
  char* lds = reinterpret_cast<char*>(lds4);
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
    LaneCtx lc{0ull, 0xFFFFFFFFu, 0u, 0u};  // pos = max: an empty lane never stores
    uint32_t seq = 0;
    if (lane < g.nrows) {
      const LaneDesc d = lanes[g.lane_first + lane];
      lc.out_off = d.out_off;
      lc.pos = d.pos;
      lc.orig = d.orig;
      seq = d.seq;
      lc.len = bt.len[seq];
    }
    {  // stage the group's masks in LDS (zero past each row's end and in the padding)
      const uint32_t Q = (g.W + 3u) >> 2;
      const uint32_t Ws = lane < g.nrows ? (bt.len[seq] + 31u) >> 5 : 0u;
      const uint64_t mo = lane < g.nrows ? bt.mask_off[seq] : 0ull;
      const uint32_t n = Q * sigma;
      for (uint32_t e = wave; e < n; e += nwaves) {
        const uint32_t q = e / sigma, c = e - q * sigma;
        uint4 v;
        const uint32_t w0 = 4u * q;
        const uint32_t* src = bt.masks + mo + (uint64_t)c * Ws;
        v.x = w0 + 0 < Ws ? src[w0 + 0] : 0u;
        v.y = w0 + 1 < Ws ? src[w0 + 1] : 0u;
        v.z = w0 + 2 < Ws ? src[w0 + 2] : 0u;
        v.w = w0 + 3 < Ws ? src[w0 + 3] : 0u;
        *reinterpret_cast<uint4*>(lds + lds_byte<SIG>(q, c, lane)) = v;
      }
    }
    if (threadIdx.x == 0) s_col = item.c0;
    __syncthreads();
    dispatch_w<WLO, WHI, SIG>(g.W, bt, colmap, rowbase, g, item.c1, lds, &s_col, lc, out);
    __syncthreads();  // LDS and s_item are reused by the next item
  }
}

// ------------------------------------------------------------ long rows

// One segment of W dwords of a long row against a whole column.  Carries
// between segments travel as one bit per column step: the segment below
// wrote the carry out of its top dword at step t into bit 31 - (t mod 32) of
// word t / 32 of this lane's carry row; this segment consumes it as its own
// carry in and, unless it is the top segment, writes its own carry out the
// same way.  `crow` points at the lane's dword for block 0; blocks are 64
// dwords apart (one per lane), so a wave's carry traffic is coalesced.
template <int W, int SIG, int PL = SIG>
__device__ __forceinline__ void long_step(uint32_t (&V)[W], const char* __restrict__ p, uint32_t& cin, uint32_t& cout) {
  constexpr int Q = (W + 3) / 4;
  uint32_t M[4 * Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint4 x = *reinterpret_cast<const uint4*>(p + q * (PL * 1024));
    M[4 * q + 0] = x.x;
    M[4 * q + 1] = x.y;
    M[4 * q + 2] = x.z;
    M[4 * q + 3] = x.w;
  }
  uint32_t c;
  cin = __builtin_addc(cin, cin, 0u, &c);  // c = this step's carry in (the top bit); shift it out
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t U = V[w] & M[w];
    uint32_t co;
    const uint32_t S = __builtin_addc(V[w], U, c, &co);
    c = co;
    V[w] = __builtin_amdgcn_bitop3_b32(S, V[w], M[w], 0xF4);
  }
  uint32_t dummy;
  cout = __builtin_addc(cout, cout, c, &dummy);  // append this step's carry out
}

template <int W, int SIG>
__device__ __forceinline__ uint32_t long_segment(const uint4* __restrict__ B, uint32_t n, const char* __restrict__ lbase,
                                                 uint32_t* __restrict__ crow, bool has_in, bool has_out) {
  uint32_t V[W];
#pragma unroll
  for (int w = 0; w < W; ++w) V[w] = 0xFFFFFFFFu;
  const uint32_t nch = n >> 3, rem = n & 7u;
  uint32_t cin = 0, cout = 0;
  uint4 nxt = B[0];
  for (uint32_t ch = 0; ch < nch; ++ch) {
    if ((ch & 3u) == 0 && has_in) cin = crow[(uint64_t)(ch >> 2) * 64];
    const uint4 q = nxt;
    nxt = B[ch + 1];  // the spare chunk makes this read safe on the last chunk
    long_step<W, SIG>(V, lbase + (q.x & 0xFFFFu), cin, cout);
    long_step<W, SIG>(V, lbase + (q.x >> 16), cin, cout);
    long_step<W, SIG>(V, lbase + (q.y & 0xFFFFu), cin, cout);
    long_step<W, SIG>(V, lbase + (q.y >> 16), cin, cout);
    long_step<W, SIG>(V, lbase + (q.z & 0xFFFFu), cin, cout);
    long_step<W, SIG>(V, lbase + (q.z >> 16), cin, cout);
    long_step<W, SIG>(V, lbase + (q.w & 0xFFFFu), cin, cout);
    long_step<W, SIG>(V, lbase + (q.w >> 16), cin, cout);
    if ((ch & 3u) == 3u) {  // 32 steps: step 32*blk at bit 31
      if (has_out) crow[(uint64_t)(ch >> 2) * 64] = cout;
      cout = 0;
    }
  }
  if (rem) {
    if ((nch & 3u) == 0 && has_in) cin = crow[(uint64_t)(nch >> 2) * 64];
    const uint32_t qw[4] = {nxt.x, nxt.y, nxt.z, nxt.w};
#pragma unroll
    for (uint32_t t = 0; t < 7; ++t)
      if (t < rem) long_step<W, SIG>(V, lbase + ((qw[t >> 1] >> (16u * (t & 1u))) & 0xFFFFu), cin, cout);
  }
  const uint32_t tn = (nch & 3u) * 8u + rem;  // steps of the last, partial 32-step block
  if (has_out && tn) crow[(uint64_t)(nch >> 2) * 64] = cout << (32u - tn);
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) cnt += __builtin_popcount(~V[w]);
  return cnt;
}

template <int W, int WHI, int SIG>
__device__ __forceinline__ uint32_t long_segment_w(uint32_t w, const uint4* __restrict__ B, uint32_t n,
                                                   const char* __restrict__ lbase, uint32_t* __restrict__ crow,
                                                   bool has_in, bool has_out) {
  if constexpr (W <= WHI) {
    if (w == W) return long_segment<W, SIG>(B, n, lbase, crow, has_in, has_out);
    return long_segment_w<W + 1, WHI, SIG>(w, B, n, lbase, crow, has_in, has_out);
  } else {
    return 0;
  }
}

// ------------------------------------------------------------ lanes per row

// Long rows spread over L neighbouring lanes ("lanes per row" mode): lane s
// of a row holds dwords [s WL, (s + 1) WL) of its bit vector, so the carry of
// every column step crosses from lane s - 1 into lane s.  The lanes run
// skewed: at pipeline step T lane s processes the column's 32-symbol chunk
// T - s, taking that chunk's 32 carry-in bits from lane s - 1, which
// processed the same chunk at step T - 1, by one DPP wave shift of its
// carry-out word.  A lane keeps its whole segment's masks in LDS, so a
// column is one pass with no barrier and no carry traffic through memory.
//
// The LDS table has SIG + 1 planes per quad: plane SIG is all zeros, and a
// step outside the lane's part of the column (pipeline fill and drain, past
// the column's end) reads it, which leaves V unchanged and, with a zero
// carry-in, carries nothing.
template <int SIG>
__device__ __forceinline__ uint32_t skew_lds_byte(uint32_t q, uint32_t c, uint32_t lane) {
  return q * ((SIG + 1) * 1024u) + c * 1024u + lane * 16u;
}

// Lane l receives lane l - 1's value (lane 0 receives 0).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

// One column through a lanes-per-row group; returns this lane's zero bits.
// B is the column's symbol stream (16-byte chunks of 8 symbols, nsub = index
// of its spare chunk); s is the lane's segment index within its row.
template <int WL, int SIG>
__device__ __forceinline__ uint32_t skew_column(const uint4* __restrict__ B, uint32_t n, uint32_t L, uint32_t s,
                                                const char* __restrict__ lbase) {
  uint32_t V[WL];
#pragma unroll
  for (int w = 0; w < WL; ++w) V[w] = 0xFFFFFFFFu;
  const uint32_t nch = (n + 31u) >> 5;  // 32-symbol chunks
  const uint32_t nsub = (n + 7u) >> 3;
  const int32_t last = (int32_t)nch - 1;
  uint32_t cw = 0;  // carry-out bits of this lane's previous chunk
  int32_t ci = -(int32_t)s;
  uint4 nxt = B[min((uint32_t)min(max(ci, 0), max(last, 0)) * 4u, nsub)];
  for (uint32_t T = 0; T + 1 < nch + L; ++T, ++ci) {
    uint32_t cin = wave_shr1(cw);
    if (s == 0) cin = 0u;
    uint32_t cout = 0u;
    const uint32_t base = (uint32_t)min(max(ci, 0), max(last, 0)) * 4u;
    const uint32_t nbase = (uint32_t)min(max(ci + 1, 0), max(last, 0)) * 4u;
    if (T + 1 >= L && T + 1 < nch) {  // every lane's chunk exists and is full (wave-uniform)
#pragma unroll 1
      for (uint32_t x = 0; x < 4; ++x) {
        const uint4 q = nxt;
        nxt = B[x < 3 ? base + x + 1 : min(nbase, nsub)];
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.x & 0xFFFFu), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.x >> 16), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.y & 0xFFFFu), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.y >> 16), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.z & 0xFFFFu), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.z >> 16), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.w & 0xFFFFu), cin, cout);
        long_step<WL, SIG, SIG + 1>(V, lbase + (q.w >> 16), cin, cout);
      }
    } else {  // pipeline fill, drain, or the column's last chunk
#pragma unroll 1
      for (uint32_t x = 0; x < 4; ++x) {
        const uint4 q = nxt;
        nxt = B[min(x < 3 ? base + x + 1 : nbase, nsub)];
        const int32_t t0 = ci * 32 + (int32_t)(x * 8);  // symbol index of q's first symbol
        const bool on = ci >= 0;
        const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t sym = (qw[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
          long_step<WL, SIG, SIG + 1>(V, lbase + (on && t0 + k < (int32_t)n ? sym : (uint32_t)SIG * 1024u), cin,
                                      cout);
        }
      }
    }
    cw = cout;
  }
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < WL; ++w) cnt += __builtin_popcount(~V[w]);
  return cnt;
}

template <int WL, int WHI, int SIG>
__device__ __forceinline__ uint32_t skew_column_w(uint32_t wl, const uint4* __restrict__ B, uint32_t n, uint32_t L,
                                                  uint32_t s, const char* __restrict__ lbase) {
  if constexpr (WL <= WHI) {
    if (wl == WL) return skew_column<WL, SIG>(B, n, L, s, lbase);
    return skew_column_w<WL + 1, WHI, SIG>(wl, B, n, L, s, lbase);
  } else {
    return 0;
  }
}

// One work item of a lanes-per-row group: stage every lane's segment masks,
// then waves take columns from an LDS counter.
template <int SIG>
__device__ __forceinline__ void skew_item(const DeviceBatch& bt, const LaneDesc* __restrict__ lanes,
                                          const uint32_t* __restrict__ colmap, const uint64_t* __restrict__ rowbase,
                                          const GroupDesc& g, const ItemDesc& item, uint32_t sigma, char* lds,
                                          uint32_t* s_col, int32_t* __restrict__ out) {
  constexpr uint32_t WHI = SIG == 20 ? 28u : 16u;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const uint32_t L = g.lpr, WL = (g.W + L - 1u) / L;
  const uint32_t r = lane / L, s = lane - r * L;
  const bool on = r < g.nrows;
  LaneCtx lc{0ull, 0xFFFFFFFFu, 0u, 0u};
  uint32_t seq = 0;
  if (on) {
    const LaneDesc d = lanes[g.lane_first + r];
    lc.out_off = d.out_off;
    lc.pos = d.pos;
    lc.orig = d.orig;
    seq = d.seq;
    lc.len = bt.len[seq];
  }
  {  // this lane's segment of its row's masks (zero past the row's end and past the segment), and the
     // zero plane of every quad
    const uint32_t Q = (WL + 3u) >> 2;
    const uint32_t Ws = on ? (lc.len + 31u) >> 5 : 0u;
    const uint64_t mo = on ? bt.mask_off[seq] : 0ull;
    const uint32_t np = sigma + 1u;
    for (uint32_t e = wave; e < Q * np; e += nwaves) {
      const uint32_t q = e / np, c = e - q * np;
      uint32_t v[4] = {0u, 0u, 0u, 0u};
      if (c < sigma) {
        const uint32_t* src = bt.masks + mo + (uint64_t)c * Ws;
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
          const uint32_t wl = 4u * q + k, wr = s * WL + wl;
          v[k] = (wl < WL && wr < Ws) ? src[wr] : 0u;
        }
      }
      const uint32_t plane = c < sigma ? c : (uint32_t)SIG;
      *reinterpret_cast<uint4*>(lds + skew_lds_byte<SIG>(q, plane, lane)) = make_uint4(v[0], v[1], v[2], v[3]);
    }
  }
  if (threadIdx.x == 0) *s_col = item.c0;
  __syncthreads();
  const char* lbase = lds + lane * 16u;
  for (;;) {
    uint32_t col = 0;
    if (lane == 0) col = atomicAdd(s_col, 1u);
    col = __builtin_amdgcn_readfirstlane(col);
    if (col >= item.c1) break;
    uint32_t b = col;
    uint64_t rb = 0;
    if (g.colmap_base != kNoMap) {
      if (col < g.nmap) {
        b = colmap[g.colmap_base + col];
        rb = rowbase[g.rowbase_base + col];
      } else {
        b = col + g.shift;
      }
    }
    const uint32_t sc = g.fam_base + b;
    const uint32_t n = bt.len[sc];
    const uint4* B = reinterpret_cast<const uint4*>(bt.sym + bt.sym_off[sc]);
    const uint32_t cnt = skew_column_w<kSkewWLMin, WHI, SIG>(WL, B, n, L, s, lbase);
    uint32_t tot = 0;  // the row's zero bits: the sum over its L lanes
    for (uint32_t x = 0; x < L; ++x) tot += (uint32_t)__shfl((int)cnt, (int)((r * L + x) & 63u), 64);
    if (on && s == 0 && col > lc.pos) {
      const uint64_t o = lc.orig < b ? lc.out_off + (b - lc.orig - 1u) : rb + (lc.orig - b - 1u);
      out[o] = tile_value(bt.values, tot, lc.len, n);
    }
  }
  __syncthreads();  // LDS and the column counter are reused by the next item
}

// Rows whose bit vectors exceed the fast classes.  A workgroup takes a work
// item (group, columns); its waves take one column each per pass, and for
// every segment of the rows (SEGQ quads) the workgroup stages that segment's
// masks in LDS and all waves run it over their columns.  Columns of a pass
// are neighbours in length order (family mode), so the barriers between
// segments cost little.
template <int SEGQ, int SIG>
__global__ __launch_bounds__(1024) void lcs_long_kernel(
    DeviceBatch bt, const GroupDesc* __restrict__ groups, const LaneDesc* __restrict__ lanes,
    const ItemDesc* __restrict__ items, const uint32_t* __restrict__ colmap, const uint64_t* __restrict__ rowbase,
    const StepRange* __restrict__ ranges, StepCtl* __restrict__ ctl, int32_t* __restrict__ out, uint32_t sigma,
    uint32_t* __restrict__ carry, uint32_t carry_words) {
  constexpr uint32_t SEGW = 4 * SEGQ;
  extern __shared__ uint4 lds4[];
  char* lds = reinterpret_cast<char*>(lds4);
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_col;
  const uint32_t step = ctl->step;
  const uint32_t begin = ranges[step].begin[3];
  const uint32_t end = ranges[step].end[3];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t nwaves = blockDim.x >> 6;
  uint32_t* crow = carry + ((uint64_t)(blockIdx.x * nwaves + wave) * carry_words) * 64u + lane;
  const char* lbase = lds + lane * 16u;
  for (;;) {
    if (threadIdx.x == 0) s_item = begin + atomicAdd(&ctl->cursor[3], 1u);
    __syncthreads();
    const uint32_t it = s_item;
    __syncthreads();  // everyone has read s_item before it can change
    if (it >= end) break;
    const ItemDesc item = items[it];
    const GroupDesc g = groups[item.group];
    if (g.lpr) {  // lanes-per-row group (uniform for the workgroup)
      skew_item<SIG>(bt, lanes, colmap, rowbase, g, item, sigma, lds, &s_col, out);
      continue;
    }
    uint32_t pos = 0xFFFFFFFFu, orig = 0, seq = 0;
    uint64_t out_off = 0;
    if (lane < g.nrows) {
      const LaneDesc d = lanes[g.lane_first + lane];
      out_off = d.out_off;
      pos = d.pos;
      orig = d.orig;
      seq = d.seq;
    }
    const uint32_t Ws = lane < g.nrows ? (bt.len[seq] + 31u) >> 5 : 0u;
    const uint64_t mo = lane < g.nrows ? bt.mask_off[seq] : 0ull;
    const uint32_t nseg = (g.W + SEGW - 1) / SEGW;
    for (uint32_t cb = item.c0; cb < item.c1; cb += nwaves) {
      const uint32_t col = cb + wave;
      const bool valid = col < item.c1;
      uint32_t b = 0, n = 0;
      uint64_t rb = 0;
      const uint4* B = nullptr;
      if (valid) {
        b = col;
        if (g.colmap_base != kNoMap) {
          if (col < g.nmap) {
            b = colmap[g.colmap_base + col];
            rb = rowbase[g.rowbase_base + col];
          } else {
            b = col + g.shift;
          }
        }
        const uint32_t s = g.fam_base + b;
        n = bt.len[s];
        B = reinterpret_cast<const uint4*>(bt.sym + bt.sym_off[s]);
      }
      uint32_t cnt = 0;
      for (uint32_t sg = 0; sg < nseg; ++sg) {
        __syncthreads();  // the previous segment's LDS reads are done
        const uint32_t wbase = sg * SEGW;
        const uint32_t segw = min(SEGW, g.W - wbase);
        const uint32_t qn = (segw + 3u) >> 2;
        for (uint32_t e = wave; e < qn * sigma; e += nwaves) {
          const uint32_t q = e / sigma, c = e - q * sigma;
          const uint32_t w0 = wbase + 4u * q;
          const uint32_t* src = bt.masks + mo + (uint64_t)c * Ws;
          uint4 v;
          v.x = w0 + 0 < Ws ? src[w0 + 0] : 0u;
          v.y = w0 + 1 < Ws ? src[w0 + 1] : 0u;
          v.z = w0 + 2 < Ws ? src[w0 + 2] : 0u;
          v.w = w0 + 3 < Ws ? src[w0 + 3] : 0u;
          *reinterpret_cast<uint4*>(lds + lds_byte<SIG>(q, c, lane)) = v;
        }
        __syncthreads();
        if (valid) {
          const bool has_in = sg > 0, has_out = sg + 1 < nseg;
          if (segw == SEGW) cnt += long_segment<SEGW, SIG>(B, n, lbase, crow, has_in, has_out);
          else cnt += long_segment_w<1, SEGW, SIG>(segw, B, n, lbase, crow, has_in, has_out);
        }
      }
      if (valid && col > pos) {
        const uint64_t o = orig < b ? out_off + (b - orig - 1u) : rb + (orig - b - 1u);
        out[o] = tile_value(bt.values, cnt, lane < g.nrows ? bt.len[seq] : 0u, n);
      }
    }
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
    const StepCtl* __restrict__ ctl, int32_t* __restrict__ out, uint64_t* __restrict__ work, uint32_t values) {
  const uint32_t step = ctl->step;
  const uint32_t rb = ranges[step].begin[4], re = ranges[step].end[4];
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
                                    : rowbase[row.rowbase_base + col] + (row.orig - b - 1u);
    out[o] = tile_value(values, cnt, m, n);
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

template <int CLS, int SIG>
static const void* fast_fn() {
  return reinterpret_cast<const void*>(&lcs_fast_kernel<CLS, SIG>);
}

static const void* fast_kernel_ptr(int cls, uint32_t sigma) {
  const bool small = sig_cap(sigma) == 20;
  switch (cls) {
    case 0: return small ? fast_fn<0, 20>() : fast_fn<0, 32>();
    case 1: return small ? fast_fn<1, 20>() : fast_fn<1, 32>();
    default: return small ? fast_fn<2, 20>() : fast_fn<2, 32>();
  }
}

// Allow the class's dynamic LDS and report how many workgroups of `waves`
// waves fit on one CU.  Call before any launch (and before graph capture).
int fast_prepare(int cls, uint32_t sigma, uint32_t qmax, uint32_t waves, int* blocks_per_cu) {
  const size_t lds = fast_lds_bytes(sigma, qmax);
  const void* fn = fast_kernel_ptr(cls, sigma);
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, fn);
  if (e != hipSuccess) return (int)e;
  if (fa.sharedSizeBytes > kLdsReserve || lds + kLdsReserve > g_max_lds) return (int)hipErrorInvalidValue;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(g_max_lds - fa.sharedSizeBytes));
  if (e != hipSuccess) return (int)e;
  int nb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)(waves * 64), lds);
  if (e != hipSuccess) return (int)e;
  if (blocks_per_cu) *blocks_per_cu = nb;
  return 0;
}

int launch_fast(int cls, const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t sigma,
                uint32_t qmax, uint32_t blocks, uint32_t waves, void* stream) {
  const size_t lds = fast_lds_bytes(sigma, qmax);
  const dim3 grid(blocks), block(waves * 64);
  const bool small = sig_cap(sigma) == 20;
#define FAMSA_FAST(C, S)                                                                                       \
  hipLaunchKernelGGL((lcs_fast_kernel<C, S>), grid, block, lds, (hipStream_t)stream, b, w.groups, w.lanes,     \
                     w.items, w.colmap, w.rowbase, w.ranges, ctl, out, sigma)
  switch (cls) {
    case 0: if (small) FAMSA_FAST(0, 20); else FAMSA_FAST(0, 32); break;
    case 1: if (small) FAMSA_FAST(1, 20); else FAMSA_FAST(1, 32); break;
    default: if (small) FAMSA_FAST(2, 20); else FAMSA_FAST(2, 32); break;
  }
#undef FAMSA_FAST
  return hip_ok(hipGetLastError());
}

template <int SQ, int SIG>
static const void* long_fn() {
  return reinterpret_cast<const void*>(&lcs_long_kernel<SQ, SIG>);
}

static const void* long_kernel_ptr(uint32_t sigma) {
  return sig_cap(sigma) == 20 ? long_fn<kLongSegQ[0], 20>() : long_fn<kLongSegQ[1], 32>();
}

int long_prepare(uint32_t sigma, uint32_t waves, int* blocks_per_cu) {
  const size_t lds = long_lds_bytes(sigma);
  const void* fn = long_kernel_ptr(sigma);
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, fn);
  if (e != hipSuccess) return (int)e;
  if (fa.sharedSizeBytes > kLdsReserve || lds + kLdsReserve > g_max_lds) return (int)hipErrorInvalidValue;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(g_max_lds - fa.sharedSizeBytes));
  if (e != hipSuccess) return (int)e;
  int nb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)(waves * 64), lds);
  if (e != hipSuccess) return (int)e;
  if (blocks_per_cu) *blocks_per_cu = nb;
  return 0;
}

int launch_long(const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t sigma,
                uint32_t* carry, uint32_t carry_words, uint32_t blocks, uint32_t waves, void* stream) {
  const size_t lds = long_lds_bytes(sigma);
  const dim3 grid(blocks), block(waves * 64);
  if (sig_cap(sigma) == 20)
    hipLaunchKernelGGL((lcs_long_kernel<kLongSegQ[0], 20>), grid, block, lds, (hipStream_t)stream, b, w.groups,
                       w.lanes, w.items, w.colmap, w.rowbase, w.ranges, ctl, out, sigma, carry, carry_words);
  else
    hipLaunchKernelGGL((lcs_long_kernel<kLongSegQ[1], 32>), grid, block, lds, (hipStream_t)stream, b, w.groups,
                       w.lanes, w.items, w.colmap, w.rowbase, w.ranges, ctl, out, sigma, carry, carry_words);
  return hip_ok(hipGetLastError());
}

uint32_t plain_register_w64_limit() { return 40; }

int launch_plain(const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t w64_max,
                 uint32_t blocks, uint64_t* d_work, void* stream) {
  const dim3 grid(blocks), block(kPlainBlock);
  hipStream_t s = (hipStream_t)stream;
#define FAMSA_PLAIN(WW)                                                                                        \
  hipLaunchKernelGGL(lcs_plain_kernel<WW>, grid, block, 0, s, b.codes, b.dev_off, b.len, b.mask_off, b.masks, \
                     w.prows, w.colmap, w.rowbase, w.ranges, ctl, out, d_work, b.values)
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
