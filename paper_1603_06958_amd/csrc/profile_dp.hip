// Aligning one sequence to a profile on gfx950: the specialised dynamic
// programming the progressive stage runs when one side of a merge is a
// single sequence (Methods, "Progressive construction of the alignment"),
// with the affine terminal / non-terminal gap costs and the gap-type
// corrections of "Gap types and costs determination".
//
// A batch holds independent problems (the alignments of one level of the
// guide tree).  Per problem, from the profile's K gapped rows of width n:
//   pdp_rows_kernel -- a wave per row: the columns of its first and last
//                      residue (ballots over 256 columns at a time);
//   pdp_cols_kernel -- a thread per column j: the profile's per-column
//                      symbol counters (LDS histogram over the rows), the
//                      column-to-symbol cost table cost[a][j] = sum_x
//                      count[j][x] S[x][a] and w_j = residues in column j; a
//                      thread per boundary p: the cost of the first and of
//                      each further gap column inserted into the profile
//                      there, from the counts of rows in each of the four
//                      situations (terminal or inside, next to a gap or
//                      opening one);
//   pdp_dp_kernel   -- a workgroup of up to sixteen waves per problem (four
//                      on levels of four problems or more per CU): the
//                      three-state DP
//                        M(i,j) = best(i-1,j-1) + cost[a_i][j]
//                        D(i,j) = max(M - o w_j, I - o w_j, D - e w_j)(i,j-1)
//                        I(i,j) = max(M - f_j, D - f_j, I - x_j)(i-1,j)
//                      over strips of 64 rows (a lane per row), each strip
//                      swept along anti-diagonals: at step t lane l does
//                      column t - l, takes the cell above from lane l - 1
//                      (and lane 0 from the strip above's last row, an edge
//                      row), and records the three choices of each cell in
//                      one byte; consecutive strips run on different waves,
//                      each a fixed number of steps behind the strip above,
//                      in phases separated by barriers; then the alignment is
//                      traced back from (m, n) by one wave, the choices
//                      staged in LDS 4 KB at a time and decoded, an 8 x 8
//                      block of cells at a time, into a per-lane table of
//                      next states (a step is one cross-lane read).
// The DP reads the per-column records, the cost table and the edge rows from
// LDS when the problem's share fits (it is copied in first), else from
// global memory.  Ties take the first maximum in the order written (M, D, I),
// as a fixed rule, so the alignment and not only its score is unique.  The
// DP runs in int32 when every value fits 28 bits, else in int64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "runtime.h"

namespace famsa {
namespace {

constexpr uint8_t kGap = FAMSA_PROFILE_GAP;
double g_profile_dp_ms = 0;  // duration of the last batch's DP launch

struct PdpProb {        // one problem's offsets into the batch arrays
  uint64_t seq;         // seqs (bytes)
  uint64_t rows;        // rows (bytes), K rows of n
  uint64_t cost;        // cost (int32), sigma x max(n, 1)
  uint64_t col;         // rec (records, n + 1)
  uint64_t rowx;        // first, last (int32, K)
  uint64_t edge;        // edge (records, 2 buffers of n + 1)
  uint64_t dir;         // dir (bytes): row 0, then strips of (n + 64) x 64
  uint64_t ops;         // ops (bytes), m + n
  uint32_t m, n, K;
  uint32_t narrow;      // 1: every DP value fits 28 bits, so the DP runs in int32
  uint32_t idx;         // the problem's place in the caller's batch (launch order is largest first)
  uint32_t lds;         // 1: the DP reads its records, costs and edge rows from LDS
  uint32_t cost16;      // 1: every cost fits int16 (K max|S| < 2^15), so LDS holds them as int16
  uint32_t pad;
};

// Four values of one column or boundary.  Column record j (0..n):
// w_j (residues in column j, 1-based; 0 for j = 0), f_j and x_j (the costs
// of a first and a further gap column inserted at boundary j), 0.  Edge
// record j: M, D, I of the strip's last row at column j.
template <typename E>
struct alignas(4 * sizeof(E)) PdpRec {
  E v[4];
};

struct PdpArrays {
  const uint8_t* seqs;
  const uint8_t* rows;
  int32_t* cost;
  PdpRec<int64_t>* rec;
  int32_t* first;
  int32_t* last;
  PdpRec<int64_t>* edge;
  uint8_t* dir;
  uint8_t* ops;
  int64_t* score;
  uint32_t* nops;
  int64_t To, Te, Go, Ge;  // gap costs: terminal open / extend, inside open / extend
  uint32_t tb_cap;         // bytes of dynamic LDS every DP workgroup has (its trace-back gathers ops there)
};

template <typename T>
__device__ __forceinline__ int argmax3(T x0, T x1, T x2, T* best) {
  int k = 0;
  T b = x0;
  if (x1 > b) { b = x1; k = 1; }
  if (x2 > b) { b = x2; k = 2; }
  *best = b;
  return k;
}

// A wave per row: first and last column holding a residue (n and -1 if
// none).  Block (p, y) takes the rows 16 y' .. 16 y' + 15 of problem p for
// y' = y, y + gridDim.y, ..., four per wave; a wave reads 256 columns of a
// row at a time (four loads in flight per lane).
constexpr uint32_t kRowsPerBlock = 16;

__global__ __launch_bounds__(256) void pdp_rows_kernel(const PdpProb* __restrict__ probs, PdpArrays A) {
  const PdpProb P = probs[blockIdx.x];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (uint32_t y = blockIdx.y; y * kRowsPerBlock < P.K; y += gridDim.y) {
    const uint32_t s1 = min(P.K, (y + 1) * kRowsPerBlock);
    for (uint32_t s = y * kRowsPerBlock + wave; s < s1; s += nw) {  // wave-uniform: the ballots see every lane
      const uint8_t* row = A.rows + P.rows + (uint64_t)s * P.n;
      int32_t f = (int32_t)P.n, l = -1;
      for (uint32_t c0 = 0; c0 < P.n; c0 += 256) {
        uint32_t x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t c = c0 + 64u * u + lane;
          const uint32_t b = row[std::min(c, P.n - 1)];  // unconditional, so the four loads are in flight together
          x[u] = c < P.n ? b : kGap;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint64_t b = __ballot(x[u] != kGap);
          if (b) {
            const uint32_t base = c0 + 64u * u;
            if (f == (int32_t)P.n) f = (int32_t)(base + __builtin_ctzll(b));
            l = (int32_t)(base + 63 - __builtin_clzll(b));
          }
        }
      }
      if (lane == 0) {
        A.first[P.rowx + s] = f;
        A.last[P.rowx + s] = l;
      }
    }
  }
}

// blockIdx.y picks 256 columns (boundaries) of problem blockIdx.x.  Dynamic
// LDS: the symbol counters hist[x][thread] (sigma x 256) and the sigma x
// sigma scores, sized by the alphabet so that more workgroups share a CU.
__global__ __launch_bounds__(256) void pdp_cols_kernel(const PdpProb* __restrict__ probs, PdpArrays A,
                                                       const int32_t* __restrict__ subst, uint32_t sigma) {
  extern __shared__ uint32_t pdp_cols_lds[];
  uint32_t (*hist)[256] = reinterpret_cast<uint32_t (*)[256]>(pdp_cols_lds);
  int32_t* S = reinterpret_cast<int32_t*>(pdp_cols_lds + sigma * 256u);
  const PdpProb P = probs[blockIdx.x];
  const uint32_t tid = threadIdx.x;
  const uint32_t j = blockIdx.y * 256u + tid;  // column j (0-based) and boundary p = j
  if (blockIdx.y * 256u > P.n) return;          // whole block past the last boundary
  for (uint32_t e = tid; e < sigma * sigma; e += 256) S[e] = subst[e];
  for (uint32_t x = 0; x < sigma; ++x) hist[x][tid] = 0;
  __syncthreads();
  if (j > P.n) return;
  // a problem without columns reads the rows part's first byte (always
  // allocated) and uses none of it
  const uint8_t* rows = P.n ? A.rows + P.rows : A.rows;
  const uint32_t jr = P.n ? std::min(j, P.n - 1) : 0, jl = j >= 1 ? j - 1 : 0;  // in-bounds columns
  uint32_t cTA = 0, cTO = 0, cIA = 0, cIO = 0;  // boundary situations: terminal/inside x next to a gap/opening
  // eight rows at a time; every load is unconditional (rows past K read row
  // K - 1), so that the eight rows' loads are in flight together
  constexpr uint32_t kU = 8;
  for (uint32_t s0 = 0; s0 < P.K; s0 += kU) {
    uint32_t xr[kU], xl[kU];
    int32_t fr[kU], lr[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) {
      const uint32_t s = std::min(s0 + u, P.K - 1);
      const uint8_t* row = rows + (uint64_t)s * P.n;
      const uint32_t br = row[jr], bl = row[jl];
      xr[u] = j < P.n ? br : kGap;
      xl[u] = j >= 1 ? bl : 0u;
      fr[u] = A.first[P.rowx + s];
      lr[u] = A.last[P.rowx + s];
    }
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) {
      if (s0 + u >= P.K) break;
      const uint32_t x = xr[u];
      if (x != kGap)  // an LDS add whose result is not read: no wait on it
        __hip_atomic_fetch_add(&hist[x][tid], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      const bool gap_right = j < P.n && x == kGap;
      const bool gap_left = j >= 1 && xl[u] == kGap;
      const bool inside = fr[u] < (int32_t)j && lr[u] >= (int32_t)j;  // residues on both sides of the boundary
      const bool adj = gap_left || gap_right;
      if (inside) { if (adj) ++cIA; else ++cIO; }
      else { if (adj) ++cTA; else ++cTO; }
    }
  }
  PdpRec<int64_t>* rec = A.rec + P.col;
  rec[j].v[1] = (int64_t)cTA * A.Te + (int64_t)cTO * A.To + (int64_t)cIA * A.Ge + (int64_t)cIO * A.Go;
  rec[j].v[2] = (int64_t)(cTA + cTO) * A.Te + (int64_t)(cIA + cIO) * A.Ge;
  rec[j].v[3] = 0;
  if (j == 0) rec[0].v[0] = 0;
  if (j == P.n) return;
  int32_t wj = 0;
  for (uint32_t x = 0; x < sigma; ++x) wj += (int32_t)hist[x][tid];
  rec[j + 1].v[0] = wj;  // 1-based column j + 1
  for (uint32_t a = 0; a < sigma; ++a) {
    int32_t c = 0;
    for (uint32_t x = 0; x < sigma; ++x) c += (int32_t)hist[x][tid] * S[x * sigma + a];
    A.cost[P.cost + (uint64_t)a * P.n + j] = c;
  }
}

// Lane l receives lane l - 1's value and lane 0 receives `in` (DPP wave
// shift right by one: the lane without a source keeps the old value).
__device__ __forceinline__ int32_t shr1(int32_t v, int32_t in) {
  return __builtin_amdgcn_update_dpp(in, v, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}
__device__ __forceinline__ int64_t shr1(int64_t v, int64_t in) {
  const int lo = (int)(uint32_t)(uint64_t)v, hi = (int)(uint32_t)((uint64_t)v >> 32);
  const int ilo = (int)(uint32_t)(uint64_t)in, ihi = (int)(uint32_t)((uint64_t)in >> 32);
  const uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(ilo, lo, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
  const uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(ihi, hi, 0x138, 0xF, 0xF, false);
  return (int64_t)(((uint64_t)b << 32) | a);
}

__device__ __forceinline__ int64_t shfl_up64(int64_t v, int d) {
  const int32_t lo = __shfl_up((int32_t)(uint32_t)(uint64_t)v, d, 64);
  const int32_t hi = __shfl_up((int32_t)(uint32_t)((uint64_t)v >> 32), d, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Products of a residue count (< 2^21) and a gap cost (|c| <= 2^20): the
// 24-bit multiply is exact for them and full rate in int32.
__device__ __forceinline__ int32_t wmul(int32_t w, int32_t c) { return __mul24(w, c); }
__device__ __forceinline__ int64_t wmul(int64_t w, int64_t c) { return w * c; }

// Region of a problem's choice bytes: row 0 (rounded up to 64 bytes), then
// per strip of 64 rows (n + 64) steps x 64 lanes.  Cell (i, j), i >= 1, is
// byte t * 64 + l of strip (i - 1) / 64, with l = (i - 1) mod 64, t = j + l.
__host__ __device__ inline uint64_t pdp_row0_bytes(uint32_t n) { return ((uint64_t)n + 1 + 63) & ~(uint64_t)63; }
__host__ __device__ inline uint64_t pdp_strip_bytes(uint32_t n) { return ((uint64_t)n + 64) * 64; }
__host__ __device__ inline uint64_t pdp_dir_bytes(uint32_t m, uint32_t n) {
  return pdp_row0_bytes(n) + (uint64_t)((m + 63) / 64) * pdp_strip_bytes(n);
}

__device__ __forceinline__ int64_t bcast64(int64_t v, uint32_t src) {
  const int32_t lo = __shfl((int32_t)(uint32_t)(uint64_t)v, (int)src, 64);
  const int32_t hi = __shfl((int32_t)(uint32_t)((uint64_t)v >> 32), (int)src, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Phases.  A problem's sweep of n + 64 steps per strip is cut into Q chunks
// of kPdpChunk steps; strip s runs chunk q in phase start(s) + q on wave
// s mod nw, and every phase ends at a barrier.  Lane 0 of strip s + 1 reads
// the edge record of column t one step before its step t; lane 63 of strip
// s writes it at its step t + 63, at most 64 / kPdpChunk phases later in the
// strip's own chunks, so strips kPdpLag = 1 + 64 / kPdpChunk phases apart
// always find it written in an earlier phase.  A wave's strips are
// Period = max(Q, nw kPdpLag) phases apart:
//   start(s) = (s mod nw) kPdpLag + (s / nw) Period,
// which keeps consecutive strips at least kPdpLag phases apart and a wave's
// strips from overlapping.  Strip s writes edge buffer s mod 2 and reads
// buffer (s + 1) mod 2 (row 0 is buffer 1): strip s + 2 rewrites a column of
// buffer s mod 2 in a later phase than the one in which strip s + 1 read it.
constexpr uint32_t kPdpWaves = 16;
constexpr uint32_t kPdpChunk = 16;
constexpr uint32_t kPdpLag = 1 + (64 + kPdpChunk - 1) / kPdpChunk;

__host__ __device__ inline uint32_t pdp_waves(uint32_t m, uint32_t n) {
  const uint32_t S = (m + 63) / 64, Q = (n + 64 + kPdpChunk - 1) / kPdpChunk;
  const uint32_t want = (Q + kPdpLag - 1) / kPdpLag;  // more waves than this would wait for their strips
  return std::max(1u, std::min(kPdpWaves, std::min(S, want)));
}

// The unreachable value of each value type: far enough below every reachable
// value (|value| < 2^28 for int32, < 2^58 for int64 within the input limits)
// that subtracting a cost from it never overflows or wins a maximum.
template <typename T>
__host__ __device__ constexpr T pdp_neg();
template <>
__host__ __device__ constexpr int32_t pdp_neg<int32_t>() { return INT32_MIN / 4; }
template <>
__host__ __device__ constexpr int64_t pdp_neg<int64_t>() { return INT64_MIN / 4; }

// One problem's DP inputs as the strips read them: in LDS (E = T, costs
// int32 or int16) or in global memory (E = int64, costs int32).
template <typename E, typename C>
struct PdpView {
  const PdpRec<E>* rec;  // n + 1 column records
  const C* cost;         // sigma rows of max(n, 1)
  PdpRec<E>* edge;       // two buffers of n + 1
};

// Edge rows keep kPdpPad unused records before column 0 and after column n:
// over a sweep the writing lane's column runs from -63 to n + 63 and lane 0
// reads up to column n + 64, so neither needs a bounds check.  Column j of
// buffer b is record b * pdp_edge_cols(n) + kPdpPad + j.
constexpr uint32_t kPdpPad = 64;
__host__ __device__ inline uint64_t pdp_edge_cols(uint32_t n) { return (uint64_t)n + 1 + 2 * kPdpPad; }

// LDS bytes a problem needs for its records, costs and edge rows.
__host__ __device__ inline uint64_t pdp_lds_bytes(uint32_t n, uint32_t sigma, uint32_t value_bytes,
                                                  uint32_t cost_bytes) {
  return 16ull * value_bytes / 4 * ((n + 1) + 2 * pdp_edge_cols(n)) +
         (uint64_t)cost_bytes * sigma * std::max(n, 1u);
}

// Wrapping int arithmetic: lanes outside the matrix run the same steps on
// values that are never used, and those may leave the range.
__device__ __forceinline__ int32_t wadd(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
__device__ __forceinline__ int32_t wsub(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }
__device__ __forceinline__ int64_t wadd(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
__device__ __forceinline__ int64_t wsub(int64_t a, int64_t b) { return (int64_t)((uint64_t)a - (uint64_t)b); }

// argmax3(a - s, b - s, c) with one subtraction: a - s and b - s compare as
// a and b (no reachable value is near the ends of the range), so the larger
// of a and b is taken first.
template <typename T>
__device__ __forceinline__ int argmax3_sub(T a, T b, T s, T c, T* best) {
  const int k1 = b > a ? 1 : 0;
  const T b01 = wsub(max(a, b), s);
  const bool k2 = c > b01;
  *best = k2 ? c : b01;
  return k2 ? 2 : k1;
}

// Row 0 (wave 0): gaps in the sequence before its first residue (terminal
// costs).  M(0,0) = 0 and D(0,1) comes from it; D(0,j), j >= 2, extends
// D(0,j-1); every other candidate starts from the unreachable value, far
// below any reachable one within the library's input limits, so row 0 is a
// prefix sum, taken 64 columns at a time across the lanes.  Written to edge
// buffer 1.
template <typename T, typename E, typename C>
__device__ void pdp_row0(const PdpProb& P, const PdpArrays& A, const PdpView<E, C>& V, uint8_t* dir,
                         int64_t* s_fin) {
  const uint32_t lane = threadIdx.x & 63u, n = P.n;
  constexpr T neg = pdp_neg<T>();
  PdpRec<E>* edge = V.edge + pdp_edge_cols(n) + kPdpPad;
  int64_t carry = 0;  // D(0, base - 1)
  for (uint32_t base = 0; base <= n; base += 64) {
    const uint32_t j = base + lane;
    int64_t x = 0;
    if (j >= 1 && j <= n) x = -(int64_t)V.rec[j].v[0] * (j == 1 ? A.To : A.Te);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = shfl_up64(x, d);
      if ((int)lane >= d) x += y;
    }
    const int64_t Dj = carry + x;
    if (j <= n) {
      const int64_t M0 = j == 0 ? 0 : (int64_t)neg, D0 = j == 0 ? (int64_t)neg : Dj;
      PdpRec<E> r;
      r.v[0] = (E)M0;
      r.v[1] = (E)D0;
      r.v[2] = (E)neg;
      r.v[3] = 0;
      edge[j] = r;
      dir[j] = (uint8_t)(j == 0 ? 0u : (1u | ((j == 1 ? 0u : 2u) << 2)));
      if (P.m == 0 && j == n) {  // the cell (0, n) ends the alignment
        s_fin[0] = M0;
        s_fin[1] = D0;
        s_fin[2] = (int64_t)neg;
      }
    }
    carry = bcast64(Dj, 63);
  }
}

// The strips of one problem in value type T; phases as described above.
template <typename T, typename E, typename C>
__device__ void pdp_strips(const PdpProb& P, const PdpArrays& A, const PdpView<E, C>& V, uint32_t nw,
                           int64_t* s_fin) {
  constexpr T neg = pdp_neg<T>();
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, m = P.m, n = P.n;
  const uint32_t S = (m + 63u) >> 6;
  const int32_t nm1 = (int32_t)std::max(n, 1u) - 1;
  uint8_t* strips = A.dir + P.dir + pdp_row0_bytes(n);
  const uint32_t steps = n + 64;
  const uint32_t Q = (steps + kPdpChunk - 1) / kPdpChunk;
  const uint32_t period = std::max(Q, nw * kPdpLag);
  const uint32_t last = S ? ((S - 1) % nw) * kPdpLag + ((S - 1) / nw) * period : 0;
  const uint32_t nphase = S ? last + Q : 0;
  const uint32_t w0 = wave * kPdpLag;  // this wave's first phase
  // this wave's current strip
  T Mc = neg, Dc = neg, Ic = neg, diag = neg, Oc = 0, Ec = 0;
  bool writes_edge = false;
  const C* crow = V.cost;
  const PdpRec<E>* ein = V.edge;
  PdpRec<E>* eout = V.edge;   // this lane's column-0 record when it writes edges
  uint8_t* dstrip = strips;
  // what one step reads: this lane's cost, w, f and x at its column and the
  // edge record lane 0 needs
  struct Col {
    C cost;  // widened where it is used, so that no step waits for the load it has just issued
    T w, f, x, eM, eD, eI;
  };
  // the values at column jj (clamped: a lane outside the matrix reads a valid
  // record) and the edge record at column je, 0 <= je <= n + 64
  auto fetch = [&](int32_t jj, uint32_t je) {
    // (a negative column, as unsigned, clamps to the top)
    const uint32_t jc = min((uint32_t)jj, n), jm = min((uint32_t)(jj - 1), (uint32_t)nm1);
    const PdpRec<E> r = V.rec[jc];
    const PdpRec<E> x = ein[je];
    return Col{crow[jm], (T)r.v[0], (T)r.v[1], (T)r.v[2], (T)x.v[0], (T)x.v[1], (T)x.v[2]};
  };
  // Every lane runs every step.  A lane before its column 0, past column n or
  // below row m computes values nothing valid reads: its choice byte lands in
  // a part of the strip the trace-back never visits, and the cell above of a
  // valid cell is always valid.  At column 0 M and D are unreachable, so the
  // values before column 0 do not reach it.
  auto step = [&](uint32_t t, const Col& c) {
    const T Mu = shr1(Mc, c.eM), Du = shr1(Dc, c.eD), Iu = shr1(Ic, c.eI);
    const bool j1 = t >= lane + 1;  // column t - lane >= 1
    const T o = wmul(c.w, Oc), e = wmul(c.w, Ec);
    T D1, I, b;
    const int ds = argmax3_sub(Mc, Ic, o, wsub(Dc, e), &D1);
    const int is = argmax3_sub(Mu, Du, c.f, wsub(Iu, c.x), &I);
    const T M = j1 ? wadd(diag, (T)c.cost) : neg;
    const T D = j1 ? D1 : neg;
    const int bk = argmax3(M, D, I, &b);
    dstrip[(uint64_t)t * 64] = (uint8_t)(bk | (ds << 2) | (is << 4));
    diag = max(max(Mu, Du), Iu);  // the cell above is the next column's diagonal
    Mc = M;
    Dc = D;
    Ic = I;
    if (writes_edge) {
      PdpRec<E> rr;
      rr.v[0] = (E)M;
      rr.v[1] = (E)D;
      rr.v[2] = (E)I;
      rr.v[3] = 0;
      eout[t] = rr;
    }
  };
  Col cur{};  // the next step's values, loaded one step ahead
  for (uint32_t p = 0; p < nphase; ++p) {
    if (p >= w0) {
      const uint32_t r = (p - w0) / period, q = p - w0 - r * period, s = wave + r * nw;
      if (s < S && q < Q) {
        if (q == 0) {  // a new strip
          const uint32_t i = 64 * s + 1 + lane;
          const bool terminal = i == m;  // gaps after the sequence's last residue
          Oc = (T)(terminal ? A.To : A.Go);
          Ec = (T)(terminal ? A.Te : A.Ge);
          const uint32_t a = i <= m ? A.seqs[P.seq + i - 1] : 0u;
          crow = V.cost + (uint64_t)a * (nm1 + 1);
          // the last row of the strip writes its edge row; the last strip's
          // row m writes one too, from which the final cell is read
          writes_edge = lane == (s + 1 < S ? 63u : (m - 1) & 63u);
          ein = V.edge + ((s + 1) & 1u) * pdp_edge_cols(n) + kPdpPad;
          eout = V.edge + (s & 1u) * pdp_edge_cols(n) + kPdpPad - lane;
          dstrip = strips + (uint64_t)s * pdp_strip_bytes(n) + lane;
          Mc = Dc = Ic = diag = neg;
          cur = fetch(-(int32_t)lane, 0);
        }
        const uint32_t t1 = min((q + 1) * kPdpChunk, steps);
        uint32_t t = q * kPdpChunk;
        // two steps per iteration, the loads alternating between two sets of
        // registers, so that no step waits for the load it has just issued
        for (; t + 1 < t1; t += 2) {
          const Col nx = fetch((int32_t)(t + 1) - (int32_t)lane, t + 1);
          step(t, cur);
          cur = fetch((int32_t)(t + 2) - (int32_t)lane, t + 2);
          step(t + 1, nx);
        }
        if (t < t1) {
          const Col nx = fetch((int32_t)(t + 1) - (int32_t)lane, t + 1);
          step(t, cur);
          cur = nx;
        }
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  if (S && threadIdx.x == 0) {  // the cell (m, n), from the last strip's edge row
    const PdpRec<E> f = V.edge[((S - 1) & 1u) * pdp_edge_cols(n) + kPdpPad + n];
    s_fin[0] = (int64_t)(T)f.v[0];
    s_fin[1] = (int64_t)(T)f.v[1];
    s_fin[2] = (int64_t)(T)f.v[2];
  }
  __syncthreads();
}

template <typename T, typename E, typename C>
__device__ void pdp_dp(const PdpProb& P, const PdpArrays& A, const PdpView<E, C>& V, uint8_t* dir, uint32_t nw,
                       int64_t* s_fin) {
  if ((threadIdx.x >> 6) == 0) pdp_row0<T, E, C>(P, A, V, dir, s_fin);
  __threadfence_block();
  __syncthreads();
  pdp_strips<T, E, C>(P, A, V, nw, s_fin);
}

// Copy one problem's records (as T) and cost table into LDS; edge rows are
// written there by the DP itself.
template <typename T, typename C>
__device__ PdpView<T, C> pdp_stage(const PdpProb& P, const PdpArrays& A, char* lds, uint32_t sigma) {
  const uint32_t n = P.n, n1 = std::max(n, 1u);
  PdpRec<T>* rec = reinterpret_cast<PdpRec<T>*>(lds);
  PdpRec<T>* edge = rec + (n + 1);
  C* cost = reinterpret_cast<C*>(edge + 2 * pdp_edge_cols(n));
  const PdpRec<int64_t>* g = A.rec + P.col;
  for (uint32_t j = threadIdx.x; j <= n; j += blockDim.x) {
    const PdpRec<int64_t> x = g[j];
    PdpRec<T> y;
    y.v[0] = (T)x.v[0];
    y.v[1] = (T)x.v[1];
    y.v[2] = (T)x.v[2];
    y.v[3] = 0;
    rec[j] = y;
  }
  const int32_t* gc = A.cost + P.cost;
  for (uint32_t e = threadIdx.x; e < sigma * n1; e += blockDim.x) cost[e] = (C)gc[e];
  return PdpView<T, C>{rec, cost, edge};
}

// A fence on LDS accesses alone: it orders them for the compiler and waits
// for no global access in flight.
constexpr uint64_t kTbMinLds = 4096;  // walks of up to 4096 ops stay in LDS
__device__ inline void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup", "local"); }

__global__ __launch_bounds__(64 * kPdpWaves) void pdp_dp_kernel(const PdpProb* __restrict__ probs, PdpArrays A,
                                                                 uint32_t sigma) {
  extern __shared__ uint4 pdp_lds4[];
  __shared__ uint4 stage4[256];  // 4 KB window of choice bytes
  __shared__ int64_t s_fin[3];
  char* lds = reinterpret_cast<char*>(pdp_lds4);
  const uint8_t* stage = reinterpret_cast<const uint8_t*>(stage4);
  const PdpProb P = probs[blockIdx.x];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, m = P.m, n = P.n;
  const uint32_t nw = std::min(pdp_waves(m, n), (uint32_t)(blockDim.x >> 6));
  uint8_t* dir = A.dir + P.dir;
  uint8_t* strips = dir + pdp_row0_bytes(n);
  if (P.lds) {  // every wave helps staging; the waves the DP does not use then leave
    if (P.narrow && P.cost16) {
      const PdpView<int32_t, int16_t> V = pdp_stage<int32_t, int16_t>(P, A, lds, sigma);
      __syncthreads();
      if (wave >= nw) return;
      pdp_dp<int32_t, int32_t, int16_t>(P, A, V, dir, nw, s_fin);
    } else if (P.narrow) {
      const PdpView<int32_t, int32_t> V = pdp_stage<int32_t, int32_t>(P, A, lds, sigma);
      __syncthreads();
      if (wave >= nw) return;
      pdp_dp<int32_t, int32_t, int32_t>(P, A, V, dir, nw, s_fin);
    } else {
      const PdpView<int64_t, int32_t> V = pdp_stage<int64_t, int32_t>(P, A, lds, sigma);
      __syncthreads();
      if (wave >= nw) return;
      pdp_dp<int64_t, int64_t, int32_t>(P, A, V, dir, nw, s_fin);
    }
  } else {
    if (wave >= nw) return;  // barriers wait for the waves that remain
    const PdpView<int64_t, int32_t> V{A.rec + P.col, A.cost + P.cost, A.edge + P.edge};
    if (P.narrow) pdp_dp<int32_t, int64_t, int32_t>(P, A, V, dir, nw, s_fin);
    else pdp_dp<int64_t, int64_t, int32_t>(P, A, V, dir, nw, s_fin);
  }
  if (wave != 0) return;  // wave 0 traces back alone
  const int64_t fM = s_fin[0], fD = s_fin[1], fI = s_fin[2];
  int64_t best;
  // Trace back, by wave 0 alone; every walk variable is wave-uniform (it
  // runs on the scalar unit). The choice bytes come through a 4 KB LDS
  // window, and the window the walk is expected to need next is loaded into
  // registers while it walks the current one. Inside a strip the walk goes
  // through a table: lane (a, b) takes the cell a rows up and b columns
  // left of the walk's cell, and decodes for each state arriving there the
  // next state and the lane the next step reads, so that a step is one
  // cross-lane read. Steps the table does not cover (edges of the 8 x 8
  // block, of a strip or of the window, row 0, column 0) read the window
  // byte by byte. Ops are gathered in one register (a lane per op), then in
  // the dynamic LDS, which the DP no longer needs, and written out reversed
  // at the end; a walk longer than that buffer puts the rest in the output
  // and reverses it there.
  int st = __builtin_amdgcn_readfirstlane(argmax3(fM, fD, fI, &best));
  uint8_t* ops = A.ops + P.ops;
  uint8_t* ops_lds = reinterpret_cast<uint8_t*>(pdp_lds4);
  const uint32_t cap = A.tb_cap;
  uint32_t i = m, j = n;
  uint32_t k0 = 0, kk = 0;  // ops stored, ops in acc
  int acc = 0;              // lane l: op k0 + l
  int win = -2;             // window in LDS: region (-1 row 0, s >= 0 strip s)
  uint32_t wlo = 0;         // and its first byte in the region (a strip is under 2^22 bytes)
  int pwin = -2;            // window in p0..p3
  uint32_t plo = 0;
  uint4 p0 = {}, p1 = {}, p2 = {}, p3 = {};
  auto fetch = [&](int region, uint32_t lo) {
    const uint8_t* base = region < 0 ? dir : strips + (uint64_t)region * pdp_strip_bytes(n);
    const uint64_t size = region < 0 ? pdp_row0_bytes(n) : pdp_strip_bytes(n);
    // lanes past the region's end load its first bytes (never read): no
    // divergent branch, so the window's bounds stay in scalar registers
    const uint64_t off = lo + (uint64_t)lane * 64;
    const uint4* src = reinterpret_cast<const uint4*>(base + (off < size ? off : 0));
    p0 = src[0];
    p1 = src[1];
    p2 = src[2];
    p3 = src[3];
  };
  // make the LDS window hold byte idx of region, the byte of cell (ci, cj)
  auto window = [&](int region, uint32_t idx, uint32_t ci, uint32_t cj) {
    if (region == win && idx >= wlo && idx < wlo + 4096) return;
    if (region != pwin || idx < plo || idx >= plo + 4096) {  // not the window loaded ahead
      pwin = region;
      plo = idx >= 4032 ? ((idx - 4032) & ~63u) : 0;
      fetch(pwin, plo);
    }
    lds_fence();  // the old window's reads are done
    stage4[lane * 4 + 0] = p0;
    stage4[lane * 4 + 1] = p1;
    stage4[lane * 4 + 2] = p2;
    stage4[lane * 4 + 3] = p3;
    lds_fence();
    win = pwin;
    wlo = plo;
    // load ahead: the next lower window of this region, or, if the walk is
    // expected to leave the region within this window (a diagonal walk from
    // row r of a strip leaves it near diagonal cj - r), the next region's
    // window around where it would enter
    const uint32_t down = wlo > 3968 ? wlo - 3968 : 0;  // overlaps this window by two diagonals
    if (win < 0) {
      pwin = wlo > 0 ? -1 : -2;
      plo = down;
    } else {
      const uint32_t r = (ci - 1) & 63u;
      if (wlo > 0 && (cj < r || cj - r < (wlo >> 6))) {
        plo = down;
      } else if (win > 0) {  // entries on row 63 of strip win - 1 at columns cj - 63 .. cj
        pwin = win - 1;
        plo = cj * 64;
      } else {
        pwin = -1;
        plo = cj >= 4032 ? ((cj - 4032) & ~63u) : 0;
      }
    }
    if (pwin != -2) fetch(pwin, plo);
  };
  auto flush = [&]() {
    const uint32_t x = k0 + lane;
    if (lane < kk && x < cap) ops_lds[x] = (uint8_t)acc;
    if (lane < kk && x >= cap) ops[x] = (uint8_t)acc;
    k0 += kk;
    kk = 0;
  };
  auto record = [&](uint32_t op) {  // lane kk of acc takes op
    acc = lane == kk ? (int)op : acc;
    ++kk;
  };
  const uint32_t ta = lane >> 3, tb = lane & 7u, tdl = ta * 65 + tb * 64;  // this lane's cell in the table
  while (i > 0 || j > 0) {
    if (kk > 48) flush();  // room for the 14 steps at most that one table takes
    if (i > 0 && j > 0) {
      const uint32_t r = (i - 1) & 63u;
      const uint32_t idx = (j + r) * 64 + r;
      window((int)((i - 1) >> 6), idx, i, j);
      const uint32_t o = idx - wlo;
      // one 10-bit field per arriving state: the next state times 10 and
      // the step to the lane the next step reads; 31 in the low five bits:
      // leave the table
      const bool cell = ta <= r && tb < j && tdl <= o;  // the cell is in this strip, past column 0 and in the window
      const uint32_t byte = stage[cell ? o - tdl : 0];
      uint32_t T = 0;
#pragma unroll
      for (uint32_t s = 0; s < 3; ++s) {
        const uint32_t c = (byte >> (2 * s)) & 3u;
        const uint32_t nx = s == 1 ? (c == 1 ? 2u : (c == 2 ? 1u : c)) : c;
        const uint32_t na = ta + (s == 2) + (nx == 0), nb = tb + (s == 1) + (nx == 0);
        const uint32_t f = !cell || nx > 2 || na > 7 || nb > 7 ? 1023u : (10 * nx) | ((na * 8 + nb - lane) << 5);
        T |= f << (10 * s);
      }
      uint32_t sh = 10u * (uint32_t)st;
      uint32_t Lr = st == 0 ? 9u : 0u;  // the lane this step reads: the cell diagonal to the walk's for M
      const uint32_t k_in = kk;
      uint32_t f = ((uint32_t)__builtin_amdgcn_readlane((int)T, (int)Lr) >> sh) & 1023u;
      while ((f & 31u) != 31u) {  // one exit: the loop stays a plain scalar loop
        record(sh >> 3);          // the state's number (0, 10, 20 -> 0, 1, 2)
        Lr += f >> 5;
        sh = f & 31u;
        f = ((uint32_t)__builtin_amdgcn_readlane((int)T, (int)Lr) >> sh) & 1023u;
      }
      if (kk != k_in) {
        st = (int)(sh >> 3);
        const uint32_t Lc = st == 0 ? Lr - 9 : Lr;
        i -= Lc >> 3;
        j -= Lc & 7u;
        continue;
      }
    }
    // one step outside the table: the byte this step needs is the walk's
    // cell for D and I, the diagonal cell for M (after the move)
    uint32_t ci = i, cj = j;
    if (st == 0) {
      if (i == 0 || j == 0) break;  // cannot happen for a consistent matrix
      ci = i - 1;
      cj = j - 1;
    } else if (st == 1) {
      if (j == 0) break;
    } else if (i == 0) {
      break;
    }
    record((uint32_t)st);
    const int region = ci == 0 ? -1 : (int)((ci - 1) >> 6);
    const uint32_t idx = ci == 0 ? cj : (cj + ((ci - 1) & 63u)) * 64 + ((ci - 1) & 63u);
    window(region, idx, ci, cj);
    const uint32_t byte = __builtin_amdgcn_readfirstlane(stage[idx - wlo]);
    if (st == 0) {
      i = ci;
      j = cj;
      st = (int)(byte & 3u);
    } else if (st == 1) {
      const uint32_t s = (byte >> 2) & 3u;
      --j;
      st = s == 0 ? 0 : (s == 1 ? 2 : 1);
    } else {
      const uint32_t s = (byte >> 4) & 3u;
      --i;
      st = s == 0 ? 0 : (s == 1 ? 1 : 2);
    }
  }
  flush();
  const uint32_t k = k0;
  lds_fence();
  if (k <= cap) {  // ops were gathered from the last column back
    for (uint32_t x = lane; x < k; x += 64) ops[x] = ops_lds[k - 1 - x];
  } else {
    for (uint32_t x = lane; x < cap; x += 64) ops[x] = ops_lds[x];
    __threadfence_block();
    __syncthreads();
    for (uint32_t x = lane; x < k / 2; x += 64) {
      const uint8_t u = ops[x], v = ops[k - 1 - x];
      ops[x] = v;
      ops[k - 1 - x] = u;
    }
  }
  if (lane == 0) {
    A.score[P.idx] = best;
    A.nops[P.idx] = (i == 0 && j == 0) ? k : 0xFFFFFFFFu;  // all ones: the walk stopped early
  }
}

}  // namespace

static uint64_t up256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

}  // namespace famsa

extern "C" int famsa_profile_align(uint32_t nprob, const uint8_t* seqs, const uint64_t* seq_off, const uint8_t* rows,
                                   const uint64_t* rows_off, const uint32_t* nrows, const uint32_t* width,
                                   uint32_t alphabet_size, const int32_t* subst, const int64_t* gap_costs, int device,
                                   int64_t* score, uint8_t* ops, const uint64_t* ops_off, uint32_t* nops) {
  using namespace famsa;
  if (nprob == 0) return 0;
  if (nprob > FAMSA_PROFILE_MAX_PROBLEMS)
    return set_error(FAMSA_LCS_EINVAL, "%u problems (at most %u)", nprob, FAMSA_PROFILE_MAX_PROBLEMS);
  if (!seq_off || !rows_off || !nrows || !width || !subst || !gap_costs || !score || !ops || !ops_off || !nops)
    return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  if (alphabet_size < 1 || alphabet_size > FAMSA_LCS_MAX_ALPHABET)
    return set_error(FAMSA_LCS_EINVAL, "alphabet_size %u not in [1, %u]", alphabet_size, FAMSA_LCS_MAX_ALPHABET);
  const uint32_t sigma = alphabet_size;
  for (uint32_t e = 0; e < sigma * sigma; ++e)
    if (subst[e] > (int32_t)FAMSA_PROFILE_MAX_SUBST || subst[e] < -(int32_t)FAMSA_PROFILE_MAX_SUBST)
      return set_error(FAMSA_LCS_EINVAL, "substitution score %d outside [-%u, %u]", subst[e],
                       FAMSA_PROFILE_MAX_SUBST, FAMSA_PROFILE_MAX_SUBST);
  for (int c = 0; c < 4; ++c)
    if (gap_costs[c] > (int64_t)FAMSA_PROFILE_MAX_GAP || gap_costs[c] < -(int64_t)FAMSA_PROFILE_MAX_GAP)
      return set_error(FAMSA_LCS_EINVAL, "gap cost %lld outside [-%u, %u]", (long long)gap_costs[c],
                       FAMSA_PROFILE_MAX_GAP, FAMSA_PROFILE_MAX_GAP);
  int64_t smax = 0, gmax = 0;  // largest score and gap cost magnitudes
  for (uint32_t e = 0; e < sigma * sigma; ++e) smax = std::max<int64_t>(smax, subst[e] < 0 ? -(int64_t)subst[e] : subst[e]);
  for (int c = 0; c < 4; ++c) gmax = std::max<int64_t>(gmax, gap_costs[c] < 0 ? -gap_costs[c] : gap_costs[c]);
  std::vector<PdpProb> pr(nprob);
  uint64_t o_seq = 0, o_rows = 0, o_cost = 0, o_col = 0, o_rowx = 0, o_edge = 0, o_dir = 0, o_ops = 0;
  uint32_t nmax = 0, kmax = 1;
  for (uint32_t p = 0; p < nprob; ++p) {
    if (seq_off[p + 1] < seq_off[p]) return set_error(FAMSA_LCS_EINVAL, "seq_off decreases at %u", p);
    const uint64_t m = seq_off[p + 1] - seq_off[p];
    const uint32_t K = nrows[p], n = width[p];
    if (m > FAMSA_LCS_MAX_LEN) return set_error(FAMSA_LCS_EINVAL, "problem %u: sequence length %llu", p,
                                                (unsigned long long)m);
    if (K < 1 || K > FAMSA_PROFILE_MAX_ROWS)
      return set_error(FAMSA_LCS_EINVAL, "problem %u: %u profile rows (1..%u)", p, K, FAMSA_PROFILE_MAX_ROWS);
    if (n > FAMSA_LCS_MAX_LEN) return set_error(FAMSA_LCS_EINVAL, "problem %u: profile width %u", p, n);
    if (m && !seqs) return set_error(FAMSA_LCS_EINVAL, "seqs is NULL");
    if (n && !rows) return set_error(FAMSA_LCS_EINVAL, "rows is NULL");
    // codes: the largest sequence code, and the largest row code plus one
    // (mod 256, so that a gap counts as 0), each taken in one pass
    uint8_t smx = 0, rmx = 0;
    for (uint64_t x = seq_off[p]; x < seq_off[p + 1]; ++x) smx = std::max(smx, seqs[x]);
    const uint8_t* r = rows ? rows + rows_off[p] : nullptr;
    for (uint64_t x = 0; x < (uint64_t)K * n; ++x) rmx = std::max(rmx, (uint8_t)(r[x] + 1u));
    if (m && smx >= sigma)
      return set_error(FAMSA_LCS_EINVAL, "problem %u: sequence code %u not below alphabet_size %u", p, smx, sigma);
    if (rmx > sigma)
      return set_error(FAMSA_LCS_EINVAL, "problem %u: profile code %u is neither a gap nor below %u", p, rmx - 1u,
                       sigma);
    PdpProb& d = pr[p];
    d.m = (uint32_t)m;
    d.n = n;
    d.K = K;
    // every DP value is a sum of at most m + n + 1 terms of magnitude at most
    // K max(|S|, |gap cost|); int32 when that stays below 2^28
    d.narrow = ((uint64_t)m + n + 2) * (uint64_t)K * (uint64_t)std::max(smax, gmax) < (1ull << 28) ? 1u : 0u;
    d.idx = p;
    d.seq = o_seq;
    d.rows = o_rows;
    d.cost = o_cost;
    d.col = o_col;
    d.rowx = o_rowx;
    d.edge = o_edge;
    d.dir = o_dir;
    d.ops = o_ops;
    o_seq += m;
    o_rows += (uint64_t)K * n;
    o_cost += (uint64_t)sigma * std::max(n, 1u);
    o_col += (uint64_t)n + 1;
    o_rowx += K;
    o_edge += 2 * pdp_edge_cols(n);  // two edge-row buffers
    o_dir += pdp_dir_bytes((uint32_t)m, n);
    o_ops += m + n;
    nmax = std::max(nmax, n);
    kmax = std::max(kmax, K);
  }
  // one device allocation, 256-byte aligned parts
  uint64_t off = 0;
  auto part = [&](uint64_t bytes) {
    const uint64_t at = off;
    off += up256(bytes ? bytes : 1);
    return at;
  };
  const uint64_t b_probs = part(sizeof(PdpProb) * nprob), b_subst = part(4ull * sigma * sigma),
                 b_seqs = part(o_seq), b_rows = part(o_rows), b_cost = part(4 * o_cost),
                 b_rec = part(sizeof(PdpRec<int64_t>) * o_col), b_first = part(4 * o_rowx),
                 b_last = part(4 * o_rowx), b_edge = part(sizeof(PdpRec<int64_t>) * o_edge), b_dir = part(o_dir),
                 b_ops = part(o_ops), b_score = part(8ull * nprob), b_nops = part(4ull * nprob);
  FAMSA_HIP(hipSetDevice(device));
  // LDS: a problem whose records, costs and edge rows fit in half a CU's LDS
  // (so that two problems share a CU) reads them from there; the launch
  // reserves the largest such share for every workgroup
  int max_lds = 0;
  FAMSA_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
  hipFuncAttributes fa;
  FAMSA_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&pdp_dp_kernel)));
  const uint64_t lds_cap = (uint64_t)std::min(max_lds, (int)kMaxLds) / 2 > fa.sharedSizeBytes
                               ? (uint64_t)std::min(max_lds, (int)kMaxLds) / 2 - fa.sharedSizeBytes
                               : 0;
  uint64_t lds_dyn = 0;
  uint32_t waves = 1;  // the launch's workgroups have as many waves as the widest problem uses
  for (PdpProb& d : pr) {
    d.cost16 = d.narrow && (uint64_t)d.K * (uint64_t)smax < 32768 ? 1u : 0u;
    const uint64_t need = pdp_lds_bytes(d.n, sigma, d.narrow ? 4 : 8, d.cost16 ? 2 : 4);
    d.lds = need <= lds_cap ? 1u : 0u;
    if (d.lds) lds_dyn = std::max(lds_dyn, need);
    waves = std::max(waves, pdp_waves(d.m, d.n));
  }
  // With four problems or more per CU the GPU is full of problems, and more
  // than four waves per problem only add contention (measured on a level of
  // 2,048 problems of widths 50..500: 0.51 ms with four, 0.54 ms with up to
  // sixteen); with fewer, the largest problem's chain bounds the level, and
  // more waves shorten it (its 512 largest problems: 0.41 ms with up to
  // sixteen, 0.47 ms with four; one problem of 555 x 499: 0.39 ms with eight
  // waves, 0.46 ms with four).
  int cus = 0;
  FAMSA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  if (nprob >= 4u * (uint32_t)std::max(cus, 1)) waves = std::min(waves, 4u);
  lds_dyn = std::max<uint64_t>(lds_dyn, kTbMinLds);  // the trace-back's ops buffer
  if (lds_dyn > 65536)
    FAMSA_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&pdp_dp_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_dyn));
  // launch order: the longest DP first (strips x sweep steps), so that the
  // problem that bounds the launch starts at once
  std::vector<uint32_t> order(nprob);
  std::iota(order.begin(), order.end(), 0u);
  auto span = [&](uint32_t p) { return (uint64_t)((pr[p].m + 63) / 64) * (pr[p].n + 64); };
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return span(a) > span(b); });
  std::vector<PdpProb> launch(nprob);
  for (uint32_t x = 0; x < nprob; ++x) launch[x] = pr[order[x]];
  hipStream_t st = nullptr;
  int rc = lib_stream(device, 0, &st);
  if (rc) return rc;
  DevMem mem;
  rc = mem.alloc(off);
  if (rc) return rc;
  uint8_t* D = mem.as<uint8_t>();
  // sequences and rows go up in one copy each when the caller's arrays
  // already hold them back to back in problem order, else through a packed
  // host copy
  bool seq_packed = true, rows_packed = true;
  for (uint32_t p = 0; p < nprob; ++p) {
    seq_packed = seq_packed && seq_off[p] - seq_off[0] == pr[p].seq;
    rows_packed = rows_packed && rows_off[p] - rows_off[0] == pr[p].rows;
  }
  std::vector<uint8_t> hseq, hrows;
  const uint8_t* up_seq = o_seq ? seqs + seq_off[0] : nullptr;
  const uint8_t* up_rows = o_rows ? rows + rows_off[0] : nullptr;
  if (o_seq && !seq_packed) {
    hseq.resize(o_seq);
    for (uint32_t p = 0; p < nprob; ++p)
      if (pr[p].m) memcpy(hseq.data() + pr[p].seq, seqs + seq_off[p], pr[p].m);
    up_seq = hseq.data();
  }
  if (o_rows && !rows_packed) {
    hrows.resize(o_rows);
    for (uint32_t p = 0; p < nprob; ++p) {
      const uint64_t rb = (uint64_t)pr[p].K * pr[p].n;
      if (rb) memcpy(hrows.data() + pr[p].rows, rows + rows_off[p], rb);
    }
    up_rows = hrows.data();
  }
  FAMSA_HIP(hipMemcpyAsync(D + b_probs, launch.data(), sizeof(PdpProb) * nprob, hipMemcpyHostToDevice, st));
  FAMSA_HIP(hipMemcpyAsync(D + b_subst, subst, 4ull * sigma * sigma, hipMemcpyHostToDevice, st));
  if (o_seq) FAMSA_HIP(hipMemcpyAsync(D + b_seqs, up_seq, o_seq, hipMemcpyHostToDevice, st));
  if (o_rows) FAMSA_HIP(hipMemcpyAsync(D + b_rows, up_rows, o_rows, hipMemcpyHostToDevice, st));
  PdpArrays A;
  A.seqs = D + b_seqs;
  A.rows = D + b_rows;
  A.cost = reinterpret_cast<int32_t*>(D + b_cost);
  A.rec = reinterpret_cast<PdpRec<int64_t>*>(D + b_rec);
  A.first = reinterpret_cast<int32_t*>(D + b_first);
  A.last = reinterpret_cast<int32_t*>(D + b_last);
  A.edge = reinterpret_cast<PdpRec<int64_t>*>(D + b_edge);
  A.dir = D + b_dir;
  A.ops = D + b_ops;
  A.score = reinterpret_cast<int64_t*>(D + b_score);
  A.nops = reinterpret_cast<uint32_t*>(D + b_nops);
  A.To = gap_costs[0];
  A.Te = gap_costs[1];
  A.Go = gap_costs[2];
  A.Ge = gap_costs[3];
  A.tb_cap = (uint32_t)lds_dyn;
  const PdpProb* dprobs = reinterpret_cast<const PdpProb*>(D + b_probs);
  hipEvent_t ev[2];
  FAMSA_HIP(hipEventCreate(&ev[0]));
  FAMSA_HIP(hipEventCreate(&ev[1]));
  hipLaunchKernelGGL(pdp_rows_kernel, dim3(nprob, std::min(64u, (kmax + kRowsPerBlock - 1) / kRowsPerBlock)),
                     dim3(256), 0, st, dprobs, A);
  FAMSA_HIP(hipGetLastError());
  hipLaunchKernelGGL(pdp_cols_kernel, dim3(nprob, nmax / 256 + 1), dim3(256), 4ull * sigma * (256 + sigma), st,
                     dprobs, A, reinterpret_cast<const int32_t*>(D + b_subst), sigma);
  FAMSA_HIP(hipGetLastError());
  FAMSA_HIP(hipEventRecord(ev[0], st));
  hipLaunchKernelGGL(pdp_dp_kernel, dim3(nprob), dim3(64 * waves), lds_dyn, st, dprobs, A, sigma);
  FAMSA_HIP(hipGetLastError());
  FAMSA_HIP(hipEventRecord(ev[1], st));
  std::vector<uint8_t> hops(o_ops ? o_ops : 1);
  FAMSA_HIP(hipMemcpyAsync(score, D + b_score, 8ull * nprob, hipMemcpyDeviceToHost, st));
  FAMSA_HIP(hipMemcpyAsync(nops, D + b_nops, 4ull * nprob, hipMemcpyDeviceToHost, st));
  if (o_ops) FAMSA_HIP(hipMemcpyAsync(hops.data(), D + b_ops, o_ops, hipMemcpyDeviceToHost, st));
  FAMSA_HIP(hipStreamSynchronize(st));
  float ms = 0;
  FAMSA_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  g_profile_dp_ms = ms;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  for (uint32_t p = 0; p < nprob; ++p) {
    if (nops[p] == 0xFFFFFFFFu) return set_error(FAMSA_LCS_EDEVICE, "problem %u: trace-back stopped early", p);
    if ((uint64_t)nops[p] > (uint64_t)pr[p].m + pr[p].n)  // an alignment has at most m + n ops
      return set_error(FAMSA_LCS_EDEVICE, "problem %u: %u ops from the device", p, nops[p]);
    memcpy(ops + ops_off[p], hops.data() + pr[p].ops, nops[p]);
  }
  return 0;
}

extern "C" double famsa_profile_last_dp_ms(void) { return famsa::g_profile_dp_ms; }

extern "C" int famsa_gap_costs_scaled(uint32_t k, const double* base, double gl, double gd, int64_t* out) {
  using namespace famsa;
  if (!base || !out) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  if (k == 0 || !(gl > 0) || gd == 0) return set_error(FAMSA_LCS_EINVAL, "k = %u, gl = %g, gd = %g", k, gl, gd);
  const double g = 1.0 + log((double)k / gl) / gd;
  for (int c = 0; c < 4; ++c) {
    const double x = base[c] * g;
    const double r = floor(fabs(x) + 0.5);
    if (!(r <= (double)FAMSA_PROFILE_MAX_GAP))
      return set_error(FAMSA_LCS_EINVAL, "scaled gap cost %g beyond %u", x, FAMSA_PROFILE_MAX_GAP);
    out[c] = (int64_t)r * (x >= 0 ? 1 : -1);
  }
  return 0;
}
