// Exact single linkage on the GPU: the maximum spanning forest of the
// similarity graph, updated tile by tile from device-resident LCS tiles.
//
// The paper builds its guide tree by single linkage, incrementally and with
// O(k) memory (Methods, "Determination of the guide tree").  Single linkage
// merges clusters in the order of the maximum spanning tree of the
// similarities, so keeping that tree is enough: after every tile, the forest
// F becomes the maximum spanning forest of F plus the tile's pairs (a forest
// that is optimal for a set of edges stays a valid summary of it, by the
// cycle property).  Each update is a Boruvka run on the device:
//   1. every vertex finds its best edge to another component -- a row pass
//      over the tile's rows, a column pass over its columns, and a pass over
//      F's edges;
//   2. every component takes the best of its vertices' edges (a two-phase
//      atomic maximum on the similarity, then minimum on the edge id);
//   3. components hook along their edges and are relabelled by pointer
//      jumping; the hooked edges form the new forest;
// until no component has an outgoing edge.
//
// Similarity (Methods, "Pairwise similarities calculation") is
// LCS / indel^2 with indel = |A| + |B| - 2 LCS, +infinity when indel = 0.
// It is compared as the correctly rounded double of that ratio: for lengths up
// to 65535 two different ratios differ by at least four units in the last
// place, so the order is exact.  Ties between equal similarities are broken
// by the edge (u, v), u < v, lexicographically, which makes every choice
// unique (no cycles).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "runtime.h"

namespace famsa {

// Key of an edge's similarity: the double's bits plus one (similarities are
// >= 0 or +inf, so the bits order like the values); 0 means "no edge".
__device__ __forceinline__ uint64_t sim_key(int32_t L, uint32_t la, uint32_t lb) {
  const int64_t d = (int64_t)la + (int64_t)lb - 2 * (int64_t)L;
  const double s = d == 0 ? __builtin_inf() : (double)L / (double)(d * d);
  return (uint64_t)__double_as_longlong(s) + 1ull;
}

// (key, id) pairs: larger key wins, then smaller id.
__device__ __forceinline__ bool better(uint64_t ka, uint64_t ia, uint64_t kb, uint64_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

struct MstDev {
  const uint32_t* len;
  uint32_t k;
  uint32_t* comp;     // component label of each vertex
  uint32_t* parent;   // hook target of each component root
  uint64_t* vkey;     // best outgoing edge per vertex: key, id, LCS
  uint64_t* vid;
  int32_t* vL;
  uint64_t* wkey;     // best forest edge per vertex (merged into vkey/vid/vL)
  uint64_t* wid;
  int32_t* wL;
  uint64_t* ckey;     // best outgoing edge per component
  uint64_t* cid;
  uint64_t* pkey;     // row partials: best edge of each (tile row, column block)
  uint64_t* pid;
  int32_t* pL;
  uint64_t* qkey;     // column partials: best edge of each (row slice, column)
  uint64_t* qid;
  int32_t* qL;
  const uint32_t* fu;  // current forest edges (ctl->nf of them)
  const uint32_t* fv;
  const int32_t* fL;
  uint32_t* nu;        // new forest edges (ctl->nnew of them)
  uint32_t* nv;
  int32_t* nL;
  struct Ctl {
    uint32_t nf;      // edges in the current forest
    uint32_t nnew;    // edges in the new forest
    uint32_t hooks;   // hooks in this round
    uint32_t done;    // no component has an outgoing edge: later rounds do nothing
    uint64_t rounds;  // rounds that did work, over all tiles
  }* ctl;
};

// The scan: a block covers 256 columns (four per lane) and a slice of 64
// tile rows, split over its four waves.
constexpr uint32_t kScanCols = 256;
constexpr uint32_t kScanSlice = 64;
constexpr uint32_t kScanWaves = 4;

// Values before tile row i (rows r0.. of the upper triangle, k - 1 - t per row t).
__device__ __forceinline__ uint64_t row_off(uint64_t k, uint32_t r0, uint32_t i) {
  const uint64_t n = i - r0;
  return n * (k - 1) - ((uint64_t)r0 + i - 1) * n / 2;
}

__device__ __forceinline__ void take(uint64_t& bk, uint64_t& bi, int32_t& bL, uint64_t k2, uint64_t i2, int32_t L2) {
  if (better(k2, i2, bk, bi)) {
    bk = k2;
    bi = i2;
    bL = L2;
  }
}

// Wave-wide best of (key, id, L); every lane gets the result.
__device__ __forceinline__ void wave_best(uint64_t& bk, uint64_t& bi, int32_t& bL) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t k2 = __shfl_xor(bk, d, 64);
    const uint64_t i2 = __shfl_xor(bi, d, 64);
    const int32_t L2 = __shfl_xor(bL, d, 64);
    take(bk, bi, bL, k2, i2, L2);
  }
}

__global__ void mst_tile_begin(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) {
    m.ctl->done = 0;
    m.ctl->hooks = 0;
    m.ctl->nnew = 0;
  }
  if (v >= m.k) return;
  m.comp[v] = v;
  m.parent[v] = v;
}

// One pass over the tile per round, in small blocks that fit beside the
// LCS kernels.  Block (bx, sy) covers columns [256 bx, 256 bx + 256) (four
// per lane) and the 64 tile rows of slice sy that have a column after them
// in the block; each element (i, j) whose ends lie in different components is
// a candidate for both ends.  A row's best over the block's columns is a wave
// reduction, stored as partial (row, bx); a column's best over the slice's
// rows is reduced over the four waves in LDS and stored as partial (sy, j).
//
// Components only grow during a tile's rounds, so the candidates of a row or
// a column only shrink: a partial whose edge still joins two components is
// still the best of its set.  After the tile's first round a block therefore
// recomputes only the partials whose edge has since fallen inside one
// component, and reads only the elements those partials need.
__global__ __launch_bounds__(256) void mst_scan(MstDev m, const int32_t* __restrict__ tile, uint32_t r0, uint32_t r1,
                                                uint32_t nblk, uint32_t bx0, uint32_t first) {
  if (m.ctl->done) return;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t bx = bx0 + blockIdx.x;  // blocks left of column r0 + 1 hold no pair and are not launched
  const uint32_t jb = bx * kScanCols;
  const uint64_t k = m.k;
  uint64_t ck[4], cid[4];
  int32_t cL[4];
  uint32_t cc[4], cl[4];
  bool cnew[4];  // column partial (sy, j) to recompute
  bool anycol = false;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    ck[c] = 0;
    cid[c] = ~0ull;
    cL[c] = 0;
    const uint32_t j = jb + 64u * c + lane;
    cc[c] = j < m.k ? m.comp[j] : 0u;
    cl[c] = j < m.k ? m.len[j] : 0u;
    cnew[c] = j < m.k;
    if (!first && j < m.k) {
      const uint64_t q = (uint64_t)blockIdx.y * k + j;
      // no candidate then means none now; else recompute once its row end joined j's component
      cnew[c] = m.qkey[q] != 0 && m.comp[(uint32_t)(m.qid[q] / k)] == cc[c];
    }
    anycol |= cnew[c];
  }
  anycol = __any(anycol);
  const uint32_t i0 = r0 + blockIdx.y * kScanSlice;
  const uint32_t iend = min(min(r1, i0 + kScanSlice), jb + kScanCols - 1u);  // rows with a column of the block after them
  // The wave's rows are i0 + wave + kScanWaves t.  Lane t reads row t's
  // component, length and partial up front, all rows at once; rows are then
  // taken kChunk at a time, each group's tile loads issued together.
  constexpr uint32_t kRows = kScanSlice / kScanWaves;
  constexpr uint32_t kChunk = 4;  // rows whose tile loads are in flight together (8: slower)
  const uint32_t myrow = i0 + wave + kScanWaves * lane;
  const bool myok = lane < kRows && myrow < iend;
  uint32_t mci = 0, mli = 0;
  bool mnew = false;
  if (myok) {
    mci = m.comp[myrow];
    mli = m.len[myrow];
    mnew = true;
    if (!first) {
      const uint64_t p = (uint64_t)(myrow - r0) * nblk + bx;
      mnew = m.pkey[p] != 0 && m.comp[(uint32_t)(m.pid[p] % k)] == mci;
    }
  }
  const uint32_t nrows = (uint32_t)__popcll(__ballot(myok));  // rows 0..nrows-1 of the wave exist
  const uint64_t newmask = __ballot(mnew);
  for (uint32_t t0 = 0; t0 < nrows && (anycol || (newmask >> t0) != 0); t0 += kChunk) {
    int32_t L[kChunk][4];
    uint32_t ci[kChunk], li[kChunk];
    bool rnew[kChunk];
#pragma unroll
    for (int u = 0; u < (int)kChunk; ++u) {
      const uint32_t t = t0 + (uint32_t)u;
      const bool live = t < nrows;
      const uint32_t i = i0 + wave + kScanWaves * t;
      ci[u] = (uint32_t)__shfl((int)mci, (int)(t & 63u), 64);
      li[u] = (uint32_t)__shfl((int)mli, (int)(t & 63u), 64);
      rnew[u] = live && ((newmask >> t) & 1ull);
      const uint64_t off = row_off(k, r0, i);  // LCS(i, j) at off + j - i - 1
#pragma unroll
      for (int c = 0; c < 4; ++c) {  // only pairs across components, and only those a partial needs
        const uint32_t j = jb + 64u * c + lane;
        L[u][c] = (live && j > i && j < m.k && cc[c] != ci[u] && (rnew[u] || cnew[c])) ? tile[off + (j - i - 1u)] : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < (int)kChunk; ++u) {
      const uint32_t t = t0 + (uint32_t)u;
      if (t >= nrows) break;
      const uint32_t i = i0 + wave + kScanWaves * t;
      uint64_t rk = 0, ri = ~0ull;
      int32_t rL = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t j = jb + 64u * c + lane;
        if (j > i && j < m.k && cc[c] != ci[u] && (rnew[u] || cnew[c])) {
          const uint64_t key = sim_key(L[u][c], li[u], cl[c]);
          const uint64_t id = (uint64_t)i * k + j;
          if (cnew[c]) take(ck[c], cid[c], cL[c], key, id, L[u][c]);
          take(rk, ri, rL, key, id, L[u][c]);
        }
      }
      if (rnew[u]) {
        if (__any(rk != 0)) wave_best(rk, ri, rL);  // else no lane has a candidate: (0, ~0, 0) as it is
        if (lane == 0) {
          const uint64_t p = (uint64_t)(i - r0) * nblk + bx;
          m.pkey[p] = rk;
          m.pid[p] = ri;
          m.pL[p] = rL;
        }
      }
    }
  }
  __shared__ uint64_t sk[kScanWaves / 2][kScanCols], si[kScanWaves / 2][kScanCols];
  __shared__ int32_t sL[kScanWaves / 2][kScanCols];
  for (uint32_t h = kScanWaves / 2; h > 0; h >>= 1) {
    if (wave >= h && wave < 2 * h) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sk[wave - h][64 * c + lane] = ck[c];
        si[wave - h][64 * c + lane] = cid[c];
        sL[wave - h][64 * c + lane] = cL[c];
      }
    }
    __syncthreads();
    if (wave < h) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        take(ck[c], cid[c], cL[c], sk[wave][64 * c + lane], si[wave][64 * c + lane], sL[wave][64 * c + lane]);
    }
    __syncthreads();
  }
  if (wave == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t j = jb + 64u * c + lane;
      if (!cnew[c]) continue;
      const uint64_t q = (uint64_t)blockIdx.y * k + j;
      m.qkey[q] = ck[c];
      m.qid[q] = cid[c];
      m.qL[q] = cL[c];
    }
  }
}

// Column results and per-round reset: vertex j takes the best of its column
// partials over the row slices; its forest and component slots are cleared.
__global__ void mst_col_reduce(MstDev m, uint32_t r0, uint32_t nslice) {
  if (m.ctl->done) return;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.k) return;
  uint64_t bk = 0, bi = ~0ull;
  int32_t bL = 0;
  if (j > r0)  // a column at or before the tile's first row has no pair in it (and no partials)
    for (uint32_t y = 0; y < nslice; ++y) {
      const uint64_t q = (uint64_t)y * m.k + j;
      take(bk, bi, bL, m.qkey[q], m.qid[q], m.qL[q]);
    }
  m.vkey[j] = bk;
  m.vid[j] = bi;
  m.vL[j] = bL;
  m.wkey[j] = 0;
  m.wid[j] = ~0ull;
  m.wL[j] = 0;
  m.ckey[j] = 0;
  m.cid[j] = ~0ull;
}

// Row results: tile row i reduces its partials over the blocks that hold a
// column after it, and merges them into its candidate.
__global__ __launch_bounds__(64) void mst_row_reduce(MstDev m, uint32_t r0, uint32_t nblk) {
  if (m.ctl->done) return;
  const uint32_t i = r0 + blockIdx.x;
  uint64_t bk = 0, bi = ~0ull;
  int32_t bL = 0;
  const uint64_t base = (uint64_t)blockIdx.x * nblk;
  for (uint32_t b = (i + 1u) / kScanCols + threadIdx.x; b < nblk; b += 64u)
    take(bk, bi, bL, m.pkey[base + b], m.pid[base + b], m.pL[base + b]);
  wave_best(bk, bi, bL);
  if (threadIdx.x == 0) {
    take(bk, bi, bL, m.vkey[i], m.vid[i], m.vL[i]);
    m.vkey[i] = bk;
    m.vid[i] = bi;
    m.vL[i] = bL;
  }
}

// Forest edges: candidates for both ends, gathered in the w* slots in three
// phases (key, id, LCS).
__global__ void mst_forest_key(MstDev m) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || e >= m.ctl->nf) return;
  const uint32_t u = m.fu[e], v = m.fv[e];
  if (m.comp[u] == m.comp[v]) return;
  const uint64_t key = sim_key(m.fL[e], m.len[u], m.len[v]);
  if (key > m.wkey[u]) atomicMax((unsigned long long*)&m.wkey[u], (unsigned long long)key);
  if (key > m.wkey[v]) atomicMax((unsigned long long*)&m.wkey[v], (unsigned long long)key);
}

__global__ void mst_forest_id(MstDev m) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || e >= m.ctl->nf) return;
  const uint32_t u = m.fu[e], v = m.fv[e];
  if (m.comp[u] == m.comp[v]) return;
  const uint64_t key = sim_key(m.fL[e], m.len[u], m.len[v]);
  const uint64_t id = (uint64_t)u * m.k + v;
  if (m.wkey[u] == key) atomicMin((unsigned long long*)&m.wid[u], (unsigned long long)id);
  if (m.wkey[v] == key) atomicMin((unsigned long long*)&m.wid[v], (unsigned long long)id);
}

__global__ void mst_forest_L(MstDev m) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || e >= m.ctl->nf) return;
  const uint32_t u = m.fu[e], v = m.fv[e];
  if (m.comp[u] == m.comp[v]) return;
  const uint64_t id = (uint64_t)u * m.k + v;
  if (m.wid[u] == id) m.wL[u] = m.fL[e];
  if (m.wid[v] == id) m.wL[v] = m.fL[e];
}

// Each vertex's candidate (tile pass results already in v*) takes its forest
// edge, and offers itself to its component's maximum.  A plain read first
// skips most atomics: once a component holds a large key few vertices beat it.
__global__ void mst_vertex_merge(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done) return;
  const bool ok = v < m.k;
  uint64_t bk = 0;
  uint32_t c = 0;
  if (ok) {
    uint64_t bi = m.vid[v];
    int32_t bL = m.vL[v];
    bk = m.vkey[v];
    if (m.wkey[v]) {
      take(bk, bi, bL, m.wkey[v], m.wid[v], m.wL[v]);
      m.vkey[v] = bk;
      m.vid[v] = bi;
      m.vL[v] = bL;
    }
    c = m.comp[v];
  }
  // Late in a tile most vertices share one large component, and their
  // atomics on its slot would queue up: the lanes of a wave in the
  // component of its first candidate take their maximum first, and one lane
  // offers it.  Every lane stays in the wave for the shuffles.
  const bool cand = ok && bk != 0;
  const uint64_t candmask = __ballot(cand);
  if (candmask == 0) return;
  const int first = __ffsll((unsigned long long)candmask) - 1;
  const uint32_t lead = (uint32_t)__shfl((int)c, first, 64);
  uint64_t x = cand && c == lead ? bk : 0;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t y = __shfl_xor(x, d, 64);
    x = y > x ? y : x;
  }
  if ((int)__lane_id() == first) {
    uint64_t* slot = &m.ckey[lead];
    if (x > *slot) atomicMax((unsigned long long*)slot, (unsigned long long)x);
  }
  if (cand && c != lead) {
    uint64_t* slot = &m.ckey[c];
    if (bk > *slot) atomicMax((unsigned long long*)slot, (unsigned long long)bk);
  }
}

__global__ void mst_comp_id(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || v >= m.k || m.vkey[v] == 0) return;
  const uint32_t c = m.comp[v];
  if (m.vkey[v] == m.ckey[c]) atomicMin((unsigned long long*)&m.cid[c], (unsigned long long)m.vid[v]);
}

// Hook every component with an outgoing edge onto the component at its other
// end.  The one vertex of the component that holds its chosen edge (the
// candidate key and id equal the component's) does it, so the edge's LCS is
// at hand.  Two components that chose the same edge hook once: the larger
// onto the smaller.  Each hook adds its edge to the new forest.
__global__ void mst_hook(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || v >= m.k) return;
  const uint64_t key = m.vkey[v];
  if (key == 0) return;
  const uint32_t c = m.comp[v];
  if (key != m.ckey[c] || m.vid[v] != m.cid[c]) return;
  const uint64_t id = m.cid[c];
  const uint32_t u = (uint32_t)(id / m.k), w = (uint32_t)(id % m.k);
  const uint32_t d = m.comp[u] == c ? m.comp[w] : m.comp[u];
  if (m.cid[d] == id && c < d) return;  // mutual choice: d hooks onto c
  m.parent[c] = d;
  const uint32_t slot = atomicAdd(&m.ctl->nnew, 1u);
  m.nu[slot] = u;
  m.nv[slot] = w;
  m.nL[slot] = m.vL[v];
  atomicAdd(&m.ctl->hooks, 1u);
}

// Every component follows its hook chain to the root (chains are acyclic:
// with a strict order on edges the only cycles of chosen edges are the mutual
// pairs, which hook once).  Concurrent shortcuts by other threads only move
// entries further up the same chain.
__global__ void mst_jump(MstDev m) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || c >= m.k) return;
  uint32_t r = m.parent[c];
  while (m.parent[r] != r) r = m.parent[r];
  m.parent[c] = r;
}

// Relabel every vertex; the first thread also ends the round: a round
// without hooks finishes the tile (its relabelling changes nothing, so blocks
// that see the flag early lose nothing).
__global__ void mst_relabel(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (m.ctl->done || v >= m.k) return;
  m.comp[v] = m.parent[m.comp[v]];
  if (v == 0) {
    if (m.ctl->hooks == 0) {
      m.ctl->done = 1;
    } else {
      m.ctl->rounds += 1;
      m.ctl->hooks = 0;
    }
  }
}

// The new forest becomes the current one (the host swaps the arrays).
__global__ void mst_tile_end(MstDev m) {
  if (threadIdx.x != 0) return;
  m.ctl->nf = m.ctl->nnew;
  m.ctl->nnew = 0;
}

}  // namespace famsa

using namespace famsa;

struct famsa_mst_s {
  uint32_t k = 0;
  int device = 0;
  DevMem len, comp, parent, vkey, vid, vL, wkey, wid, wL, ckey, cid, pkey, pid, pL, qkey, qid, qL;
  DevMem fu, fv, fL, nu, nv, nL, ctl;
  uint64_t part_cap = 0;   // row partials the p* arrays hold
  uint32_t slice_cap = 0;  // row slices the q* arrays hold
  PinMem hctl;
  uint64_t tiles = 0;
  // Tiles arrive on whatever stream their producer used (a plan alternates
  // two); this event marks the end of the last tile's work, and the next
  // tile's work waits for it, so merges never overlap whatever the streams.
  hipEvent_t last = nullptr;
  bool has_last = false;
  ~famsa_mst_s() {
    if (last) {
      if (has_last) (void)hipEventSynchronize(last);
      (void)hipEventDestroy(last);
    }
  }
  int wait_last() const {
    if (has_last) FAMSA_HIP(hipEventSynchronize(last));
    return 0;
  }
  MstDev view() {
    MstDev m;
    m.len = len.as<uint32_t>();
    m.k = k;
    m.comp = comp.as<uint32_t>();
    m.parent = parent.as<uint32_t>();
    m.vkey = vkey.as<uint64_t>();
    m.vid = vid.as<uint64_t>();
    m.vL = vL.as<int32_t>();
    m.wkey = wkey.as<uint64_t>();
    m.wid = wid.as<uint64_t>();
    m.wL = wL.as<int32_t>();
    m.ckey = ckey.as<uint64_t>();
    m.cid = cid.as<uint64_t>();
    m.pkey = pkey.as<uint64_t>();
    m.pid = pid.as<uint64_t>();
    m.pL = pL.as<int32_t>();
    m.qkey = qkey.as<uint64_t>();
    m.qid = qid.as<uint64_t>();
    m.qL = qL.as<int32_t>();
    m.fu = fu.as<uint32_t>();
    m.fv = fv.as<uint32_t>();
    m.fL = fL.as<int32_t>();
    m.nu = nu.as<uint32_t>();
    m.nv = nv.as<uint32_t>();
    m.nL = nL.as<int32_t>();
    m.ctl = ctl.as<MstDev::Ctl>();
    return m;
  }
  int merge_tile(const famsa_lcs_tile* t, hipStream_t s);
  int read_ctl(MstDev::Ctl* out, hipStream_t s);
};

static inline dim3 grid_for(uint64_t n, uint32_t b = 256) { return dim3((uint32_t)std::max<uint64_t>(1, (n + b - 1) / b)); }

int famsa_mst_s::read_ctl(MstDev::Ctl* out, hipStream_t s) {
  FAMSA_HIP(hipMemcpyAsync(hctl.p, ctl.p, sizeof(MstDev::Ctl), hipMemcpyDeviceToHost, s));
  FAMSA_HIP(hipStreamSynchronize(s));
  memcpy(out, hctl.p, sizeof(MstDev::Ctl));
  return 0;
}

// Boruvka rounds are queued in batches without waiting: every kernel of a
// round after the last useful one returns at once (the `done` flag), so the
// host only checks after each batch.  Borůvka needs at most ceil(log2 k) + 1
// rounds, and few tiles need more than the first batch.
int famsa_mst_s::merge_tile(const famsa_lcs_tile* t, hipStream_t s) {
  const uint32_t r0 = t->row_begin, r1 = t->row_end;
  const bool has_tile = t->count && r1 > r0;
  if (r1 - r0 > 65535u) return set_error(FAMSA_LCS_EINVAL, "tiles of more than 65535 rows are not supported");
  if (has_last) FAMSA_HIP(hipStreamWaitEvent(s, last, 0));  // the previous tile's merge, on any stream
  const uint32_t nblk = (uint32_t)((k + kScanCols - 1) / kScanCols);
  const uint32_t nslice = has_tile ? (r1 - r0 + kScanSlice - 1) / kScanSlice : 0;
  if (has_tile && ((uint64_t)nblk * (r1 - r0) > part_cap || nslice > slice_cap)) {
    FAMSA_HIP(hipStreamSynchronize(s));  // the old partials may still be in use
    int rc;
    if ((uint64_t)nblk * (r1 - r0) > part_cap) {
      part_cap = (uint64_t)nblk * (r1 - r0);
      if ((rc = pkey.alloc(part_cap * 8)) || (rc = pid.alloc(part_cap * 8)) || (rc = pL.alloc(part_cap * 4))) return rc;
    }
    if (nslice > slice_cap) {
      slice_cap = nslice;
      const uint64_t n = (uint64_t)slice_cap * k;
      if ((rc = qkey.alloc(n * 8)) || (rc = qid.alloc(n * 8)) || (rc = qL.alloc(n * 4))) return rc;
    }
  }
  const MstDev m = view();
  const dim3 gk = grid_for(k);
  // first column block holding a column after row r0 (has_tile: r0 + 1 < k, so bx0 < nblk)
  const uint32_t bx0 = (uint32_t)((r0 + 1ull) / kScanCols);
  hipLaunchKernelGGL(mst_tile_begin, gk, dim3(256), 0, s, m);
  const uint32_t kmax_rounds = 2 + (uint32_t)ceil(log2((double)std::max<uint32_t>(k, 2)));
  uint32_t queued = 0;
  for (uint32_t batch = 6;; batch = 2) {
    for (uint32_t r = 0; r < batch; ++r) {
      const uint32_t first = queued == 0 && r == 0;  // the tile's first round computes every partial
      if (has_tile)
        hipLaunchKernelGGL(mst_scan, dim3(nblk - bx0, nslice), dim3(64 * kScanWaves), 0, s, m, t->lcs, r0, r1, nblk,
                           bx0, first);
      hipLaunchKernelGGL(mst_col_reduce, gk, dim3(256), 0, s, m, r0, nslice);
      if (has_tile) hipLaunchKernelGGL(mst_row_reduce, dim3(r1 - r0), dim3(64), 0, s, m, r0, nblk);
      hipLaunchKernelGGL(mst_forest_key, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_forest_id, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_forest_L, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_vertex_merge, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_comp_id, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_hook, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_jump, gk, dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_relabel, gk, dim3(256), 0, s, m);
      FAMSA_HIP(hipGetLastError());
    }
    queued += batch;
    MstDev::Ctl c;
    int rc = read_ctl(&c, s);
    if (rc) return rc;
    if (c.done) break;
    if (queued > kmax_rounds) return set_error(FAMSA_LCS_EDEVICE, "spanning forest did not converge in %u rounds", queued);
  }
  hipLaunchKernelGGL(mst_tile_end, dim3(1), dim3(64), 0, s, m);
  FAMSA_HIP(hipGetLastError());
  FAMSA_HIP(hipEventRecord(last, s));
  has_last = true;
  std::swap(fu.p, nu.p);
  std::swap(fv.p, nv.p);
  std::swap(fL.p, nL.p);
  ++tiles;
  return 0;
}

extern "C" {

int famsa_mst_create(const uint32_t* lengths, uint32_t k, int device, famsa_mst_t** out) {
  clear_error();
  if (!out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  *out = nullptr;
  if (k && !lengths) return set_error(FAMSA_LCS_EINVAL, "lengths is NULL");
  if (k > (1u << 31)) return set_error(FAMSA_LCS_EINVAL, "k %u too large", k);
  for (uint32_t i = 0; i < k; ++i)
    if (lengths[i] > FAMSA_LCS_MAX_LEN)
      return set_error(FAMSA_LCS_EINVAL, "length %u of sequence %u exceeds %u", lengths[i], i, FAMSA_LCS_MAX_LEN);
  if (device < 0) return set_error(FAMSA_LCS_EINVAL, "device %d < 0", device);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return set_error(FAMSA_LCS_EDEVICE, "no HIP device available");
  }
  if (device >= ndev) return set_error(FAMSA_LCS_EINVAL, "device %d >= device count %d", device, ndev);
  FAMSA_HIP(hipSetDevice(device));
  famsa_mst_s* m = new (std::nothrow) famsa_mst_s();
  if (!m) return set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  m->k = k;
  m->device = device;
  const size_t n = std::max<uint32_t>(k, 1);
  int rc;
  if ((rc = m->len.alloc(n * 4)) || (rc = m->comp.alloc(n * 4)) || (rc = m->parent.alloc(n * 4)) ||
      (rc = m->vkey.alloc(n * 8)) || (rc = m->vid.alloc(n * 8)) || (rc = m->vL.alloc(n * 4)) ||
      (rc = m->wkey.alloc(n * 8)) || (rc = m->wid.alloc(n * 8)) || (rc = m->wL.alloc(n * 4)) ||
      (rc = m->ckey.alloc(n * 8)) || (rc = m->cid.alloc(n * 8)) ||
      (rc = m->fu.alloc(n * 4)) || (rc = m->fv.alloc(n * 4)) || (rc = m->fL.alloc(n * 4)) ||
      (rc = m->nu.alloc(n * 4)) || (rc = m->nv.alloc(n * 4)) || (rc = m->nL.alloc(n * 4)) ||
      (rc = m->ctl.alloc(sizeof(MstDev::Ctl))) || (rc = m->hctl.alloc(sizeof(MstDev::Ctl)))) {
    delete m;
    return rc;
  }
  if (hipEventCreateWithFlags(&m->last, hipEventDisableTiming) != hipSuccess) {
    m->last = nullptr;
    delete m;
    return set_error(FAMSA_LCS_EDEVICE, "hipEventCreate failed");
  }
  if ((k && hipMemcpy(m->len.p, lengths, (size_t)k * 4, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemset(m->ctl.p, 0, sizeof(MstDev::Ctl)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    delete m;
    return set_error(FAMSA_LCS_EDEVICE, "initialising the forest failed");
  }
  *out = m;
  return 0;
}

int famsa_mst_consume(void* user, const famsa_lcs_tile* t) {
  famsa_mst_s* m = static_cast<famsa_mst_s*>(user);
  if (!m || !t || t->k != m->k || t->row_begin > t->row_end || t->row_end > m->k) return 1;
  if (t->count && !t->lcs) return 1;
  if (t->values != FAMSA_LCS_VALUES_LCS) return 1;  // the forest is built from LCS values
  if (t->count != tri_rows(m->k, t->row_begin, t->row_end)) return 1;
  if (hipSetDevice(m->device) != hipSuccess) return 1;
  return m->merge_tile(t, (hipStream_t)t->stream) == 0 ? 0 : 1;
}

int famsa_mst_result(const famsa_mst_t* m, uint32_t* u, uint32_t* v, int64_t* lcs, int64_t* indel2,
                     uint32_t* nedges) {
  clear_error();
  if (!m || !nedges) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  FAMSA_HIP(hipSetDevice(m->device));
  int rc = m->wait_last();
  if (rc) return rc;
  MstDev::Ctl c;
  FAMSA_HIP(hipMemcpy(&c, m->ctl.p, sizeof c, hipMemcpyDeviceToHost));
  const uint32_t n = c.nf;
  std::vector<uint32_t> hu(n), hv(n), hl(m->k);
  std::vector<int32_t> hL(n);
  if (n) {
    FAMSA_HIP(hipMemcpy(hu.data(), m->fu.p, n * 4, hipMemcpyDeviceToHost));
    FAMSA_HIP(hipMemcpy(hv.data(), m->fv.p, n * 4, hipMemcpyDeviceToHost));
    FAMSA_HIP(hipMemcpy(hL.data(), m->fL.p, n * 4, hipMemcpyDeviceToHost));
  }
  if (m->k) FAMSA_HIP(hipMemcpy(hl.data(), m->len.p, (size_t)m->k * 4, hipMemcpyDeviceToHost));
  for (uint32_t e = 0; e < n; ++e) {
    if (u) u[e] = hu[e];
    if (v) v[e] = hv[e];
    if (lcs) lcs[e] = hL[e];
    const int64_t d = (int64_t)hl[hu[e]] + hl[hv[e]] - 2 * (int64_t)hL[e];
    if (indel2) indel2[e] = d * d;
  }
  *nedges = n;
  return 0;
}

int famsa_mst_guide_tree(const famsa_mst_t* m, uint32_t* left, uint32_t* right, int64_t* lcs, int64_t* indel2,
                         uint32_t* nmerges) {
  clear_error();
  if (!m || !nmerges) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  const size_t n = std::max<uint32_t>(m->k, 1);
  std::vector<uint32_t> u(n), v(n);
  std::vector<int64_t> L(n), D(n);
  uint32_t ne = 0;
  int rc = famsa_mst_result(m, u.data(), v.data(), L.data(), D.data(), &ne);
  if (rc) return rc;
  return guide_tree(m->k, u.data(), v.data(), L.data(), D.data(), ne, left, right, lcs, indel2, nmerges);
}

int famsa_mst_get_stats(const famsa_mst_t* m, uint64_t* tiles, uint64_t* rounds) {
  clear_error();
  if (!m) return set_error(FAMSA_LCS_EINVAL, "mst is NULL");
  FAMSA_HIP(hipSetDevice(m->device));
  int rc = m->wait_last();
  if (rc) return rc;
  MstDev::Ctl c;
  FAMSA_HIP(hipMemcpy(&c, m->ctl.p, sizeof c, hipMemcpyDeviceToHost));
  if (tiles) *tiles = m->tiles;
  if (rounds) *rounds = c.rounds;
  return 0;
}

void famsa_mst_destroy(famsa_mst_t* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  delete m;  // waits for the last tile's work
}

}  // extern "C"
