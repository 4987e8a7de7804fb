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
  uint64_t* wkey;     // best forest edge per vertex (merged into vkey/vid/vL after the forest pass)
  uint64_t* wid;
  int32_t* wL;
  uint64_t* ckey;     // best outgoing edge per component
  uint64_t* cid;
  int32_t* cL;
  const uint32_t* fu;  // current forest edges
  const uint32_t* fv;
  const int32_t* fL;
  uint32_t nf;
  uint32_t* nu;        // new forest edges
  uint32_t* nv;
  int32_t* nL;
  uint32_t* counters;  // [0] new forest size, [1] hooks this round
};

__global__ void mst_reset_vertices(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k) return;
  m.vkey[v] = 0;
  m.vid[v] = ~0ull;
  m.vL[v] = 0;
  m.wkey[v] = 0;
  m.wid[v] = ~0ull;
  m.wL[v] = 0;
  m.ckey[v] = 0;
  m.cid[v] = ~0ull;
}

__global__ void mst_init_components(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k) return;
  m.comp[v] = v;
  m.parent[v] = v;
}

// Row pass: one block per tile row i, best edge (i, j), j > i, leaving i's component.
__global__ __launch_bounds__(256) void mst_rows(MstDev m, const int32_t* __restrict__ tile, uint32_t r0, uint32_t r1) {
  const uint32_t i = r0 + blockIdx.x;
  if (i >= r1) return;
  const uint64_t k = m.k;
  const uint64_t off = (i - r0) * (k - 1) - ((uint64_t)(r0 + i - 1) * (i - r0)) / 2;  // rows before i in the tile
  const uint32_t ci = m.comp[i], li = m.len[i];
  uint64_t bk = 0, bi = ~0ull;
  int32_t bL = 0;
  for (uint32_t j = i + 1 + threadIdx.x; j < m.k; j += blockDim.x) {
    if (m.comp[j] == ci) continue;
    const int32_t L = tile[off + (j - i - 1)];
    const uint64_t key = sim_key(L, li, m.len[j]);
    const uint64_t id = (uint64_t)i * k + j;
    if (better(key, id, bk, bi)) {
      bk = key;
      bi = id;
      bL = L;
    }
  }
  __shared__ uint64_t sk[256], si[256];
  __shared__ int32_t sL[256];
  sk[threadIdx.x] = bk;
  si[threadIdx.x] = bi;
  sL[threadIdx.x] = bL;
  __syncthreads();
  for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && better(sk[threadIdx.x + s], si[threadIdx.x + s], sk[threadIdx.x], si[threadIdx.x])) {
      sk[threadIdx.x] = sk[threadIdx.x + s];
      si[threadIdx.x] = si[threadIdx.x + s];
      sL[threadIdx.x] = sL[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && better(sk[0], si[0], m.vkey[i], m.vid[i])) {
    m.vkey[i] = sk[0];
    m.vid[i] = si[0];
    m.vL[i] = sL[0];
  }
}

// Column pass: one thread per column j > r0, best edge (i, j) over tile rows i < j.
__global__ __launch_bounds__(256) void mst_cols(MstDev m, const int32_t* __restrict__ tile, uint32_t r0, uint32_t r1) {
  const uint32_t j = r0 + 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.k) return;
  const uint64_t k = m.k;
  const uint32_t cj = m.comp[j], lj = m.len[j];
  uint64_t bk = m.vkey[j], bi = m.vid[j];
  int32_t bL = m.vL[j];
  const uint32_t iend = j < r1 ? j : r1;
  uint64_t off = 0;  // start of row i in the tile
  for (uint32_t i = r0; i < iend; ++i) {
    if (m.comp[i] != cj) {
      const int32_t L = tile[off + (j - i - 1)];
      const uint64_t key = sim_key(L, m.len[i], lj);
      const uint64_t id = (uint64_t)i * k + j;
      if (better(key, id, bk, bi)) {
        bk = key;
        bi = id;
        bL = L;
      }
    }
    off += k - 1 - i;
  }
  m.vkey[j] = bk;
  m.vid[j] = bi;
  m.vL[j] = bL;
}

// Forest edges: candidates for both ends, gathered in the w* slots in three
// phases (key, id, LCS), then merged with the tile's candidates.
__global__ void mst_forest_key(MstDev m) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nf) return;
  const uint32_t u = m.fu[e], v = m.fv[e];
  if (m.comp[u] == m.comp[v]) return;
  const uint64_t key = sim_key(m.fL[e], m.len[u], m.len[v]);
  atomicMax((unsigned long long*)&m.wkey[u], (unsigned long long)key);
  atomicMax((unsigned long long*)&m.wkey[v], (unsigned long long)key);
}

__global__ void mst_forest_id(MstDev m) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nf) return;
  const uint32_t u = m.fu[e], v = m.fv[e];
  if (m.comp[u] == m.comp[v]) return;
  const uint64_t key = sim_key(m.fL[e], m.len[u], m.len[v]);
  const uint64_t id = (uint64_t)u * m.k + v;
  if (m.wkey[u] == key) atomicMin((unsigned long long*)&m.wid[u], (unsigned long long)id);
  if (m.wkey[v] == key) atomicMin((unsigned long long*)&m.wid[v], (unsigned long long)id);
}

__global__ void mst_forest_L(MstDev m) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nf) return;
  const uint32_t u = m.fu[e], v = m.fv[e];
  if (m.comp[u] == m.comp[v]) return;
  const uint64_t id = (uint64_t)u * m.k + v;
  if (m.wid[u] == id) m.wL[u] = m.fL[e];
  if (m.wid[v] == id) m.wL[v] = m.fL[e];
}

__global__ void mst_forest_merge(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k || m.wkey[v] == 0) return;
  if (better(m.wkey[v], m.wid[v], m.vkey[v], m.vid[v])) {
    m.vkey[v] = m.wkey[v];
    m.vid[v] = m.wid[v];
    m.vL[v] = m.wL[v];
  }
}

__global__ void mst_comp_key(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k || m.vkey[v] == 0) return;
  atomicMax((unsigned long long*)&m.ckey[m.comp[v]], (unsigned long long)m.vkey[v]);
}

__global__ void mst_comp_id(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k || m.vkey[v] == 0) return;
  const uint32_t c = m.comp[v];
  if (m.vkey[v] == m.ckey[c]) atomicMin((unsigned long long*)&m.cid[c], (unsigned long long)m.vid[v]);
}

__global__ void mst_comp_L(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k || m.vkey[v] == 0) return;
  const uint32_t c = m.comp[v];
  if (m.vkey[v] == m.ckey[c] && m.vid[v] == m.cid[c]) m.cL[c] = m.vL[v];  // one vertex per component matches
}

// Hook every component with an outgoing edge onto the component at its other
// end.  Two components that chose the same edge hook once: the larger onto
// the smaller.  Each hook adds its edge to the new forest.
__global__ void mst_hook(MstDev m) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m.k || m.comp[c] != c || m.ckey[c] == 0) return;
  const uint64_t id = m.cid[c];
  const uint32_t u = (uint32_t)(id / m.k), v = (uint32_t)(id % m.k);
  const uint32_t d = m.comp[u] == c ? m.comp[v] : m.comp[u];
  if (m.cid[d] == id && c < d) return;  // mutual choice: d hooks onto c
  m.parent[c] = d;
  const uint32_t slot = atomicAdd(&m.counters[0], 1u);
  m.nu[slot] = u;
  m.nv[slot] = v;
  m.nL[slot] = m.cL[c];
  atomicAdd(&m.counters[1], 1u);
}

// Every component follows its hook chain to the root (chains are acyclic:
// with a strict order on edges the only cycles of chosen edges are the mutual
// pairs, which hook once).  Concurrent shortcuts by other threads only move
// entries further up the same chain.
__global__ void mst_jump(MstDev m) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m.k) return;
  uint32_t r = m.parent[c];
  while (m.parent[r] != r) r = m.parent[r];
  m.parent[c] = r;
}

__global__ void mst_relabel(MstDev m) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.k) return;
  m.comp[v] = m.parent[m.comp[v]];
}

__global__ void mst_zero(uint32_t* p, uint32_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace famsa

using namespace famsa;

struct famsa_mst_s {
  uint32_t k = 0;
  int device = 0;
  DevMem len, comp, parent, vkey, vid, vL, wkey, wid, wL, ckey, cid, cL, fu, fv, fL, nu, nv, nL, counters;
  PinMem hcount;
  uint32_t nf = 0;
  uint64_t tiles = 0, rounds = 0;
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
    m.cL = cL.as<int32_t>();
    m.fu = fu.as<uint32_t>();
    m.fv = fv.as<uint32_t>();
    m.fL = fL.as<int32_t>();
    m.nf = nf;
    m.nu = nu.as<uint32_t>();
    m.nv = nv.as<uint32_t>();
    m.nL = nL.as<int32_t>();
    m.counters = counters.as<uint32_t>();
    return m;
  }
  int merge_tile(const famsa_lcs_tile* t, hipStream_t s);
};

static inline dim3 grid_for(uint64_t n, uint32_t b = 256) { return dim3((uint32_t)((n + b - 1) / b)); }

int famsa_mst_s::merge_tile(const famsa_lcs_tile* t, hipStream_t s) {
  const uint32_t r0 = t->row_begin, r1 = t->row_end;
  const dim3 gk = grid_for(k);
  uint32_t* hc = hcount.as<uint32_t>();
  MstDev m = view();
  hipLaunchKernelGGL(mst_init_components, gk, dim3(256), 0, s, m);
  hipLaunchKernelGGL(mst_zero, dim3(1), dim3(64), 0, s, m.counters, 4u);
  for (;;) {
    m = view();
    hipLaunchKernelGGL(mst_reset_vertices, gk, dim3(256), 0, s, m);
    if (t->count && r1 > r0) {
      hipLaunchKernelGGL(mst_rows, dim3(r1 - r0), dim3(256), 0, s, m, t->lcs, r0, r1);
      if (r0 + 1 < k) hipLaunchKernelGGL(mst_cols, grid_for(k - r0 - 1), dim3(256), 0, s, m, t->lcs, r0, r1);
    }
    if (nf) {
      hipLaunchKernelGGL(mst_forest_key, grid_for(nf), dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_forest_id, grid_for(nf), dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_forest_L, grid_for(nf), dim3(256), 0, s, m);
      hipLaunchKernelGGL(mst_forest_merge, gk, dim3(256), 0, s, m);
    }
    hipLaunchKernelGGL(mst_comp_key, gk, dim3(256), 0, s, m);
    hipLaunchKernelGGL(mst_comp_id, gk, dim3(256), 0, s, m);
    hipLaunchKernelGGL(mst_comp_L, gk, dim3(256), 0, s, m);
    hipLaunchKernelGGL(mst_hook, gk, dim3(256), 0, s, m);
    FAMSA_HIP(hipGetLastError());
    hipLaunchKernelGGL(mst_jump, gk, dim3(256), 0, s, m);
    hipLaunchKernelGGL(mst_relabel, gk, dim3(256), 0, s, m);
    FAMSA_HIP(hipGetLastError());
    FAMSA_HIP(hipMemcpyAsync(hc, m.counters, 8, hipMemcpyDeviceToHost, s));
    FAMSA_HIP(hipStreamSynchronize(s));
    ++rounds;
    const uint32_t hooks = hc[1];
    hipLaunchKernelGGL(mst_zero, dim3(1), dim3(64), 0, s, m.counters + 1, 1u);  // hooks of the next round
    if (hooks == 0) break;
  }
  // the new forest replaces the old one
  FAMSA_HIP(hipMemcpyAsync(hc, m.counters, 4, hipMemcpyDeviceToHost, s));
  FAMSA_HIP(hipStreamSynchronize(s));
  nf = hc[0];
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
      (rc = m->ckey.alloc(n * 8)) || (rc = m->cid.alloc(n * 8)) || (rc = m->cL.alloc(n * 4)) ||
      (rc = m->fu.alloc(n * 4)) || (rc = m->fv.alloc(n * 4)) || (rc = m->fL.alloc(n * 4)) ||
      (rc = m->nu.alloc(n * 4)) || (rc = m->nv.alloc(n * 4)) || (rc = m->nL.alloc(n * 4)) ||
      (rc = m->counters.alloc(16)) || (rc = m->hcount.alloc(16))) {
    delete m;
    return rc;
  }
  if (k && hipMemcpy(m->len.p, lengths, (size_t)k * 4, hipMemcpyHostToDevice) != hipSuccess) {
    delete m;
    return set_error(FAMSA_LCS_EDEVICE, "copying lengths failed");
  }
  *out = m;
  return 0;
}

int famsa_mst_consume(void* user, const famsa_lcs_tile* t) {
  famsa_mst_s* m = static_cast<famsa_mst_s*>(user);
  if (!m || !t || t->k != m->k || t->row_begin > t->row_end || t->row_end > m->k) return 1;
  if (t->count && !t->lcs) return 1;
  if (t->count != tri_rows(m->k, t->row_begin, t->row_end)) return 1;
  if (hipSetDevice(m->device) != hipSuccess) return 1;
  return m->merge_tile(t, (hipStream_t)t->stream) == 0 ? 0 : 1;
}

int famsa_mst_result(const famsa_mst_t* m, uint32_t* u, uint32_t* v, int64_t* lcs, int64_t* indel2,
                     uint32_t* nedges) {
  clear_error();
  if (!m || !nedges) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  FAMSA_HIP(hipSetDevice(m->device));
  FAMSA_HIP(hipDeviceSynchronize());
  const uint32_t n = m->nf;
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

void famsa_mst_destroy(famsa_mst_t* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  delete m;
}

}  // extern "C"
