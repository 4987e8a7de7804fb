// Gapped sequence representation on the GPU (paper, Methods, "Progressive
// construction of the alignment", and Fig. 1).
//
// A sequence in a profile is kept as its symbols (with a guard at position
// 0), one gap counter per position -- the gap columns right after that
// position's symbol, so position 0 counts the leading gaps -- and a binary
// tree of column counts, the dynamic position statistics dps: with P the
// number of positions rounded up to a power of two, leaf P/2 + j counts the
// columns spanned by positions 2j and 2j+1 (a position spans its symbol and
// its gap run), and dps[v] = dps[2v] + dps[2v+1] above; dps[1] is the number
// of columns, guard included.  Column c of the sequence is found by walking
// down the tree, and inserting g gap columns before column c adds g to one
// counter and to the counts on the path back to the root: O(log n), whatever
// the number of sequences that move along.
//
// A batch (typically every sequence of a profile) lives in HBM as arrays of
// structures per sequence: symbols (uint8, guard 0xFF), counters (uint32)
// and tree (uint32), each sequence at its own offset.  Gap insertion runs one
// thread per sequence over the same list of runs, which is how a profile
// takes the gap columns of the other profile when two are merged.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "runtime.h"

namespace famsa {

struct GappedDev {
  uint8_t* sym;            // per position (guard 0xFF)
  uint32_t* gaps;          // per position
  uint32_t* dps;           // per tree node (index 0 unused)
  const uint64_t* pos_off; // first position of each sequence
  const uint64_t* tree_off;
  const uint32_t* npos;    // positions (guard + symbols)
  const uint32_t* ptree;   // P, a power of two >= 2
};

__device__ __forceinline__ uint32_t span_of(const GappedDev& g, uint64_t po, uint32_t npos, uint32_t p) {
  return p < npos ? 1u + g.gaps[po + p] : 0u;
}

// Column counts from the counters: leaves, then one tree level at a time.
__global__ __launch_bounds__(256) void gapped_rebuild(GappedDev g, uint32_t first) {
  const uint32_t s = first + blockIdx.x;
  const uint64_t po = g.pos_off[s], to = g.tree_off[s];
  const uint32_t npos = g.npos[s], P = g.ptree[s];
  for (uint32_t j = threadIdx.x; j < P / 2; j += blockDim.x)
    g.dps[to + P / 2 + j] = span_of(g, po, npos, 2 * j) + span_of(g, po, npos, 2 * j + 1);
  for (uint32_t lo = P / 4; lo >= 1; lo /= 2) {
    __syncthreads();
    for (uint32_t v = lo + threadIdx.x; v < 2 * lo; v += blockDim.x) g.dps[to + v] = g.dps[to + 2 * v] + g.dps[to + 2 * v + 1];
  }
}

// The position whose span holds column x (0 = the guard's column) and its leaf.
__device__ __forceinline__ uint32_t find_position(const GappedDev& g, uint64_t po, uint64_t to, uint32_t npos,
                                                  uint32_t P, uint32_t x, uint32_t* leaf) {
  uint32_t v = 1;
  while (v < P / 2) {
    const uint32_t l = g.dps[to + 2 * v];
    if (x < l) {
      v = 2 * v;
    } else {
      x -= l;
      v = 2 * v + 1;
    }
  }
  *leaf = v;
  const uint32_t p = 2 * (v - P / 2);
  return x < span_of(g, po, npos, p) ? p : p + 1;
}

// One thread per sequence applies every run, the rightmost first, so each
// run's column keeps the meaning it had before the call.
__global__ __launch_bounds__(256) void gapped_insert(GappedDev g, uint32_t first, uint32_t nseq,
                                                     const uint32_t* __restrict__ col,
                                                     const uint32_t* __restrict__ len, uint32_t nruns) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nseq) return;
  const uint32_t s = first + t;
  const uint64_t po = g.pos_off[s], to = g.tree_off[s];
  const uint32_t npos = g.npos[s], P = g.ptree[s];
  for (uint32_t r = nruns; r-- > 0;) {
    const uint32_t n = len[r];
    if (n == 0) continue;
    uint32_t leaf;
    // gaps before column c go right after whatever column c-1 belongs to
    const uint32_t p = find_position(g, po, to, npos, P, col[r] - 1u, &leaf);
    g.gaps[po + p] += n;
    for (uint32_t v = leaf; v >= 1; v /= 2) g.dps[to + v] += n;
  }
}

__global__ __launch_bounds__(256) void gapped_locate(GappedDev g, const uint32_t* __restrict__ seq,
                                                     const uint32_t* __restrict__ col, uint32_t nq,
                                                     uint32_t* __restrict__ out) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const uint32_t s = seq[q];
  uint32_t leaf;
  out[q] = find_position(g, g.pos_off[s], g.tree_off[s], g.npos[s], g.ptree[s], col[q], &leaf);
}

// One wave per sequence: positions in chunks of 64, their first columns by a
// wave prefix sum of the spans; each lane writes its symbol and its gap run.
// Row t of `out` holds columns 1.. of sequence first + t (the guard's column
// is left out); gaps are 0xFF, and the rest of the row is left as it is.
__global__ __launch_bounds__(64) void gapped_decode(GappedDev g, uint32_t first, uint8_t* __restrict__ out,
                                                    uint64_t row_bytes) {
  const uint32_t s = first + blockIdx.x, lane = threadIdx.x;
  const uint64_t po = g.pos_off[s];
  const uint32_t npos = g.npos[s];
  uint8_t* row = out + (uint64_t)blockIdx.x * row_bytes;
  uint32_t base = 0;  // first column of the chunk's first position
  for (uint32_t c0 = 0; c0 < npos; c0 += 64) {
    const uint32_t p = c0 + lane;
    const uint32_t sp = span_of(g, po, npos, p);
    uint32_t incl = sp;  // inclusive prefix over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= (uint32_t)d) incl += y;
    }
    const uint32_t c = base + incl - sp;  // column of position p's symbol
    if (p < npos) {
      if (p > 0) row[c - 1] = g.sym[po + p];
      for (uint32_t k = 1; k < sp; ++k) row[c + k - 1] = 0xFF;
    }
    base += __shfl(incl, 63, 64);
  }
}

}  // namespace famsa

using namespace famsa;

struct famsa_gapped_s {
  int device = 0;
  uint32_t nseq = 0;
  DevMem sym, gaps, dps, pos_off, tree_off, npos, ptree, runs, qbuf, obuf;
  std::vector<uint32_t> h_npos, h_ptree, h_width;  // width = columns, guard included
  std::vector<uint64_t> h_pos_off, h_tree_off;
  hipStream_t s = nullptr;
  GappedDev view() const {
    return GappedDev{sym.as<uint8_t>(), gaps.as<uint32_t>(), dps.as<uint32_t>(), pos_off.as<uint64_t>(),
                     tree_off.as<uint64_t>(), npos.as<uint32_t>(), ptree.as<uint32_t>()};
  }
};

extern "C" {

int famsa_gapped_create(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, int device,
                        famsa_gapped_t** out) {
  clear_error();
  if (!out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!seq_off) return set_error(FAMSA_LCS_EINVAL, "seq_off is NULL");
  if (device < 0) return set_error(FAMSA_LCS_EINVAL, "device %d < 0", device);
  uint64_t total_pos = 0, total_tree = 0;
  for (uint32_t i = 0; i < nseq; ++i) {
    if (seq_off[i + 1] < seq_off[i]) return set_error(FAMSA_LCS_EINVAL, "seq_off decreases at %u", i);
    const uint64_t n = seq_off[i + 1] - seq_off[i];
    if (n > FAMSA_LCS_MAX_LEN) return set_error(FAMSA_LCS_EINVAL, "sequence %u has %llu > %u symbols", i,
                                                (unsigned long long)n, FAMSA_LCS_MAX_LEN);
    total_pos += n + 1;
  }
  if (seq_off[nseq] > seq_off[0] && !codes) return set_error(FAMSA_LCS_EINVAL, "codes is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return set_error(FAMSA_LCS_EDEVICE, "no HIP device available");
  }
  if (device >= ndev) return set_error(FAMSA_LCS_EINVAL, "device %d >= device count %d", device, ndev);
  FAMSA_HIP(hipSetDevice(device));
  famsa_gapped_s* g = new (std::nothrow) famsa_gapped_s();
  if (!g) return set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  g->device = device;
  g->nseq = nseq;
  g->h_npos.resize(nseq);
  g->h_ptree.resize(nseq);
  g->h_width.resize(nseq);
  g->h_pos_off.resize(nseq + 1);
  g->h_tree_off.resize(nseq + 1);
  std::vector<uint8_t> hsym(std::max<uint64_t>(total_pos, 1));
  uint64_t po = 0, to = 0;
  for (uint32_t i = 0; i < nseq; ++i) {
    const uint32_t n = (uint32_t)(seq_off[i + 1] - seq_off[i]);
    uint32_t P = 2;
    while (P < n + 1) P *= 2;
    g->h_npos[i] = n + 1;
    g->h_ptree[i] = P;
    g->h_width[i] = n + 1;
    g->h_pos_off[i] = po;
    g->h_tree_off[i] = to;
    hsym[po] = 0xFF;
    if (n) memcpy(&hsym[po + 1], codes + seq_off[i], n);
    po += n + 1;
    to += P;
  }
  g->h_pos_off[nseq] = po;
  g->h_tree_off[nseq] = to;
  total_tree = to;
  int rc;
  hipStream_t st = nullptr;
  if ((rc = lib_stream(device, 0, &st))) {
    delete g;
    return rc;
  }
  g->s = st;
  if ((rc = upload(g->sym, hsym, st)) || (rc = g->gaps.alloc(std::max<uint64_t>(total_pos, 1) * 4)) ||
      (rc = g->dps.alloc(std::max<uint64_t>(total_tree, 1) * 4)) || (rc = upload(g->pos_off, g->h_pos_off, st)) ||
      (rc = upload(g->tree_off, g->h_tree_off, st)) || (rc = upload(g->npos, g->h_npos, st)) ||
      (rc = upload(g->ptree, g->h_ptree, st))) {
    delete g;
    return rc;
  }
  if (hipMemsetAsync(g->gaps.p, 0, std::max<uint64_t>(total_pos, 1) * 4, st) != hipSuccess) {
    delete g;
    return set_error(FAMSA_LCS_EDEVICE, "clearing gap counters failed");
  }
  if (nseq) hipLaunchKernelGGL(gapped_rebuild, dim3(nseq), dim3(256), 0, st, g->view(), 0u);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    delete g;
    return set_error(FAMSA_LCS_EDEVICE, "building the position trees failed");
  }
  *out = g;
  return 0;
}

int famsa_gapped_insert(famsa_gapped_t* g, uint32_t first, uint32_t count, const uint32_t* col, const uint32_t* len,
                        uint32_t nruns) {
  clear_error();
  if (!g) return set_error(FAMSA_LCS_EINVAL, "gapped is NULL");
  if (first > g->nseq || count > g->nseq - first) return set_error(FAMSA_LCS_EINVAL, "sequences out of range");
  if (nruns && (!col || !len)) return set_error(FAMSA_LCS_EINVAL, "NULL run array");
  if (!count || !nruns) return 0;
  uint64_t add = 0;
  for (uint32_t r = 0; r < nruns; ++r) {
    if (col[r] < 1) return set_error(FAMSA_LCS_EINVAL, "run %u: column %u < 1", r, col[r]);
    if (r && col[r] < col[r - 1]) return set_error(FAMSA_LCS_EINVAL, "runs are not sorted by column");
    add += len[r];
  }
  for (uint32_t i = first; i < first + count; ++i) {
    if (col[nruns - 1] > g->h_width[i])
      return set_error(FAMSA_LCS_EINVAL, "run column %u beyond sequence %u's %u columns", col[nruns - 1], i,
                       g->h_width[i]);
    if (g->h_width[i] + add > 0xFFFFFFFFull) return set_error(FAMSA_LCS_EINVAL, "sequence %u too wide", i);
  }
  FAMSA_HIP(hipSetDevice(g->device));
  std::vector<uint32_t> h(2 * (size_t)nruns);
  memcpy(h.data(), col, nruns * 4);
  memcpy(h.data() + nruns, len, nruns * 4);
  int rc;
  if (g->runs.bytes < h.size() * 4 && (rc = g->runs.alloc(h.size() * 4))) return rc;
  FAMSA_HIP(hipMemcpyAsync(g->runs.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, g->s));
  const uint32_t* d = g->runs.as<uint32_t>();
  hipLaunchKernelGGL(gapped_insert, dim3((count + 255) / 256), dim3(256), 0, g->s, g->view(), first, count, d,
                     d + nruns, nruns);
  FAMSA_HIP(hipGetLastError());
  FAMSA_HIP(hipStreamSynchronize(g->s));
  for (uint32_t i = first; i < first + count; ++i) g->h_width[i] += (uint32_t)add;
  return 0;
}

int famsa_gapped_width(const famsa_gapped_t* g, uint32_t* width) {
  clear_error();
  if (!g || !width) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  for (uint32_t i = 0; i < g->nseq; ++i) width[i] = g->h_width[i] - 1;
  return 0;
}

int famsa_gapped_locate(famsa_gapped_t* g, const uint32_t* seq, const uint32_t* col, uint32_t nq, uint32_t* pos) {
  clear_error();
  if (!g) return set_error(FAMSA_LCS_EINVAL, "gapped is NULL");
  if (!nq) return 0;
  if (!seq || !col || !pos) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  for (uint32_t q = 0; q < nq; ++q) {
    if (seq[q] >= g->nseq) return set_error(FAMSA_LCS_EINVAL, "query %u: sequence %u out of range", q, seq[q]);
    if (col[q] >= g->h_width[seq[q]]) return set_error(FAMSA_LCS_EINVAL, "query %u: column %u out of range", q, col[q]);
  }
  FAMSA_HIP(hipSetDevice(g->device));
  int rc;
  if (g->qbuf.bytes < (size_t)nq * 12 && (rc = g->qbuf.alloc((size_t)nq * 12))) return rc;
  uint32_t* d = g->qbuf.as<uint32_t>();
  FAMSA_HIP(hipMemcpyAsync(d, seq, (size_t)nq * 4, hipMemcpyHostToDevice, g->s));
  FAMSA_HIP(hipMemcpyAsync(d + nq, col, (size_t)nq * 4, hipMemcpyHostToDevice, g->s));
  hipLaunchKernelGGL(gapped_locate, dim3((nq + 255) / 256), dim3(256), 0, g->s, g->view(), d, d + nq, nq, d + 2 * (size_t)nq);
  FAMSA_HIP(hipGetLastError());
  FAMSA_HIP(hipMemcpyAsync(pos, d + 2 * (size_t)nq, (size_t)nq * 4, hipMemcpyDeviceToHost, g->s));
  FAMSA_HIP(hipStreamSynchronize(g->s));
  return 0;
}

int famsa_gapped_decode(famsa_gapped_t* g, uint32_t first, uint32_t count, uint8_t* out, uint64_t row_bytes) {
  clear_error();
  if (!g) return set_error(FAMSA_LCS_EINVAL, "gapped is NULL");
  if (first > g->nseq || count > g->nseq - first) return set_error(FAMSA_LCS_EINVAL, "sequences out of range");
  if (!count) return 0;
  if (!out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  for (uint32_t i = first; i < first + count; ++i)
    if (g->h_width[i] - 1 > row_bytes)
      return set_error(FAMSA_LCS_EINVAL, "sequence %u has %u columns, more than row_bytes %llu", i, g->h_width[i] - 1,
                       (unsigned long long)row_bytes);
  FAMSA_HIP(hipSetDevice(g->device));
  const uint64_t bytes = (uint64_t)count * row_bytes;
  int rc;
  if (g->obuf.bytes < bytes && (rc = g->obuf.alloc(bytes))) return rc;
  hipLaunchKernelGGL(gapped_decode, dim3(count), dim3(64), 0, g->s, g->view(), first, g->obuf.as<uint8_t>(), row_bytes);
  FAMSA_HIP(hipGetLastError());
  FAMSA_HIP(hipMemcpyAsync(out, g->obuf.p, bytes, hipMemcpyDeviceToHost, g->s));
  FAMSA_HIP(hipStreamSynchronize(g->s));
  return 0;
}

int famsa_gapped_state(famsa_gapped_t* g, uint32_t s, uint32_t* no_gaps, uint32_t* dps, uint32_t* npos,
                       uint32_t* ptree) {
  clear_error();
  if (!g) return set_error(FAMSA_LCS_EINVAL, "gapped is NULL");
  if (s >= g->nseq) return set_error(FAMSA_LCS_EINVAL, "sequence %u out of range", s);
  if (npos) *npos = g->h_npos[s];
  if (ptree) *ptree = g->h_ptree[s];
  FAMSA_HIP(hipSetDevice(g->device));
  FAMSA_HIP(hipStreamSynchronize(g->s));
  if (no_gaps)
    FAMSA_HIP(hipMemcpy(no_gaps, g->gaps.as<uint32_t>() + g->h_pos_off[s], (size_t)g->h_npos[s] * 4,
                        hipMemcpyDeviceToHost));
  if (dps)
    FAMSA_HIP(hipMemcpy(dps, g->dps.as<uint32_t>() + g->h_tree_off[s], (size_t)g->h_ptree[s] * 4,
                        hipMemcpyDeviceToHost));
  return 0;
}

void famsa_gapped_destroy(famsa_gapped_t* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->s) (void)hipStreamSynchronize(g->s);
  delete g;
}

}  // extern "C"
