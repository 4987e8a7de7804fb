// famsa_lcs_family_noalloc: the LCS of every pair of one family, from device
// inputs into a device output, with no allocation of any kind.
//
// The plan path (famsa_lcs_plan / famsa_lcs_tiles) allocates its device
// batch, work lists, queue counters and step buffers, and plans the work on
// the host.  Here every one of those lives in `scratch`, one file-scope
// device array of fixed size per GPU, and the planning runs on the device:
//   na_plan_kernel   -- one workgroup: lengths and offsets checked, rows
//                       sorted by length (bitonic sort in LDS), the family
//                       mode work lists of the plan path (64-row groups,
//                       column items, class ranges) and the queue counters;
//   na_stage_kernel  -- a workgroup per sequence: codes checked, the
//                       column stream (code c stored as c * 1024) and the
//                       match masks PM[c][w] written into the sequence's slot;
//   lcs_fast_kernel  -- the plan path's own kernels, classes 2, 1, 0;
//   na_finish_kernel -- status word; every output set to -1 on invalid input.
// Results are the plan path's bit for bit (same kernels, same recurrence).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "runtime.h"

namespace famsa {
namespace {

constexpr uint32_t kNaMaxSeq = FAMSA_LCS_NOALLOC_MAX_SEQ;
constexpr uint32_t kNaMaxGroups = kNaMaxSeq / kLanes;
constexpr uint32_t kNaMaxItems = 8192;  // the item count never exceeds 4480 (columns per item >= span / 4096)
constexpr uint32_t kNaMaxLen20 = FAMSA_LCS_NOALLOC_MAX_LEN;      // 28 dwords: the fast classes for sigma <= 20
constexpr uint32_t kNaMaxLen32 = FAMSA_LCS_NOALLOC_MAX_LEN_S32;  // 16 dwords: class 2 holds 4 quads of 32 planes
constexpr uint32_t kNaSymSlot = 2 * kNaMaxLen20 + 16;  // bytes: uint16 per residue and the spare chunk
constexpr uint32_t kNaMaskSlot = 20 * 28;               // dwords: >= 20 x 28 and >= 32 x 16
constexpr int kNaMaxDevices = 64;
constexpr uint32_t kNaPlanThreads = 1024;

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffCtl = 0;    // StepCtl
constexpr size_t kOffErr = 64;   // uint32: 0 valid, nonzero invalid input
constexpr size_t kOffRange = 128;  // StepRange of the one step
constexpr size_t kOffGroups = 256;
constexpr size_t kOffLanes = align256(kOffGroups + sizeof(GroupDesc) * kNaMaxGroups);
constexpr size_t kOffItems = align256(kOffLanes + sizeof(LaneDesc) * kNaMaxSeq);
constexpr size_t kOffColmap = align256(kOffItems + sizeof(ItemDesc) * kNaMaxItems);
constexpr size_t kOffRowbase = align256(kOffColmap + sizeof(uint32_t) * kNaMaxSeq);
constexpr size_t kOffLen = align256(kOffRowbase + sizeof(uint64_t) * kNaMaxSeq);
constexpr size_t kOffSymOff = align256(kOffLen + sizeof(uint32_t) * kNaMaxSeq);
constexpr size_t kOffMaskOff = align256(kOffSymOff + sizeof(uint64_t) * kNaMaxSeq);
constexpr size_t kOffSym = align256(kOffMaskOff + sizeof(uint64_t) * kNaMaxSeq);
constexpr size_t kOffMasks = align256(kOffSym + (size_t)kNaSymSlot * kNaMaxSeq);
constexpr size_t kNaBytes = align256(kOffMasks + sizeof(uint32_t) * kNaMaskSlot * kNaMaxSeq);
static_assert(kNaBytes == FAMSA_LCS_NOALLOC_SCRATCH_BYTES, "header states the scratch size");
static_assert(kNaSymSlot % 16 == 0, "column streams are read in 16-byte chunks");
static_assert(sizeof(StepCtl) <= 64 && sizeof(StepRange) <= 128, "control block layout");

// Each GPU holds its own copy.  Host code never passes this name to a kernel:
// it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[kNaBytes];

struct NaView {  // device addresses inside one GPU's scratch
  uint8_t* base;
  StepCtl* ctl() const { return reinterpret_cast<StepCtl*>(base + kOffCtl); }
  StepRange* range() const { return reinterpret_cast<StepRange*>(base + kOffRange); }
};

__device__ __forceinline__ uint32_t* na_err(uint8_t* base) { return reinterpret_cast<uint32_t*>(base + kOffErr); }

__device__ __forceinline__ void na_empty_ranges(uint8_t* base) {
  StepRange* r = reinterpret_cast<StepRange*>(base + kOffRange);
  for (int c = 0; c < 5; ++c) {
    r->begin[c] = 0;
    r->end[c] = 0;
  }
  r->plain_pairs = 0;
}

// One workgroup.  Rows sorted longest first (ties by index, as the plan
// path's stable sort); groups of 64 consecutive sorted rows; group g's rows
// need the column positions after their own, [64g + 1, k), cut into items
// of C columns; column position q is sequence colmap[q], and a pair lands in
// the upper-triangle row of its smaller index.
__global__ __launch_bounds__(kNaPlanThreads) void na_plan_kernel(const uint64_t* __restrict__ seq_off, uint32_t k,
                                                                 uint32_t maxlen, uint8_t* __restrict__ base) {
  __shared__ uint32_t key[kNaMaxSeq];
  __shared__ uint32_t s_first[kNaMaxGroups + 1];
  __shared__ uint32_t s_err, s_C;
  uint32_t* len = reinterpret_cast<uint32_t*>(base + kOffLen);
  uint64_t* sym_off = reinterpret_cast<uint64_t*>(base + kOffSymOff);
  uint64_t* mask_off = reinterpret_cast<uint64_t*>(base + kOffMaskOff);
  uint32_t* colmap = reinterpret_cast<uint32_t*>(base + kOffColmap);
  uint64_t* rowbase = reinterpret_cast<uint64_t*>(base + kOffRowbase);
  LaneDesc* lanes = reinterpret_cast<LaneDesc*>(base + kOffLanes);
  GroupDesc* groups = reinterpret_cast<GroupDesc*>(base + kOffGroups);
  ItemDesc* items = reinterpret_cast<ItemDesc*>(base + kOffItems);
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_err = 0;
  __syncthreads();
  uint32_t N = 1;
  while (N < k) N <<= 1;
  for (uint32_t i = tid; i < N; i += kNaPlanThreads) {
    uint32_t kk = 0xFFFFFFFFu;
    if (i < k) {
      const uint64_t a = seq_off[i], b = seq_off[i + 1];
      uint32_t L = 0;
      if (b < a || b - a > maxlen) atomicOr(&s_err, 1u);
      else L = (uint32_t)(b - a);
      len[i] = L;
      sym_off[i] = (uint64_t)i * kNaSymSlot;
      mask_off[i] = (uint64_t)i * kNaMaskSlot;
      kk = ((1023u - L) << 13) | i;  // L <= 896 < 1024, i < 8192
    }
    key[i] = kk;
  }
  __syncthreads();
  for (uint32_t size = 2; size <= N; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = tid; t < N / 2; t += kNaPlanThreads) {
        const uint32_t i = 2 * t - (t & (stride - 1));  // bit `stride` of i is clear
        const uint32_t j = i + stride;
        const uint32_t a = key[i], b = key[j];
        if ((a > b) == ((i & size) == 0)) {
          key[i] = b;
          key[j] = a;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t q = tid; q < k; q += kNaPlanThreads) {
    const uint32_t a = key[q] & 0x1FFFu;
    const uint64_t ro = (uint64_t)a * k - (uint64_t)a * (a + 1) / 2;  // offset of pair (a, a + 1)
    colmap[q] = a;
    rowbase[q] = ro;
    LaneDesc d;
    d.out_off = ro;
    d.seq = a;
    d.pos = q;
    d.orig = a;
    d.pad = 0;
    lanes[q] = d;
  }
  const uint32_t G = k >= 2 ? (k - 2) / kLanes + 1 : 0;  // groups with a pair: 64 g + 1 < k
  if (tid == 0) {
    uint64_t span = 0;
    for (uint32_t g = 0; g < G; ++g) span += k - (kLanes * g + 1);
    uint32_t C = 256;
    if (span / C < 4096) C = (uint32_t)max<uint64_t>(16, min<uint64_t>(C, span / 4096));
    uint32_t n = 0, cnt[3] = {0, 0, 0};
    for (uint32_t g = 0; g < G; ++g) {
      const uint32_t P = kLanes * g;
      const uint32_t L = 1023u - (key[P] >> 13);
      const uint32_t W = max(1u, (L + 31u) >> 5);
      const uint32_t Q = (W + 3u) >> 2;
      const int cls = Q <= (uint32_t)kClassQMax[0] ? 0 : (Q <= (uint32_t)kClassQMax[1] ? 1 : 2);
      GroupDesc gd;
      gd.lane_first = P;
      gd.nrows = min((uint32_t)kLanes, k - P);
      gd.W = W;
      gd.fam_base = 0;
      gd.colmap_base = 0;
      gd.rowbase_base = 0;
      gd.nmap = k;
      gd.shift = 0;
      gd.lpr = 0;
      gd.pad[0] = gd.pad[1] = gd.pad[2] = 0;
      groups[g] = gd;
      const uint32_t ni = (k - P - 1 + C - 1) / C;
      s_first[g] = n;
      n += ni;
      cnt[cls] += ni;  // classes do not increase with g: rows are sorted longest first
    }
    s_first[G] = n;
    s_C = C;
    if (n > kNaMaxItems) s_err |= 4u;
    StepRange* r = reinterpret_cast<StepRange*>(base + kOffRange);
    r->begin[2] = 0;
    r->end[2] = cnt[2];
    r->begin[1] = cnt[2];
    r->end[1] = cnt[2] + cnt[1];
    r->begin[0] = cnt[2] + cnt[1];
    r->end[0] = n;
    r->begin[3] = r->end[3] = n;
    r->begin[4] = r->end[4] = 0;
    r->plain_pairs = 0;
    if (s_err) na_empty_ranges(base);
    StepCtl* ctl = reinterpret_cast<StepCtl*>(base + kOffCtl);
    ctl->step = 0;
    ctl->next_step = 0;
    ctl->stride = 0;
    ctl->pad = 0;
    for (int c = 0; c < 4; ++c) ctl->cursor[c] = 0;
    *na_err(base) = s_err;
  }
  __syncthreads();
  if (s_err) return;
  const uint32_t C = s_C;
  for (uint32_t g = 0; g < G; ++g) {
    const uint32_t f = s_first[g], ni = s_first[g + 1] - f, c0 = kLanes * g + 1;
    for (uint32_t t = tid; t < ni; t += kNaPlanThreads) {
      ItemDesc it;
      it.group = g;
      it.c0 = c0 + t * C;
      it.c1 = min(k, it.c0 + C);
      it.pad = 0;
      items[f + t] = it;
    }
  }
}

// A workgroup per sequence: its column stream and its match masks
// (bit p of PM[c][w] set iff residue 32 w + p equals c; zero past the end).
__global__ __launch_bounds__(256) void na_stage_kernel(const uint8_t* __restrict__ codes,
                                                       const uint64_t* __restrict__ seq_off, uint32_t sigma,
                                                       uint8_t* __restrict__ base) {
  if (*na_err(base)) return;  // lengths or offsets were rejected: nothing to stage
  const uint32_t s = blockIdx.x, tid = threadIdx.x;
  const uint32_t L = reinterpret_cast<const uint32_t*>(base + kOffLen)[s];
  const uint8_t* src = codes + seq_off[s];
  uint16_t* sym = reinterpret_cast<uint16_t*>(base + kOffSym + (size_t)s * kNaSymSlot);
  bool bad = false;
  for (uint32_t p = tid; p < L; p += blockDim.x) {
    const uint32_t c = src[p];
    bad |= c >= sigma;
    sym[p] = (uint16_t)(c * 1024u);
  }
  const uint32_t W = (L + 31u) >> 5;
  if (tid < W) {
    uint32_t cp[32];
#pragma unroll
    for (int p = 0; p < 32; ++p) {
      const uint32_t pos = 32u * tid + (uint32_t)p;
      cp[p] = pos < L ? (uint32_t)src[pos] : 0xFFFFFFFFu;
    }
    uint32_t* m = reinterpret_cast<uint32_t*>(base + kOffMasks) + (size_t)s * kNaMaskSlot + tid;
    for (uint32_t c = 0; c < sigma; ++c) {
      uint32_t x = 0;
#pragma unroll
      for (int p = 0; p < 32; ++p) x |= (cp[p] == c ? 1u : 0u) << p;
      m[(size_t)c * W] = x;
    }
  }
  if (bad) {  // a code outside the alphabet: no LCS kernel may run
    atomicOr(na_err(base), 2u);
    na_empty_ranges(base);
  }
}

__global__ __launch_bounds__(256) void na_finish_kernel(const uint8_t* __restrict__ base, int32_t* __restrict__ out,
                                                        uint64_t npairs, int32_t* __restrict__ status) {
  const uint32_t e = *reinterpret_cast<const uint32_t*>(base + kOffErr);
  if (blockIdx.x == 0 && threadIdx.x == 0 && status) *status = e ? FAMSA_LCS_EINVAL : FAMSA_LCS_OK;
  if (!e) return;
  const uint64_t n = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npairs; p += n) out[p] = -1;
}

// Per device: the scratch address and the fast kernels' launch shapes.
struct NaDevice {
  uint8_t* ptr = nullptr;
  int cus = 0;
  uint32_t blocks[2][3] = {};  // [sigma <= 20, sigma <= 32][class]: workgroups per launch
  uint32_t waves[2][3] = {};
  bool ready = false;
};
std::mutex g_na_mu;
NaDevice g_na[kNaMaxDevices];

uint32_t na_qcap(int sig32, int cls) { return (sig32 && cls == 2) ? 4u : (uint32_t)kClassQMax[cls]; }

// Once per device, with that device current.
int na_setup(int device, NaDevice** out) {
  std::lock_guard<std::mutex> lock(g_na_mu);
  NaDevice& d = g_na[device];
  if (!d.ready) {
    void* p = nullptr;
    FAMSA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    int cus = 0, lds = 0;
    FAMSA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    FAMSA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if (lds > 0) g_max_lds = std::min<size_t>(kMaxLds, (size_t)lds);
    const LaunchParams lp;
    for (int s = 0; s < 2; ++s) {
      const uint32_t sigma = s ? 32u : 20u;
      for (int c = 0; c < 3; ++c) {
        uint32_t waves = lp.waves[c];
        int n = 0;
        int e = fast_prepare(c, sigma, na_qcap(s, c), waves, &n);
        while (e == 0 && n == 0 && waves > 1) {
          waves /= 2;
          e = fast_prepare(c, sigma, na_qcap(s, c), waves, &n);
        }
        if (e || n == 0)
          return set_error(FAMSA_LCS_EDEVICE, "fast kernel %d setup for sigma %u failed", c, sigma);
        d.blocks[s][c] = (uint32_t)n * (uint32_t)cus;
        d.waves[s][c] = waves;
      }
    }
    d.ptr = static_cast<uint8_t*>(p);
    d.cus = cus;
    d.ready = true;
  }
  *out = &d;
  return 0;
}

int na_run(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, uint32_t sigma, int32_t* out,
           int32_t* status, int device, hipStream_t st) {
  NaDevice* d = nullptr;
  int rc = na_setup(device, &d);
  if (rc) return rc;
  uint8_t* base = d->ptr;
  const int s32 = sig_cap(sigma) == 32 ? 1 : 0;
  const uint32_t maxlen = s32 ? kNaMaxLen32 : kNaMaxLen20;
  hipLaunchKernelGGL(na_plan_kernel, dim3(1), dim3(kNaPlanThreads), 0, st, seq_off, nseq, maxlen, base);
  FAMSA_HIP(hipGetLastError());
  if (nseq) {
    hipLaunchKernelGGL(na_stage_kernel, dim3(nseq), dim3(256), 0, st, codes, seq_off, sigma, base);
    FAMSA_HIP(hipGetLastError());
  }
  const uint64_t npairs = (uint64_t)nseq * (nseq ? nseq - 1 : 0) / 2;
  if (npairs) {
    DeviceBatch b{};
    b.sym = base + kOffSym;
    b.sym_off = reinterpret_cast<const uint64_t*>(base + kOffSymOff);
    b.len = reinterpret_cast<const uint32_t*>(base + kOffLen);
    b.mask_off = reinterpret_cast<const uint64_t*>(base + kOffMaskOff);
    b.masks = reinterpret_cast<const uint32_t*>(base + kOffMasks);
    b.values = FAMSA_LCS_VALUES_LCS;
    DeviceWork w{};
    w.groups = reinterpret_cast<const GroupDesc*>(base + kOffGroups);
    w.lanes = reinterpret_cast<const LaneDesc*>(base + kOffLanes);
    w.items = reinterpret_cast<const ItemDesc*>(base + kOffItems);
    w.colmap = reinterpret_cast<const uint32_t*>(base + kOffColmap);
    w.rowbase = reinterpret_cast<const uint64_t*>(base + kOffRowbase);
    w.ranges = reinterpret_cast<const StepRange*>(base + kOffRange);
    StepCtl* ctl = reinterpret_cast<StepCtl*>(base + kOffCtl);
    for (int c = 2; c >= 0; --c) {  // heaviest class first; a class with no items returns at once
      const int e = launch_fast(c, b, w, ctl, out, sigma, na_qcap(s32, c), d->blocks[s32][c], d->waves[s32][c], st);
      if (e) return set_error(FAMSA_LCS_EDEVICE, "lcs_fast<%d> launch failed: %s", c, hipGetErrorString((hipError_t)e));
    }
  }
  hipLaunchKernelGGL(na_finish_kernel, dim3(256), dim3(256), 0, st, base, out, npairs, status);
  FAMSA_HIP(hipGetLastError());
  return 0;
}

}  // namespace
}  // namespace famsa

extern "C" int famsa_lcs_family_noalloc(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq,
                                        uint32_t alphabet_size, int32_t* out, int32_t* status, int device,
                                        void* stream) {
  using namespace famsa;
  if (alphabet_size < 1 || alphabet_size > FAMSA_LCS_MAX_ALPHABET)
    return set_error(FAMSA_LCS_EINVAL, "alphabet_size %u not in [1, %u]", alphabet_size, FAMSA_LCS_MAX_ALPHABET);
  if (nseq > kNaMaxSeq)
    return set_error(FAMSA_LCS_EINVAL, "nseq %u exceeds the static scratch limit of %u sequences", nseq, kNaMaxSeq);
  if (!seq_off) return set_error(FAMSA_LCS_EINVAL, "seq_off is NULL");
  if (nseq && !codes) return set_error(FAMSA_LCS_EINVAL, "codes is NULL");
  if (nseq >= 2 && !out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  if (device < 0 || device >= kNaMaxDevices) return set_error(FAMSA_LCS_EINVAL, "device %d out of range", device);
  int ndev = 0;
  FAMSA_HIP(hipGetDeviceCount(&ndev));
  if (device >= ndev) return set_error(FAMSA_LCS_EINVAL, "device %d of %d", device, ndev);
  int cur = 0;
  FAMSA_HIP(hipGetDevice(&cur));
  FAMSA_HIP(hipSetDevice(device));
  const int rc = na_run(codes, seq_off, nseq, alphabet_size, out, status, device, (hipStream_t)stream);
  FAMSA_HIP(hipSetDevice(cur));
  return rc;
}
