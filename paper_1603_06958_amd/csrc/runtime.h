// Host runtime internals shared by the plan, the serving loop and the tuner.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/famsa_lcs.h"
#include "lcs_common.h"

namespace famsa {

int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define FAMSA_HIP(call)                                                                                    \
  do {                                                                                                     \
    hipError_t e_ = (call);                                                                                \
    if (e_ != hipSuccess) return ::famsa::set_error(FAMSA_LCS_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// RAII device / pinned buffers.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevMem() { reset(); }
  void reset();
  int alloc(size_t n);  // 0 or FAMSA_LCS_ENOMEM / EDEVICE (error text set)
  template <class T> T* as() const { return static_cast<T*>(p); }
};

struct PinMem {
  void* p = nullptr;
  size_t bytes = 0;
  PinMem() = default;
  PinMem(const PinMem&) = delete;
  PinMem& operator=(const PinMem&) = delete;
  ~PinMem() { reset(); }
  void reset();
  int alloc(size_t n);
  template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T>
int upload(DevMem& d, const std::vector<T>& h, hipStream_t s) {
  const size_t n = h.size() * sizeof(T);
  int rc = d.alloc(n ? n : sizeof(T));
  if (rc) return rc;
  if (n) FAMSA_HIP(hipMemcpyAsync(d.p, h.data(), n, hipMemcpyHostToDevice, s));
  return 0;
}

// Normalised options.
struct Opts {
  uint32_t sigma = 20;
  uint32_t tile_rows = 1024;
  int device = 0;
  hipStream_t user_stream = nullptr;
  uint64_t hbm_budget = 0;
  uint32_t flags = 0;
  uint32_t cols_per_item = 0;
  uint64_t step_values = 0;
  uint64_t step_cells = 0;
};
int normalize_options(const famsa_lcs_options* in, Opts* out);

// Host-side checks of one batch (no HIP calls).
int validate_batch(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, const uint32_t* fam_off,
                   uint32_t nfam, uint32_t sigma, std::vector<uint32_t>* fam_out, uint32_t* max_len);

// A batch resident on the device with its masks, in one device allocation
// (codes, offsets, lengths, column streams and masks at 256-byte aligned
// offsets), so a serving job costs one allocation and its memory can be
// handed to the next job instead of freed.
struct DeviceBatchOwner {
  DevMem mem;
  uint8_t* codes = nullptr;      // 32-byte aligned, zero-padded sequences
  uint64_t* dev_off = nullptr;
  uint32_t* len = nullptr;
  uint64_t* mask_off = nullptr;
  uint64_t* wprefix = nullptr;   // prefix sums of mask dwords per sequence
  uint8_t* sym = nullptr;        // column streams
  uint64_t* sym_off = nullptr;
  uint32_t* masks = nullptr;
  std::vector<uint32_t> h_len;       // per sequence
  std::vector<uint64_t> h_lenprefix; // prefix sums of lengths (nseq + 1)
  std::vector<uint64_t> h_dev_off;   // device byte offset of each sequence in `codes`
  std::vector<uint64_t> h_mask_off;  // dword offset of each sequence's masks in `masks`
  std::vector<uint64_t> h_sym_off;   // byte offset of each sequence's column stream in `sym`
  // host sources of the uploads, kept while they may be in flight (create with wait = false)
  std::vector<uint8_t> st_codes;
  std::vector<uint16_t> st_sym;
  std::vector<uint64_t> st_wprefix;
  uint32_t nseq = 0, max_len = 0, sigma = 0;
  uint32_t values = FAMSA_LCS_VALUES_LCS;  // tile contents, from the plan's flags
  uint64_t bytes = 0;                      // device bytes held (mem's size)
  DeviceBatch view() const;
  // Copies the batch (validated) to the device and builds the masks on `s`,
  // reusing `mem` when it is already large enough.  With wait = false the call
  // does not synchronise: the host sources stay in this object, and work
  // ordered on `s` after the call sees the batch.
  int create(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, uint32_t sigma, hipStream_t s,
             bool wait = true);
  // Device bytes create() needs for this batch.
  static uint64_t footprint(const uint64_t* seq_off, uint32_t nseq, uint32_t sigma);
};

// A row tile to compute inside a launch step.
struct TileWork {
  uint32_t fam_base;     // global index of the family's first sequence
  uint32_t k;            // family size
  uint32_t r0, r1;       // rows
  uint64_t out_off;      // step-buffer offset of the tile
};

constexpr uint32_t kLongWlAuto = 0xFFFFFFFFu;
struct LaunchParams {
  uint32_t waves[4] = {4, 8, 16, 16};  // wavefronts per workgroup per class (3 = long rows)
  uint32_t cols_per_item = 256;
  // Long rows (class 3): the most dwords a lane holds in the lanes-per-row
  // mode (which fixes the lanes per row and so the rows per wave), kLongWlAuto
  // for the largest the LDS allows, 0 for the segmented kernel only.
  uint32_t long_wl = kLongWlAuto;
};

// Lanes per row for a long row of W dwords in the lanes-per-row mode, 0 when
// the row goes to the segmented kernel (mode off, or W beyond 64 lanes).
uint32_t skew_lanes(uint32_t W, uint32_t sigma, const LaunchParams& lp);

// The launches one step needs: for each fast class the quad count of its
// widest group (0: no items), and whether long-row items and plain rows
// exist.  LDS and grid sizes follow it, so a step never launches a kernel
// that has nothing to do or reserves more LDS than it uses.
struct StepSig {
  uint8_t q[3] = {0, 0, 0};
  uint8_t lng = 0, plain = 0;
  uint64_t key() const {
    return (uint64_t)q[0] | ((uint64_t)q[1] << 8) | ((uint64_t)q[2] << 16) | ((uint64_t)lng << 24) |
           ((uint64_t)plain << 32);
  }
  bool has(int c) const { return c < 3 ? q[c] != 0 : (c == 3 ? lng != 0 : plain != 0); }
};

// Host copies of the descriptor arrays for one or more steps.
struct WorkLists {
  std::vector<GroupDesc> groups;
  std::vector<LaneDesc> lanes;
  std::vector<ItemDesc> items;
  std::vector<PlainRow> prows;
  std::vector<uint32_t> colmap;
  std::vector<uint64_t> rowbase;
  std::vector<StepRange> ranges;
  std::vector<StepSig> sigs;       // per step
  uint32_t qmax[3] = {0, 0, 0};   // largest mask quad count per fast class
  bool has_long = false;           // items for the long-row kernel (segmented or lanes per row)
  uint32_t long_col_max = 0;       // longest column a segmented long-row item streams
  uint32_t w64max_plain = 0;       // largest ceil(len/64) in plain rows
  uint64_t cells[5] = {0, 0, 0, 0, 0};
  uint64_t max_plain_pairs = 0;
};

struct FamilyRef {
  uint32_t fam_base, k;
};

// Appends one step.  `tiles` lists the step's tiles; a family all of whose
// tiles are in the step (whole == true) uses family mode.  `plain_only`
// sends every row to the plain kernel (baseline).
struct StepFamily {
  FamilyRef fam;
  bool whole;                       // all tiles of the family are in this step
  std::vector<TileWork> tiles;      // this family's tiles in the step
};
void build_step(WorkLists& wl, const std::vector<StepFamily>& fams, const std::vector<uint32_t>& len,
                const std::vector<uint64_t>& lenprefix, uint32_t sigma, const LaunchParams& lp, bool plain_only);

// Element count of rows [r0, r1) of a k-family upper triangle.
inline uint64_t tri_rows(uint64_t k, uint64_t r0, uint64_t r1) {
  if (r1 > k) r1 = k;
  if (r0 >= r1) return 0;
  // sum_{i=r0}^{r1-1} (k-1-i)
  const uint64_t n = r1 - r0;
  return n * (k - 1) - (r0 + r1 - 1) * n / 2;
}

struct GpuInfo {
  int cus = 256;
  std::string arch;
};
int gpu_info(int device, GpuInfo* gi);

// The streams the library runs on, per device: two compute streams and one
// copy stream, made on first use and kept until the process ends.  HIP backs
// a process's streams with a few hardware queues (four by default) and
// streams beyond those share a queue, running one after the other; streams
// made per plan would therefore lose their overlap as plans come and go.
// Every plan and server on a device shares these three.
constexpr int kLibStreams = 3;
constexpr int kCopyStream = 2;
int lib_stream(int device, int i, hipStream_t* out);

// Maximum spanning forest of an edge set (guide_tree.cpp).
int spanning_forest(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num, const int64_t* den,
                    uint64_t nedges, uint32_t* ou, uint32_t* ov, int64_t* onum, int64_t* oden, uint32_t* nout);
// Single-linkage merge list from a spanning forest's edges (guide_tree.cpp).
int guide_tree(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num, const int64_t* den,
               uint32_t nedges, uint32_t* left, uint32_t* right, int64_t* mnum, int64_t* mden, uint32_t* nmerges);

// Class of a group with W dwords per lane (3 = segmented long rows).
int class_of(uint32_t W, uint32_t sigma);

// Executes the launches of one step for a set of descriptor arrays.
struct StepExec {
  uint32_t sigma = 20;
  uint32_t qmax[3] = {0, 0, 0};        // plan-wide, per fast class
  uint32_t waves[4] = {4, 8, 16, 16};
  uint32_t bpc[3][8] = {};             // resident workgroups per CU for fast class c at q quads
  uint32_t blocks[4] = {0, 0, 0, 0};   // [3]: long-row kernel grid
  int cus = 256;
  bool has_long = false;
  uint32_t carry_words = 0;            // per lane, for the longest column of a long-row item
  uint32_t plain_blocks = 0;
  uint32_t w64max_plain = 0;
  int prepare(int cus, const LaunchParams& lp, const WorkLists& wl, uint32_t sigma);
  uint64_t carry_bytes() const { return has_long ? (uint64_t)blocks[3] * waves[3] * carry_words * 64u * 4u : 0; }
  // Enqueue one step: step_begin, then the step's kernels heaviest first
  // (long rows, fast classes 2, 1, 0, plain).  With `ev` != NULL records
  // per-kernel events ev[2c], ev[2c+1] for c = 0..4.
  int enqueue(const StepSig& sig, const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out,
              uint64_t* plain_work, uint32_t* carry, hipStream_t s, hipEvent_t* ev) const;
};

}  // namespace famsa
