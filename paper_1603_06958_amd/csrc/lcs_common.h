// Internal descriptors shared by the HIP kernels and the host runtime.
//
// Device layout of a batch (built once per plan or serving job):
//   codes   : every sequence starts at a 32-byte aligned offset dev_off[s]
//             and is zero-padded to a multiple of 32 bytes, so whole 16- and
//             32-byte chunks can be read past the last residue.
//   len     : residues per sequence (uint32).
//   masks   : per-symbol match bit masks of the bit-parallel LCS method
//             (paper, Methods, "Pairwise similarities calculation": w cells
//             per machine word).  For sequence s with W_s = ceil(len/32)
//             dwords, masks[mask_off[s] + c*W_s + w] has bit p set iff
//             residue 32w+p equals code c.  Bits past the end are zero.
//
// Work decomposition.  Rows go to lanes: a group is up to 64 rows of
// similar length (one per lane of a wavefront), and a work item is a group
// against a run of column positions.  One workgroup does an item: the
// group's masks go to LDS, and each wave takes one column sequence at a time
// and streams it through the recurrence for all 64 rows at once (the
// column's symbol is the same for the whole wave: it is read from the
// column's pre-scaled symbol stream at a wave-uniform address).  Two layouts:
//   family mode -- a family whose whole upper triangle fits one launch step
//     is sorted by length (longest first); rows and columns are positions in
//     that order and a lane needs the columns after its own position, so
//     every unordered pair is computed once;
//   tile mode -- a family too large for one step is done row tile by row
//     tile: the rows of a step's tiles are pooled and sorted by length, and
//     each needs the columns (in the caller's order) after its own index.
#pragma once
#include <stdint.h>

#include "../../include/famsa_lcs.h"

namespace famsa {

constexpr int kLanes = 64;        // wavefront size on gfx950
constexpr int kNumClasses = 5;    // 0..2 fast kernels by row length, 3 segmented long-row kernel, 4 plain kernel
constexpr int kClassQMax[3] = {2, 3, 7};   // 128-bit mask quads per lane covered by classes 0..2 (W <= 8, 12, 28)
constexpr int kSeqAlign = 32;     // device code padding / alignment (bytes)
constexpr size_t kMaxLds = 163840;  // LDS bytes per workgroup on gfx950 (capped by the device's own limit)
extern size_t g_max_lds;          // min(kMaxLds, device limit), set when a plan or server opens a device
constexpr size_t kLdsReserve = 64; // static LDS of the fast kernels (queue slots) fits in this
constexpr uint32_t kPlainBlock = 256;

struct GroupDesc {          // 48 bytes
  uint32_t lane_first;      // index of lane 0 in the LaneDesc array
  uint32_t nrows;           // rows in this group (1..64)
  uint32_t W;               // dwords per lane = ceil(max row length / 32), >= 1
  uint32_t fam_base;        // global sequence index of the family's first member
  uint32_t colmap_base;     // kNoMap: column positions are the family-local indices themselves.
                            //   Otherwise positions c < nmap are mapped, index colmap[colmap_base + c],
                            //   and positions c >= nmap are the indices c + shift
  uint32_t rowbase_base;    // mapped position c -> step offset of that column's own row,
                            //   rowbase[rowbase_base + c] (kNoMap with colmap_base)
  uint32_t nmap;            // mapped positions
  uint32_t shift;           // index of an unmapped position c is c + shift
  uint32_t lpr;             // lanes per row: 0 = one lane per row (up to 64 rows, W dwords per lane); L >= 2 =
                            //   long rows each spread over L neighbouring lanes of ceil(W / L) dwords (the
                            //   long-row kernel's lanes-per-row mode), floor(64 / L) rows at most
  uint32_t pad[3];
};
constexpr uint32_t kNoMap = 0xFFFFFFFFu;

// Lanes-per-row mode: dwords per lane between kSkewWLMin and the largest a
// lane holds in LDS (28 for alphabets up to 20, 16 up to 32).
constexpr uint32_t kSkewWLMin = 8;
inline uint32_t skew_wl_max(uint32_t sigma) { return sigma <= 20 ? 28u : 16u; }

// A lane's row.  Columns are walked by position c; the lane needs column c
// iff c > pos.  Its result for column index b at position c goes to
//   out_off + (b - orig - 1)            if orig < b  (this row's own tile row)
//   rowbase[c] + (orig - b - 1)         otherwise    (row b holds the pair;
//                                                     only mapped positions)
struct LaneDesc {           // 24 bytes
  uint64_t out_off;         // step-buffer offset of LCS(orig, orig + 1)
  uint32_t seq;             // global sequence index
  uint32_t pos;             // position of this row among the columns
  uint32_t orig;            // family-local index
  uint32_t pad;
};

struct ItemDesc {           // 16 bytes
  uint32_t group;           // GroupDesc index
  uint32_t c0, c1;          // column positions [c0, c1)
  uint32_t pad;
};

// Rows handled by the plain (one pair per lane) kernel.  A launch covers a
// contiguous range of these; pair p of the range belongs to the last row
// whose pair_first <= p and is column position c = pos + 1 + (p - pair_first).
struct PlainRow {           // 48 bytes
  uint64_t out_off;         // as LaneDesc::out_off
  uint64_t pair_first;      // prefix sum of (ncols - 1 - pos) over earlier rows in the launch range
  uint32_t seq, pos, orig;
  uint32_t fam_base;
  uint32_t ncols;           // column positions run over [0, ncols)
  uint32_t colmap_base, rowbase_base;  // as GroupDesc, every position mapped
  uint32_t pad;
};

// Per-step control block in device memory.  A captured graph replays the
// same launches every step; the first node advances `step`, clears the
// queue cursors, and every kernel reads its ranges for that step.
struct StepCtl {
  uint32_t step;            // step the current replay computes
  uint32_t next_step;       // step the next replay will compute
  uint32_t cursor[4];       // work-queue cursors of classes 0..3
  uint32_t stride;          // steps between consecutive replays on this block
  uint32_t pad;
};

struct StepRange {          // per step: classes 0..3 index items, class 4 indexes plain rows
  uint32_t begin[5];
  uint32_t end[5];
  uint64_t plain_pairs;     // pairs in the class-4 row range
};

// Segmented long-row kernel: rows longer than the fast classes cover are cut
// into segments of kLongSegQ[sigcap == 32] quads; the carry out of a
// segment's top dword at each column step is passed to the next segment as
// one bit per step through a scratch buffer of kLongCarryWords(n) dwords per
// lane for a column of n residues.
constexpr int kLongSegQ[2] = {7, 4};  // sigma <= 20, sigma <= 32
inline uint32_t long_seg_q(uint32_t sigma) { return sigma <= 20 ? 7u : 4u; }
// LDS of the long-row kernel: a segment's mask table, or the lanes-per-row
// table (sigcap + 1 planes per quad, the last all zeros), whichever is larger.
inline size_t long_lds_bytes(uint32_t sigma) {
  const size_t cap = sigma <= 20 ? 20u : 32u;
  const size_t seg = (size_t)long_seg_q(sigma) * cap * 1024u;
  const size_t lpr = (size_t)((skew_wl_max(sigma) + 3u) / 4u) * (cap + 1u) * 1024u;
  return seg > lpr ? seg : lpr;
}

struct DeviceBatch {
  const uint8_t* codes;
  const uint64_t* dev_off;
  const uint8_t* sym;       // column streams: residue c stored as uint16 c * 1024 (its LDS plane offset)
  const uint64_t* sym_off;  // byte offset of each sequence's stream; 16-byte aligned, padded with one
                            // spare 16-byte chunk so the kernels may read one chunk ahead
  const uint32_t* len;
  const uint64_t* mask_off;
  const uint32_t* masks;
  uint32_t values;          // what the tiles hold: FAMSA_LCS_VALUES_LCS, _INDEL or _SIM (float32 bits)
};

struct DeviceWork {         // descriptor arrays of a plan (all steps) or of one serving step
  const GroupDesc* groups;
  const LaneDesc* lanes;
  const ItemDesc* items;
  const PlainRow* prows;
  const uint32_t* colmap;
  const uint64_t* rowbase;
  const StepRange* ranges;
};

// ---- launch wrappers (lcs_kernels.hip) ----
int launch_build_masks(const DeviceBatch& b, const uint64_t* d_wprefix, uint32_t nseq, uint64_t total_words,
                       uint32_t sigma, uint32_t* d_masks, void* stream);
int launch_step_begin(StepCtl* ctl, void* stream);
// Fast kernel for length class cls (0..2): persistent, `blocks` workgroups of
// `waves` wavefronts each.
int launch_fast(int cls, const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t sigma,
                uint32_t qmax, uint32_t blocks, uint32_t waves, void* stream);
// LDS mask table of a fast kernel: qmax quads x sigcap symbols x 64 lanes x 16 bytes.
inline uint32_t sig_cap(uint32_t sigma) { return sigma <= 20 ? 20u : 32u; }
inline size_t fast_lds_bytes(uint32_t sigma, uint32_t qmax) { return (size_t)qmax * sig_cap(sigma) * 1024u; }
int fast_prepare(int cls, uint32_t sigma, uint32_t qmax, uint32_t waves, int* blocks_per_cu);
// Plain kernel: one pair per lane over the class-3 row range of the current
// step; w64_max bounds ceil(len/64) of the rows; d_work is scratch for rows
// longer than the register variants cover (may be NULL otherwise).
int launch_plain(const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t w64_max,
                 uint32_t blocks, uint64_t* d_work, void* stream);
uint32_t plain_register_w64_limit();
// Long-row kernel: `carry` holds blocks*waves*carry_words*64 dwords.
int launch_long(const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out, uint32_t sigma,
                uint32_t* carry, uint32_t carry_words, uint32_t blocks, uint32_t waves, void* stream);
int long_prepare(uint32_t sigma, uint32_t waves, int* blocks_per_cu);

}  // namespace famsa
