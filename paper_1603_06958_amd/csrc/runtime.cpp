// Host runtime pieces shared by plans and the serving loop: errors, memory,
// validation, the device batch with its masks, and the work decomposition.
#include "runtime.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <numeric>

namespace famsa {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

const char* last_error_text() { return g_err.c_str(); }

void DevMem::reset() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

int DevMem::alloc(size_t n) {
  reset();
  if (n == 0) n = 16;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? FAMSA_LCS_ENOMEM : FAMSA_LCS_EDEVICE, "hipMalloc(%zu): %s", n,
                     hipGetErrorString(e));
  }
  bytes = n;
  return 0;
}

void PinMem::reset() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  bytes = 0;
}

int PinMem::alloc(size_t n) {
  reset();
  if (n == 0) n = 16;
  hipError_t e = hipHostMalloc(&p, n, hipHostMallocDefault);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return set_error(FAMSA_LCS_ENOMEM, "hipHostMalloc(%zu): %s", n, hipGetErrorString(e));
  }
  bytes = n;
  return 0;
}

int normalize_options(const famsa_lcs_options* in, Opts* o) {
  famsa_lcs_options d;
  famsa_lcs_default_options(&d);
  if (in) {
    if (in->struct_size < offsetof(famsa_lcs_options, cols_per_item))
      return set_error(FAMSA_LCS_EINVAL, "options.struct_size %u is too small", in->struct_size);
    const size_t n = std::min<size_t>(in->struct_size, sizeof d);
    memcpy(&d, in, n);
    d.struct_size = sizeof d;
  }
  if (d.alphabet_size < 1 || d.alphabet_size > FAMSA_LCS_MAX_ALPHABET)
    return set_error(FAMSA_LCS_EINVAL, "alphabet_size %u not in [1, %u]", d.alphabet_size, FAMSA_LCS_MAX_ALPHABET);
  if (d.tile_rows < 1) return set_error(FAMSA_LCS_EINVAL, "tile_rows must be >= 1");
  if (d.device < 0) return set_error(FAMSA_LCS_EINVAL, "device %d < 0", d.device);
  const uint32_t known = FAMSA_LCS_PLAIN | FAMSA_LCS_DESCENDING | FAMSA_LCS_DEVICE_TILES | FAMSA_LCS_NO_GRAPH |
                         FAMSA_LCS_NO_AUTOTUNE | FAMSA_LCS_ONE_STREAM | FAMSA_LCS_OUT_INDEL | FAMSA_LCS_OUT_SIM |
                         FAMSA_LCS_PLAIN_ASYNC | FAMSA_LCS_TWO_STREAMS | FAMSA_LCS_LONG_SEGMENTED;
  if (d.flags & ~known) return set_error(FAMSA_LCS_EINVAL, "unknown flag bits 0x%x", d.flags & ~known);
  if ((d.flags & FAMSA_LCS_OUT_INDEL) && (d.flags & FAMSA_LCS_OUT_SIM))
    return set_error(FAMSA_LCS_EINVAL, "FAMSA_LCS_OUT_INDEL and FAMSA_LCS_OUT_SIM exclude each other");
  if ((d.flags & FAMSA_LCS_ONE_STREAM) && (d.flags & FAMSA_LCS_TWO_STREAMS))
    return set_error(FAMSA_LCS_EINVAL, "FAMSA_LCS_ONE_STREAM and FAMSA_LCS_TWO_STREAMS exclude each other");
  if ((d.flags & FAMSA_LCS_PLAIN_ASYNC) && !(d.flags & FAMSA_LCS_PLAIN))
    return set_error(FAMSA_LCS_EINVAL, "FAMSA_LCS_PLAIN_ASYNC needs FAMSA_LCS_PLAIN");
  if (d.cols_per_item > (1u << 20)) return set_error(FAMSA_LCS_EINVAL, "cols_per_item %u too large", d.cols_per_item);
  o->sigma = d.alphabet_size;
  o->tile_rows = d.tile_rows;
  o->device = d.device;
  o->user_stream = (hipStream_t)d.stream;
  o->hbm_budget = d.hbm_budget;
  o->flags = d.flags;
  o->cols_per_item = d.cols_per_item;
  o->step_values = d.step_values ? d.step_values : (1ull << 27);
  o->step_cells = d.step_cells;
  return 0;
}

int validate_batch(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, const uint32_t* fam_off,
                   uint32_t nfam, uint32_t sigma, std::vector<uint32_t>* fam_out, uint32_t* max_len) {
  if (!seq_off) return set_error(FAMSA_LCS_EINVAL, "seq_off is NULL");
  if (nseq >= 0xFFFFFFF0u) return set_error(FAMSA_LCS_EINVAL, "nseq %u too large", nseq);
  uint32_t mx = 0;
  for (uint32_t i = 0; i < nseq; ++i) {
    if (seq_off[i + 1] < seq_off[i])
      return set_error(FAMSA_LCS_EINVAL, "seq_off decreases at %u (%llu > %llu)", i,
                       (unsigned long long)seq_off[i], (unsigned long long)seq_off[i + 1]);
    const uint64_t L = seq_off[i + 1] - seq_off[i];
    if (L > FAMSA_LCS_MAX_LEN)
      return set_error(FAMSA_LCS_EINVAL, "sequence %u has length %llu > %u", i, (unsigned long long)L,
                       FAMSA_LCS_MAX_LEN);
    mx = std::max<uint32_t>(mx, (uint32_t)L);
  }
  const uint64_t lo = nseq ? seq_off[0] : 0, hi = nseq ? seq_off[nseq] : 0;
  if (hi > lo && !codes) return set_error(FAMSA_LCS_EINVAL, "codes is NULL but %llu residues are given",
                                          (unsigned long long)(hi - lo));
  for (uint64_t p = lo; p < hi; ++p)
    if (codes[p] >= sigma)
      return set_error(FAMSA_LCS_EINVAL, "code %u at offset %llu is not below alphabet_size %u", codes[p],
                       (unsigned long long)p, sigma);
  fam_out->clear();
  if (!fam_off) {
    fam_out->push_back(0);
    fam_out->push_back(nseq);
  } else {
    if (nfam == 0 && nseq != 0) return set_error(FAMSA_LCS_EINVAL, "nfam is 0 but nseq is %u", nseq);
    if (fam_off[0] != 0) return set_error(FAMSA_LCS_EINVAL, "fam_off[0] must be 0");
    if (fam_off[nfam] != nseq) return set_error(FAMSA_LCS_EINVAL, "fam_off[nfam] = %u != nseq %u", fam_off[nfam], nseq);
    for (uint32_t f = 0; f < nfam; ++f)
      if (fam_off[f + 1] < fam_off[f]) return set_error(FAMSA_LCS_EINVAL, "fam_off decreases at %u", f);
    fam_out->assign(fam_off, fam_off + nfam + 1);
  }
  *max_len = mx;
  return 0;
}

DeviceBatch DeviceBatchOwner::view() const {
  return DeviceBatch{codes, dev_off, sym, sym_off, len, mask_off, masks, values};
}

static inline uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

namespace {
// Parts of a batch's device allocation, in bytes, from the code bytes (each
// sequence padded to 32), the stream bytes and the mask dwords.
struct BatchLayout {
  uint64_t off[8], total;
  BatchLayout(uint64_t cb, uint64_t sb, uint64_t mw, uint32_t n) {
    const uint64_t sz[8] = {cb + 32, 8ull * (n + 1), 4ull * std::max<uint32_t>(n, 1), 8ull * (n + 1),
                            8ull * (n + 1), std::max<uint64_t>(sb, 16), 8ull * (n + 1), mw * 4 + 16};
    total = 0;
    for (int i = 0; i < 8; ++i) {
      off[i] = total;
      total += round_up(sz[i], 256);
    }
  }
};
}  // namespace

uint64_t DeviceBatchOwner::footprint(const uint64_t* seq_off, uint32_t nseq, uint32_t sigma) {
  uint64_t cb = 0, words = 0, sb = 0;
  for (uint32_t i = 0; i < nseq; ++i) {
    const uint64_t L = seq_off[i + 1] - seq_off[i];
    cb += round_up(L, kSeqAlign);
    words += (L + 31) / 32;
    sb += ((L + 7) / 8 + 1) * 16;
  }
  return BatchLayout(cb, sb, words * sigma, nseq).total;
}

int DeviceBatchOwner::create(const uint8_t* hcodes, const uint64_t* seq_off, uint32_t n, uint32_t sig,
                             hipStream_t s, bool wait) {
  nseq = n;
  sigma = sig;
  h_len.resize(n);
  h_lenprefix.assign(n + 1, 0);
  std::vector<uint64_t> hoff(n + 1), hmo(n + 1), hwp(n + 1);
  uint64_t cb = 0, mw = 0, words = 0;
  max_len = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t L = (uint32_t)(seq_off[i + 1] - seq_off[i]);
    h_len[i] = L;
    h_lenprefix[i + 1] = h_lenprefix[i] + L;
    max_len = std::max(max_len, L);
    hoff[i] = cb;
    cb += round_up(L, kSeqAlign);
    const uint64_t W = (L + 31) / 32;
    hmo[i] = mw;
    mw += W * sigma;
    hwp[i] = words;
    words += W;
  }
  hoff[n] = cb;
  hmo[n] = mw;
  hwp[n] = words;
  std::vector<uint8_t> packed(cb + 32, 0);
  for (uint32_t i = 0; i < n; ++i)
    if (h_len[i]) memcpy(packed.data() + hoff[i], hcodes + seq_off[i], h_len[i]);
  // column streams: residue c as uint16 c * 1024, ceil(L/8) 16-byte chunks plus one spare
  h_sym_off.assign(n + 1, 0);
  uint64_t sb = 0;
  for (uint32_t i = 0; i < n; ++i) {
    h_sym_off[i] = sb;
    sb += ((uint64_t)(h_len[i] + 7) / 8 + 1) * 16;
  }
  h_sym_off[n] = sb;
  std::vector<uint16_t> stream(std::max<uint64_t>(sb, 16) / 2, 0);
  for (uint32_t i = 0; i < n; ++i) {
    uint16_t* d = stream.data() + h_sym_off[i] / 2;
    const uint8_t* c = hcodes + seq_off[i];
    for (uint32_t t = 0; t < h_len[i]; ++t) d[t] = (uint16_t)(c[t] * 1024u);
  }
  h_dev_off = hoff;
  h_mask_off = hmo;
  const BatchLayout lay(cb, sb, mw, n);
  if (mem.bytes < lay.total) {
    const int rc = mem.alloc(lay.total);
    if (rc) return rc;
  }
  uint8_t* base = mem.as<uint8_t>();
  codes = base + lay.off[0];
  dev_off = reinterpret_cast<uint64_t*>(base + lay.off[1]);
  len = reinterpret_cast<uint32_t*>(base + lay.off[2]);
  mask_off = reinterpret_cast<uint64_t*>(base + lay.off[3]);
  wprefix = reinterpret_cast<uint64_t*>(base + lay.off[4]);
  sym = base + lay.off[5];
  sym_off = reinterpret_cast<uint64_t*>(base + lay.off[6]);
  masks = reinterpret_cast<uint32_t*>(base + lay.off[7]);
  FAMSA_HIP(hipMemcpyAsync(codes, packed.data(), packed.size(), hipMemcpyHostToDevice, s));
  FAMSA_HIP(hipMemcpyAsync(dev_off, h_dev_off.data(), 8ull * (n + 1), hipMemcpyHostToDevice, s));
  if (n) FAMSA_HIP(hipMemcpyAsync(len, h_len.data(), 4ull * n, hipMemcpyHostToDevice, s));
  FAMSA_HIP(hipMemcpyAsync(mask_off, h_mask_off.data(), 8ull * (n + 1), hipMemcpyHostToDevice, s));
  FAMSA_HIP(hipMemcpyAsync(wprefix, hwp.data(), 8ull * (n + 1), hipMemcpyHostToDevice, s));
  FAMSA_HIP(hipMemcpyAsync(sym, stream.data(), stream.size() * 2, hipMemcpyHostToDevice, s));
  FAMSA_HIP(hipMemcpyAsync(sym_off, h_sym_off.data(), 8ull * (n + 1), hipMemcpyHostToDevice, s));
  const DeviceBatch v = view();
  int e = launch_build_masks(v, wprefix, n, words, sigma, masks, s);
  if (e) return set_error(FAMSA_LCS_EDEVICE, "build_masks launch failed: %s", hipGetErrorString((hipError_t)e));
  if (wait) {
    // the host sources above are freed on return: wait for the copies
    FAMSA_HIP(hipStreamSynchronize(s));
  } else {
    st_codes.swap(packed);
    st_sym.swap(stream);
    st_wprefix.swap(hwp);
  }
  bytes = mem.bytes;
  return 0;
}

int class_of(uint32_t W, uint32_t sigma) {
  const uint32_t Q = (W + 3) / 4;
  if (fast_lds_bytes(sigma, Q) + kLdsReserve > g_max_lds) return 3;
  for (int c = 0; c < 3; ++c)
    if (Q <= (uint32_t)kClassQMax[c]) return c;
  return 3;
}

uint32_t skew_lanes(uint32_t W, uint32_t sigma, const LaunchParams& lp) {
  if (lp.long_wl == 0) return 0;
  const uint32_t wmax = std::min(lp.long_wl, skew_wl_max(sigma));
  if (wmax < kSkewWLMin || W <= wmax) return 0;
  // L maximising the lanes doing useful work (rows per wave x lanes per row
  // over 64, the row's dwords over its lanes' dwords) times the share of the
  // recurrence's 3 WL instructions per step against the 3 per step for the
  // symbol address and the carry bits
  double best = 0;
  uint32_t bl = 0;
  for (uint32_t L = (W + wmax - 1) / wmax; L <= (uint32_t)kLanes; ++L) {
    const uint32_t WL = (W + L - 1) / L;
    if (WL < kSkewWLMin) break;
    const double u = (double)((kLanes / L) * L) / kLanes * (double)W / (double)(L * WL) * (3.0 * WL) / (3.0 * WL + 3.0);
    if (u > best + 1e-12) {
      best = u;
      bl = L;
    }
  }
  return bl;
}

namespace {
struct CostItem {
  uint64_t cost;
  ItemDesc it;
};
}  // namespace

void build_step(WorkLists& wl, const std::vector<StepFamily>& fams, const std::vector<uint32_t>& len,
                const std::vector<uint64_t>& lenprefix, uint32_t sigma, const LaunchParams& lp, bool plain_only) {
  StepRange r{};
  std::vector<CostItem> ci[4];
  std::vector<PlainRow> pr;
  uint64_t plain_pairs = 0;

  struct PendingGroup {
    GroupDesc g;
    uint32_t c0, c1;          // column positions
    const uint64_t* colpref;  // prefix sums of column lengths by position (family mode), or NULL
    uint64_t fam_pref0;       // lenprefix base (tile mode)
  };
  std::vector<PendingGroup> pend;
  std::vector<std::vector<uint64_t>> colprefs;
  colprefs.reserve(fams.size());
  uint64_t span = 0;

  auto add_plain = [&](const LaneDesc& ld, uint32_t fb, uint32_t ncols, uint32_t cm, uint32_t rb) {
    if (ld.pos + 1 >= ncols) return;  // no pairs
    PlainRow p{};
    p.out_off = ld.out_off;
    p.pair_first = plain_pairs;
    p.seq = ld.seq;
    p.pos = ld.pos;
    p.orig = ld.orig;
    p.fam_base = fb;
    p.ncols = ncols;
    p.colmap_base = cm;
    p.rowbase_base = rb;
    plain_pairs += ncols - 1 - ld.pos;
    pr.push_back(p);
    wl.w64max_plain = std::max(wl.w64max_plain, (len[ld.seq] + 63u) / 64u);
  };

  for (const StepFamily& sf : fams) {
    const uint32_t fb = sf.fam.fam_base, k = sf.fam.k;
    if (k < 2) continue;
    if (sf.whole && !plain_only) {
      std::vector<uint64_t> rowoff(k, 0);  // step offset of (i, i+1), by row
      for (const TileWork& t : sf.tiles)
        for (uint32_t i = t.r0; i < t.r1; ++i) rowoff[i] = t.out_off + tri_rows(k, t.r0, i);
      std::vector<uint32_t> perm(k);
      std::iota(perm.begin(), perm.end(), 0u);
      std::stable_sort(perm.begin(), perm.end(),
                       [&](uint32_t a, uint32_t b) { return len[fb + a] > len[fb + b]; });
      const uint32_t cm_base = (uint32_t)wl.colmap.size();
      wl.colmap.insert(wl.colmap.end(), perm.begin(), perm.end());
      const uint32_t rb_base = (uint32_t)wl.rowbase.size();
      for (uint32_t q = 0; q < k; ++q) wl.rowbase.push_back(rowoff[perm[q]]);
      colprefs.emplace_back(k + 1, 0);
      std::vector<uint64_t>& cp = colprefs.back();
      for (uint32_t q = 0; q < k; ++q) cp[q + 1] = cp[q] + len[fb + perm[q]];
      for (uint32_t P = 0, nrows = 0; P + 1 < k; P += nrows) {
        const uint32_t W = std::max<uint32_t>(1, (len[fb + perm[P]] + 31) / 32);
        const uint32_t lpr = class_of(W, sigma) == 3 ? skew_lanes(W, sigma, lp) : 0;
        nrows = std::min<uint32_t>(lpr ? kLanes / lpr : kLanes, k - P);
        GroupDesc g{};
        g.lpr = lpr;
        g.lane_first = (uint32_t)wl.lanes.size();
        g.nrows = nrows;
        g.W = W;
        g.fam_base = fb;
        g.colmap_base = cm_base;
        g.rowbase_base = rb_base;
        g.nmap = k;
        g.shift = 0;
        const int cls = class_of(W, sigma);
        for (uint32_t l = 0; l < nrows; ++l) {
          const uint32_t a = perm[P + l];
          LaneDesc ld{rowoff[a], fb + a, P + l, a, 0};
          wl.cells[cls] += (uint64_t)len[fb + a] * (cp[k] - cp[P + l + 1]);
          wl.lanes.push_back(ld);
        }
        if (cls == 3 && !lpr) wl.long_col_max = std::max(wl.long_col_max, len[fb + perm[std::min(P + 1, k - 1)]]);
        pend.push_back(PendingGroup{g, P + 1, k, cp.data(), 0});
        span += k - (P + 1);
      }
    } else {
      // tile mode: the rows of all this family's tiles in the step, pooled
      // and sorted by length so each group's rows have similar lengths
      std::vector<uint32_t> rows;
      std::vector<uint64_t> rowoff;  // step offset of (i, i+1), by position in `rows`
      uint32_t R0 = k, R1 = 0;
      for (const TileWork& t : sf.tiles) {
        for (uint32_t i = t.r0; i < t.r1; ++i) {
          rows.push_back(i);
          rowoff.push_back(t.out_off + tri_rows(k, t.r0, i));
        }
        R0 = std::min(R0, t.r0);
        R1 = std::max(R1, t.r1);
      }
      std::vector<uint32_t> ord(rows.size());
      std::iota(ord.begin(), ord.end(), 0u);
      if (!plain_only)
        std::stable_sort(ord.begin(), ord.end(),
                         [&](uint32_t a, uint32_t b) { return len[fb + rows[a]] > len[fb + rows[b]]; });
      const uint32_t ns = (uint32_t)rows.size();
      if (!plain_only && ns && R1 - R0 == ns) {
        // The step's rows are one range [R0, R1).  Column positions: first
        // those rows in the groups' (length) order, then the columns R1..k-1.
        // A pair of two step rows is computed once, by the row that comes
        // first in that order, as in family mode; every later column is
        // above every step row.  A group then walks no column below its
        // rows beyond its own 64 x 64 corner.
        const uint32_t np = ns + (k - R1);
        const uint32_t cm_base = (uint32_t)wl.colmap.size();
        const uint32_t rb_base = (uint32_t)wl.rowbase.size();
        colprefs.emplace_back(np + 1, 0);
        std::vector<uint64_t>& cp = colprefs.back();
        uint32_t colmax = 0;  // longest column (bounds the long-row kernel's carry rows)
        for (uint32_t q = 0; q < np; ++q) {
          const uint32_t j = q < ns ? rows[ord[q]] : R1 + (q - ns);
          if (q < ns) {
            wl.colmap.push_back(j);
            wl.rowbase.push_back(rowoff[ord[q]]);
          }
          cp[q + 1] = cp[q] + len[fb + j];
          colmax = std::max(colmax, len[fb + j]);
        }
        for (uint32_t P = 0, nrows = 0; P < ns; P += nrows) {
          const uint32_t W = std::max<uint32_t>(1, (len[fb + rows[ord[P]]] + 31) / 32);
          const uint32_t lpr = class_of(W, sigma) == 3 ? skew_lanes(W, sigma, lp) : 0;
          nrows = std::min<uint32_t>(lpr ? kLanes / lpr : kLanes, ns - P);
          if (P + 1 >= np) continue;  // only the family's last row: no pairs
          GroupDesc g{};
          g.lpr = lpr;
          g.lane_first = (uint32_t)wl.lanes.size();
          g.nrows = nrows;
          g.W = W;
          g.fam_base = fb;
          g.colmap_base = cm_base;
          g.rowbase_base = rb_base;
          g.nmap = ns;
          g.shift = R1 - ns;
          const int cls = class_of(W, sigma);
          for (uint32_t l = 0; l < nrows; ++l) {
            const uint32_t i = rows[ord[P + l]];
            LaneDesc ld{rowoff[ord[P + l]], fb + i, P + l, i, 0};
            wl.cells[cls] += (uint64_t)len[fb + i] * (lenprefix[fb + k] - lenprefix[fb + i + 1]);
            wl.lanes.push_back(ld);
          }
          if (cls == 3 && !lpr) wl.long_col_max = std::max(wl.long_col_max, colmax);
          pend.push_back(PendingGroup{g, P + 1, np, cp.data(), 0});
          span += np - (P + 1);
        }
        continue;
      }
      for (size_t P = 0, nrows = 0; P < ord.size(); P += nrows) {
        uint32_t lpr = 0;
        if (!plain_only) {  // rows sorted longest first: the first row is the group's widest
          const uint32_t W0 = std::max<uint32_t>(1, (len[fb + rows[ord[P]]] + 31) / 32);
          lpr = class_of(W0, sigma) == 3 ? skew_lanes(W0, sigma, lp) : 0;
        }
        nrows = (uint32_t)std::min<size_t>(lpr ? kLanes / lpr : kLanes, ord.size() - P);
        uint32_t maxlen = 0, mini = 0xFFFFFFFFu;
        for (uint32_t l = 0; l < nrows; ++l) {
          maxlen = std::max(maxlen, len[fb + rows[ord[P + l]]]);
          mini = std::min(mini, rows[ord[P + l]]);
        }
        if (mini + 1 >= k) continue;  // only the last row: no pairs
        const uint32_t W = std::max<uint32_t>(1, (maxlen + 31) / 32);
        GroupDesc g{};
        g.lane_first = (uint32_t)wl.lanes.size();
        g.nrows = nrows;
        g.W = W;
        g.fam_base = fb;
        g.colmap_base = kNoMap;
        g.rowbase_base = kNoMap;
        g.lpr = lpr;
        const int cls = plain_only ? 4 : class_of(W, sigma);
        for (uint32_t l = 0; l < nrows; ++l) {
          const uint32_t i = rows[ord[P + l]];
          LaneDesc ld{rowoff[ord[P + l]], fb + i, i, i, 0};
          wl.cells[cls] += (uint64_t)len[fb + i] * (lenprefix[fb + k] - lenprefix[fb + i + 1]);
          if (cls < 4) wl.lanes.push_back(ld);
          else add_plain(ld, fb, k, kNoMap, kNoMap);
        }
        if (cls == 3 && !lpr)
          for (uint32_t j = mini + 1; j < k; ++j) wl.long_col_max = std::max(wl.long_col_max, len[fb + j]);
        if (cls < 4) {
          pend.push_back(PendingGroup{g, mini + 1, k, nullptr, lenprefix[fb]});
          span += k - (mini + 1);
        }
      }
    }
  }

  // column chunk: the configured size, smaller when the step is small so
  // there are enough work items to fill the GPU
  uint32_t C = lp.cols_per_item ? lp.cols_per_item : 256;
  const uint64_t want_items = 4096;
  if (span / C < want_items) C = (uint32_t)std::max<uint64_t>(16, std::min<uint64_t>(C, span / want_items));
  StepSig sig;
  for (const PendingGroup& pg : pend) {
    const uint32_t gi = (uint32_t)wl.groups.size();
    wl.groups.push_back(pg.g);
    const int cls = class_of(pg.g.W, sigma);
    const uint32_t q = (pg.g.W + 3) / 4;
    if (cls < 3) {
      wl.qmax[cls] = std::max(wl.qmax[cls], q);
      sig.q[cls] = (uint8_t)std::max<uint32_t>(sig.q[cls], q);
    } else {
      wl.has_long = true;
      sig.lng = 1;
    }
    for (uint32_t c = pg.c0; c < pg.c1; c += C) {
      const uint32_t c1 = std::min<uint32_t>(pg.c1, c + C);
      uint64_t colsum;
      if (pg.colpref) colsum = pg.colpref[c1] - pg.colpref[c];
      else colsum = lenprefix[pg.g.fam_base + c1] - lenprefix[pg.g.fam_base + c];
      const uint64_t wlane = pg.g.lpr ? (pg.g.W + pg.g.lpr - 1) / pg.g.lpr : pg.g.W;  // dwords per lane
      ci[cls].push_back(CostItem{wlane * colsum + 64, ItemDesc{gi, c, c1, 0}});
    }
  }
  for (int c = 0; c < 4; ++c) {
    std::stable_sort(ci[c].begin(), ci[c].end(), [](const CostItem& a, const CostItem& b) { return a.cost > b.cost; });
    r.begin[c] = (uint32_t)wl.items.size();
    for (const CostItem& x : ci[c]) wl.items.push_back(x.it);
    r.end[c] = (uint32_t)wl.items.size();
  }
  r.begin[4] = (uint32_t)wl.prows.size();
  wl.prows.insert(wl.prows.end(), pr.begin(), pr.end());
  r.end[4] = (uint32_t)wl.prows.size();
  r.plain_pairs = plain_pairs;
  wl.max_plain_pairs = std::max(wl.max_plain_pairs, plain_pairs);
  sig.plain = plain_pairs ? 1 : 0;
  wl.ranges.push_back(r);
  wl.sigs.push_back(sig);
}

int lib_stream(int device, int i, hipStream_t* out) {
  static std::mutex mu;
  static std::map<int, std::array<hipStream_t, kLibStreams>> pool;
  if (i < 0 || i >= kLibStreams) return set_error(FAMSA_LCS_EINVAL, "stream index %d", i);
  std::lock_guard<std::mutex> lock(mu);
  auto it = pool.find(device);
  if (it == pool.end()) it = pool.emplace(device, std::array<hipStream_t, kLibStreams>{}).first;
  hipStream_t& st = it->second[i];
  if (!st) {
    int cur = 0;
    FAMSA_HIP(hipGetDevice(&cur));
    FAMSA_HIP(hipSetDevice(device));
    const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    FAMSA_HIP(hipSetDevice(cur));
    if (e != hipSuccess) {
      st = nullptr;
      return set_error(FAMSA_LCS_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
  }
  *out = st;
  return 0;
}

int gpu_info(int device, GpuInfo* gi) {
  hipDeviceProp_t prop;
  FAMSA_HIP(hipGetDeviceProperties(&prop, device));
  gi->cus = prop.multiProcessorCount;
  gi->arch = prop.gcnArchName;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    g_max_lds = std::min<size_t>(kMaxLds, (size_t)lds);
  return 0;
}

int StepExec::prepare(int ncu, const LaunchParams& lp, const WorkLists& wl, uint32_t sig) {
  sigma = sig;
  cus = ncu;
  for (int c = 0; c < 3; ++c) {
    qmax[c] = wl.qmax[c];
    waves[c] = lp.waves[c];
    for (int q = 0; q < 8; ++q) bpc[c][q] = 0;
    if (!qmax[c]) continue;
    // every quad count a step of this class may use
    bool need[8] = {};
    for (const StepSig& s : wl.sigs)
      if (s.q[c]) need[s.q[c]] = true;
    for (int q = 1; q < 8; ++q) {
      if (!need[q]) continue;
      int n = 0;
      int e = fast_prepare(c, sigma, (uint32_t)q, waves[c], &n);
      while (e == 0 && n == 0 && waves[c] > 1) {  // too many waves for the registers: shrink the workgroup
        waves[c] /= 2;
        e = fast_prepare(c, sigma, (uint32_t)q, waves[c], &n);
      }
      if (e || n == 0)
        return set_error(FAMSA_LCS_EDEVICE, "fast kernel %d setup (sigma %u, %d quads, %u waves) failed: %s", c, sigma,
                         q, waves[c], e ? hipGetErrorString((hipError_t)e) : "not resident");
      bpc[c][q] = (uint32_t)n;
    }
  }
  has_long = wl.has_long;
  waves[3] = lp.waves[3];
  blocks[3] = 0;
  carry_words = 0;
  if (has_long) {
    int n = 0;
    int e = long_prepare(sigma, waves[3], &n);
    while (e == 0 && n == 0 && waves[3] > 1) {
      waves[3] /= 2;
      e = long_prepare(sigma, waves[3], &n);
    }
    if (e || n == 0)
      return set_error(FAMSA_LCS_EDEVICE, "long-row kernel setup (sigma %u, %u waves) failed", sigma, waves[3]);
    blocks[3] = (uint32_t)(n * cus);
    carry_words = std::max<uint32_t>(1, (wl.long_col_max + 31) / 32);
  }
  w64max_plain = wl.prows.empty() ? 0 : std::max<uint32_t>(1, wl.w64max_plain);
  plain_blocks = wl.prows.empty() ? 0 : (uint32_t)(cus * 8);
  return 0;
}

int StepExec::enqueue(const StepSig& sig, const DeviceBatch& b, const DeviceWork& w, StepCtl* ctl, int32_t* out,
                      uint64_t* plain_work, uint32_t* carry, hipStream_t s, hipEvent_t* ev) const {
  int e = launch_step_begin(ctl, s);
  if (e) return set_error(FAMSA_LCS_EDEVICE, "step_begin launch failed: %s", hipGetErrorString((hipError_t)e));
  if (sig.lng) {
    if (!carry) return set_error(FAMSA_LCS_EDEVICE, "long-row kernel without a carry buffer");
    if (ev) FAMSA_HIP(hipEventRecord(ev[6], s));
    e = launch_long(b, w, ctl, out, sigma, carry, carry_words, blocks[3], waves[3], s);
    if (e) return set_error(FAMSA_LCS_EDEVICE, "lcs_long launch failed: %s", hipGetErrorString((hipError_t)e));
    if (ev) FAMSA_HIP(hipEventRecord(ev[7], s));
  }
  for (int c = 2; c >= 0; --c) {
    const uint32_t q = sig.q[c];
    if (!q) continue;
    if (q >= 8 || !bpc[c][q]) return set_error(FAMSA_LCS_EDEVICE, "fast kernel %d was not prepared for %u quads", c, q);
    if (ev) FAMSA_HIP(hipEventRecord(ev[2 * c], s));
    e = launch_fast(c, b, w, ctl, out, sigma, q, bpc[c][q] * (uint32_t)cus, waves[c], s);
    if (e) return set_error(FAMSA_LCS_EDEVICE, "lcs_fast<%d> launch failed: %s", c, hipGetErrorString((hipError_t)e));
    if (ev) FAMSA_HIP(hipEventRecord(ev[2 * c + 1], s));
  }
  if (sig.plain) {
    if (ev) FAMSA_HIP(hipEventRecord(ev[8], s));
    e = launch_plain(b, w, ctl, out, w64max_plain, plain_blocks, plain_work, s);
    if (e) return set_error(FAMSA_LCS_EDEVICE, "lcs_plain launch failed: %s", hipGetErrorString((hipError_t)e));
    if (ev) FAMSA_HIP(hipEventRecord(ev[9], s));
  }
  return 0;
}

}  // namespace famsa
