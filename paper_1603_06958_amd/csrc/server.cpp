// Serving: continuous batching of similarity jobs (one family each).
//
// A job is admitted when its resident footprint (codes, masks and index
// arrays) fits the HBM budget next to the server's fixed step buffers; its
// sequences and masks then stay on the device until its last tile is
// delivered.  Every scheduler step gathers pending tiles of all admitted
// jobs -- jobs with the least remaining work first, a job whose whole
// triangle fits the step (values and cells) as one family-mode unit, larger
// jobs tile by tile --
// into one launch per length class.  The step's sequence index space is
// assembled from the jobs' own device arrays: per-sequence byte addresses
// and mask addresses are absolute, so the kernels read every job in place.
// Step s is computing while the tiles of step s-1 are delivered, and a job
// that arrives meanwhile joins on the next step.
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <memory>

#include "runtime.h"

namespace famsa {
int tune_lookup(const GpuInfo& gi, uint32_t sigma, LaunchParams* lp);
}
using namespace famsa;

namespace {

struct Job {
  uint32_t id = 0;
  int state = 0;  // 0 queued, 1 admitted, 2 done
  uint32_t k = 0;
  std::vector<uint8_t> codes;
  std::vector<uint64_t> off;
  uint64_t footprint = 0;
  std::unique_ptr<DeviceBatchOwner> dev;
  struct T {
    uint32_t r0, r1;
    uint64_t count;
  };
  std::vector<T> tiles;
  uint32_t next_tile = 0;       // first tile not yet issued
  uint32_t delivered = 0;       // tiles delivered
  bool whole = false;           // the whole triangle goes in one step
  uint64_t remaining_cells = 0;
  std::vector<uint64_t> tile_cells;
  uint32_t bypassed = 0;        // jobs admitted while this one was the oldest queued
};

constexpr uint32_t kMaxBypass = 64;

struct StepTile {
  Job* job;
  uint32_t tile;     // index in job->tiles
  uint64_t out_off;  // in the step buffer
};

struct Slot {
  DevMem d_out;
  PinMem h_out;
  DevMem d_groups, d_lanes, d_items, d_prows, d_colmap, d_rowbase, d_ranges, d_devoff, d_len, d_maskoff, d_ctl;
  DevMem d_symoff;
  DevMem d_plainwork, d_carry;
  StepExec exec;
  std::vector<StepTile> tiles;
  uint64_t values = 0;
  bool busy = false;
  hipEvent_t done = nullptr;
};

template <class T>
int upload_grow(DevMem& d, const std::vector<T>& h, hipStream_t s) {
  const size_t n = std::max<size_t>(h.size() * sizeof(T), 16);
  if (d.bytes < n) {
    int rc = d.alloc(n + n / 2);
    if (rc) return rc;
  }
  if (!h.empty()) FAMSA_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return 0;
}

}  // namespace

struct famsa_lcs_server_s {
  Opts opt;
  GpuInfo gi;
  LaunchParams lp;
  uint64_t budget = 0, fixed = 0, in_use = 0, peak = 0;
  uint64_t step_values = 0;
  uint64_t step_cells = 0;  // 0: steps bounded by values only
  std::map<uint32_t, std::unique_ptr<Job>> jobs;
  std::deque<Job*> queue;
  // device memory of finished jobs, kept for later jobs: freeing device
  // memory waits for the whole device, which would stall the step pipeline
  std::vector<DevMem> spare;
  uint64_t spare_bytes = 0;
  std::vector<Job*> active;
  uint32_t next_id = 0;
  hipStream_t cs = nullptr, xs = nullptr;  // the device's shared compute and copy streams
  Slot slot[2];
  uint64_t step_no = 0;
  // host staging kept alive until the step's uploads complete
  struct Staging {
    WorkLists wl;
    std::vector<uint64_t> devoff, maskoff, symoff;
    std::vector<uint32_t> len;
  } stage[2];
  ~famsa_lcs_server_s() {
    if (cs) (void)hipStreamSynchronize(cs);
    if (xs) (void)hipStreamSynchronize(xs);
    for (auto& sl : slot)
      if (sl.done) (void)hipEventDestroy(sl.done);
  }
  int admit();
  int compose(Slot& sl, Staging& st);
  int issue(int si);
  int deliver(int si, famsa_lcs_tile_fn fn, void* user);
};

// Admission: every queued job whose footprint fits what the budget has left
// is admitted, oldest first; a job that does not fit stays queued and later
// (smaller) jobs may pass it.  So that a large job is not passed forever, once
// kMaxBypass jobs have been admitted past the oldest queued job, nothing more
// is admitted until that one fits.
int famsa_lcs_server_s::admit() {
  for (auto it = queue.begin(); it != queue.end();) {
    Job* j = *it;
    // the smallest spare block that holds the job, if any (no more than twice its size)
    int reuse = -1;
    for (size_t b = 0; b < spare.size(); ++b)
      if (spare[b].bytes >= j->footprint && spare[b].bytes <= 2 * j->footprint + (1u << 20) &&
          (reuse < 0 || spare[b].bytes < spare[reuse].bytes))
        reuse = (int)b;
    const uint64_t need = reuse >= 0 ? 0 : j->footprint;
    while (reuse < 0 && !spare.empty() && in_use + spare_bytes + need > budget - fixed) {
      spare_bytes -= spare.back().bytes;  // make room: this free waits for the device
      spare.pop_back();
    }
    if (in_use + spare_bytes + need > budget - fixed) {
      if (queue.front()->bypassed >= kMaxBypass) break;
      ++it;
      continue;
    }
    j->dev.reset(new DeviceBatchOwner());
    if (reuse >= 0) {
      spare_bytes -= spare[reuse].bytes;
      std::swap(j->dev->mem.p, spare[reuse].p);
      std::swap(j->dev->mem.bytes, spare[reuse].bytes);
      spare.erase(spare.begin() + reuse);
    }
    // no wait: the uploads and mask build are ordered on cs before the job's first step
    int rc = j->dev->create(j->codes.data(), j->off.data(), j->k, opt.sigma, cs, false);
    if (rc) return rc;
    in_use += j->dev->bytes;
    peak = std::max(peak, in_use + spare_bytes + fixed);
    j->state = 1;
    std::vector<uint8_t>().swap(j->codes);
    active.push_back(j);
    if (it != queue.begin()) ++queue.front()->bypassed;
    it = queue.erase(it);
  }
  return 0;
}

int famsa_lcs_server_s::compose(Slot& sl, Staging& st) {
  sl.tiles.clear();
  sl.values = 0;
  std::vector<Job*> cand;
  for (Job* j : active)
    if (j->next_tile < j->tiles.size()) cand.push_back(j);
  std::stable_sort(cand.begin(), cand.end(),
                   [](const Job* a, const Job* b) { return a->remaining_cells < b->remaining_cells; });
  std::vector<StepFamily> fams;
  st.devoff.clear();
  st.maskoff.clear();
  st.symoff.clear();
  st.len.clear();
  std::vector<uint64_t> lenprefix(1, 0);
  uint64_t cells = 0;  // of the tiles taken so far
  // a step that is still empty takes the next unit whatever its size
  auto fits = [&](uint64_t v, uint64_t c) {
    return sl.values == 0 || (sl.values + v <= step_values && (!step_cells || cells + c <= step_cells));
  };
  for (Job* j : cand) {
    const uint32_t first = j->next_tile;
    uint32_t last = first;  // tiles [first, last) go in this step
    uint64_t vals = 0, jc = 0;
    if (j->whole) {
      for (uint32_t t = first; t < j->tiles.size(); ++t) {
        vals += j->tiles[t].count;
        jc += j->tile_cells[t];
      }
      if (!fits(vals, jc)) continue;
      last = (uint32_t)j->tiles.size();
    } else {
      while (last < j->tiles.size() &&
             ((vals == 0 && fits(j->tiles[last].count, j->tile_cells[last])) ||
              (vals && sl.values + vals + j->tiles[last].count <= step_values &&
               (!step_cells || cells + jc + j->tile_cells[last] <= step_cells)))) {
        vals += j->tiles[last].count;
        jc += j->tile_cells[last++];
      }
    }
    if (last == first) continue;
    cells += jc;
    StepFamily sf;
    sf.fam = FamilyRef{(uint32_t)st.len.size(), j->k};
    sf.whole = j->whole;
    const DeviceBatchOwner& d = *j->dev;
    const uint64_t cbase = (uint64_t)(uintptr_t)d.codes, mbase = (uint64_t)(uintptr_t)d.masks / 4;
    const uint64_t sbase = (uint64_t)(uintptr_t)d.sym;
    for (uint32_t i = 0; i < j->k; ++i) {
      st.devoff.push_back(cbase + d.h_dev_off[i]);
      st.symoff.push_back(sbase + d.h_sym_off[i]);
      st.maskoff.push_back(mbase + d.h_mask_off[i]);
      st.len.push_back(d.h_len[i]);
      lenprefix.push_back(lenprefix.back() + d.h_len[i]);
    }
    for (uint32_t t = first; t < last; ++t) {
      sf.tiles.push_back(TileWork{sf.fam.fam_base, j->k, j->tiles[t].r0, j->tiles[t].r1, sl.values});
      sl.tiles.push_back(StepTile{j, t, sl.values});
      sl.values += j->tiles[t].count;
      j->remaining_cells -= j->tile_cells[t];
    }
    j->next_tile = last;
    fams.push_back(std::move(sf));
    if (sl.values >= step_values || (step_cells && cells >= step_cells)) break;
  }
  st.wl = WorkLists();
  if (!fams.empty()) build_step(st.wl, fams, st.len, lenprefix, opt.sigma, lp, false);
  return 0;
}

int famsa_lcs_server_s::issue(int si) {
  Slot& sl = slot[si];
  Staging& st = stage[si];
  int rc = compose(sl, st);
  if (rc) return rc;
  sl.busy = !sl.tiles.empty();
  if (!sl.busy) return 0;
  hipStream_t s = cs;
  if ((rc = upload_grow(sl.d_groups, st.wl.groups, s)) || (rc = upload_grow(sl.d_lanes, st.wl.lanes, s)) ||
      (rc = upload_grow(sl.d_items, st.wl.items, s)) || (rc = upload_grow(sl.d_prows, st.wl.prows, s)) ||
      (rc = upload_grow(sl.d_colmap, st.wl.colmap, s)) || (rc = upload_grow(sl.d_rowbase, st.wl.rowbase, s)) ||
      (rc = upload_grow(sl.d_ranges, st.wl.ranges, s)) || (rc = upload_grow(sl.d_devoff, st.devoff, s)) ||
      (rc = upload_grow(sl.d_len, st.len, s)) || (rc = upload_grow(sl.d_maskoff, st.maskoff, s)) ||
      (rc = upload_grow(sl.d_symoff, st.symoff, s)))
    return rc;
  StepCtl hc{};
  hc.next_step = 0;
  hc.stride = 1;
  if (!sl.d_ctl.p && (rc = sl.d_ctl.alloc(sizeof(StepCtl)))) return rc;
  FAMSA_HIP(hipMemcpyAsync(sl.d_ctl.p, &hc, sizeof hc, hipMemcpyHostToDevice, s));
  if ((rc = sl.exec.prepare(gi.cus, lp, st.wl, opt.sigma))) return rc;
  if (sl.exec.w64max_plain > plain_register_w64_limit()) {
    sl.exec.plain_blocks = std::min<uint32_t>(sl.exec.plain_blocks, (uint32_t)gi.cus * 8u);
    const uint64_t need = (uint64_t)sl.exec.plain_blocks * kPlainBlock * sl.exec.w64max_plain * 8;
    if (sl.d_plainwork.bytes < need && (rc = sl.d_plainwork.alloc(need))) return rc;
  }
  // codes, sym and masks are null: the step's offsets are absolute device addresses
  DeviceBatch b{nullptr, sl.d_devoff.as<uint64_t>(),  nullptr, sl.d_symoff.as<uint64_t>(),
                sl.d_len.as<uint32_t>(), sl.d_maskoff.as<uint64_t>(), nullptr, FAMSA_LCS_VALUES_LCS};
  DeviceWork w{sl.d_groups.as<GroupDesc>(), sl.d_lanes.as<LaneDesc>(), sl.d_items.as<ItemDesc>(),
               sl.d_prows.as<PlainRow>(), sl.d_colmap.as<uint32_t>(), sl.d_rowbase.as<uint64_t>(),
               sl.d_ranges.as<StepRange>()};
  if (sl.exec.has_long && sl.d_carry.bytes < sl.exec.carry_bytes() && (rc = sl.d_carry.alloc(sl.exec.carry_bytes())))
    return rc;
  if ((rc = sl.exec.enqueue(st.wl.sigs[0], b, w, sl.d_ctl.as<StepCtl>(), sl.d_out.as<int32_t>(),
                            sl.d_plainwork.as<uint64_t>(), sl.d_carry.as<uint32_t>(), s, nullptr)))
    return rc;
  FAMSA_HIP(hipEventRecord(sl.done, s));
  FAMSA_HIP(hipStreamWaitEvent(xs, sl.done, 0));
  FAMSA_HIP(hipMemcpyAsync(sl.h_out.p, sl.d_out.p, sl.values * sizeof(int32_t), hipMemcpyDeviceToHost, xs));
  FAMSA_HIP(hipEventRecord(sl.done, xs));
  // the staged host vectors must outlive the async uploads: they live in stage[si]
  // until this slot is composed again, after its delivery has synchronised.
  return 0;
}

int famsa_lcs_server_s::deliver(int si, famsa_lcs_tile_fn fn, void* user) {
  Slot& sl = slot[si];
  if (!sl.busy) return 0;
  FAMSA_HIP(hipEventSynchronize(sl.done));
  sl.busy = false;
  int rc = 0;
  for (const StepTile& t : sl.tiles) {
    Job* j = t.job;
    const auto& tr = j->tiles[t.tile];
    famsa_lcs_tile tile{};
    tile.tile_index = t.tile;
    tile.family = j->id;
    tile.k = j->k;
    tile.row_begin = tr.r0;
    tile.row_end = tr.r1;
    tile.count = tr.count;
    tile.lcs = sl.h_out.as<int32_t>() + t.out_off;
    tile.stream = cs;
    if (!rc && fn && fn(user, &tile) != 0)
      rc = set_error(FAMSA_LCS_ECANCELED, "tile callback returned nonzero (job %u tile %u)", j->id, t.tile);
    j->delivered++;
    if (j->delivered == j->tiles.size()) {
      j->state = 2;
      in_use -= j->dev->bytes;
      // keep the job's device memory for a later job; the step that read it has
      // completed (its copy event was waited on above), and later steps do not
      spare.emplace_back();
      std::swap(spare.back().p, j->dev->mem.p);
      std::swap(spare.back().bytes, j->dev->mem.bytes);
      spare_bytes += spare.back().bytes;
      j->dev.reset();
      active.erase(std::find(active.begin(), active.end(), j));
    }
  }
  return rc;
}

extern "C" {

int famsa_lcs_server_create(const famsa_lcs_options* opt, famsa_lcs_server_t** out) {
  clear_error();
  if (!out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  *out = nullptr;
  Opts o;
  int rc = normalize_options(opt, &o);
  if (rc) return rc;
  if (o.flags & ~(FAMSA_LCS_NO_AUTOTUNE | FAMSA_LCS_NO_GRAPH))
    return set_error(FAMSA_LCS_EINVAL, "serving supports only the NO_AUTOTUNE and NO_GRAPH flags");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return set_error(FAMSA_LCS_EDEVICE, "no HIP device available");
  }
  if (o.device >= ndev) return set_error(FAMSA_LCS_EINVAL, "device %d >= device count %d", o.device, ndev);
  FAMSA_HIP(hipSetDevice(o.device));
  std::unique_ptr<famsa_lcs_server_s> s(new (std::nothrow) famsa_lcs_server_s());
  if (!s) return set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  s->opt = o;
  if ((rc = gpu_info(o.device, &s->gi))) return rc;
  if (!(o.flags & FAMSA_LCS_NO_AUTOTUNE)) tune_lookup(s->gi, o.sigma, &s->lp);
  if (o.cols_per_item) s->lp.cols_per_item = o.cols_per_item;
  if (o.flags & FAMSA_LCS_LONG_SEGMENTED) s->lp.long_wl = 0;
  size_t freeb = 0, totalb = 0;
  FAMSA_HIP(hipMemGetInfo(&freeb, &totalb));
  s->budget = o.hbm_budget ? o.hbm_budget : (uint64_t)(freeb * 0.9);
  s->step_values = o.step_values;
  s->step_cells = o.step_cells;
  s->fixed = 2 * s->step_values * 4 + (64u << 20);  // step buffers + descriptor headroom
  if (s->fixed >= s->budget) {
    s->step_values = std::max<uint64_t>(1024, (s->budget / 4) / 8);
    s->fixed = 2 * s->step_values * 4 + (s->budget / 8);
  }
  if (s->fixed >= s->budget) return set_error(FAMSA_LCS_ENOMEM, "budget %llu too small", (unsigned long long)s->budget);
  if ((rc = lib_stream(o.device, 0, &s->cs)) || (rc = lib_stream(o.device, kCopyStream, &s->xs))) return rc;
  for (auto& sl : s->slot) {
    FAMSA_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    if ((rc = sl.d_out.alloc(s->step_values * 4)) || (rc = sl.h_out.alloc(s->step_values * 4))) return rc;
  }
  s->peak = s->fixed;
  *out = s.release();
  return 0;
}

int famsa_lcs_server_submit(famsa_lcs_server_t* s, const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq,
                            uint32_t* job_id) {
  clear_error();
  if (!s || !job_id) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  std::vector<uint32_t> fo;
  uint32_t maxlen = 0;
  int rc = validate_batch(codes, seq_off, nseq, nullptr, 0, s->opt.sigma, &fo, &maxlen);
  if (rc) return rc;
  std::unique_ptr<Job> j(new (std::nothrow) Job());
  if (!j) return set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  j->k = nseq;
  j->off.resize(nseq + 1);
  const uint64_t base = nseq ? seq_off[0] : 0;
  for (uint32_t i = 0; i <= nseq; ++i) j->off[i] = seq_off[i] - base;
  const uint64_t total = nseq ? seq_off[nseq] - base : 0;
  j->codes.assign(codes ? codes + base : nullptr, codes ? codes + base + total : nullptr);
  j->footprint = DeviceBatchOwner::footprint(j->off.data(), nseq, s->opt.sigma);
  if (j->footprint + s->fixed > s->budget)
    return set_error(FAMSA_LCS_ENOMEM, "job needs %llu device bytes; the budget leaves %llu",
                     (unsigned long long)j->footprint, (unsigned long long)(s->budget - s->fixed));
  const uint32_t R = s->opt.tile_rows;
  uint64_t tri = 0;
  std::vector<uint64_t> L(nseq);
  for (uint32_t i = 0; i < nseq; ++i) L[i] = j->off[i + 1] - j->off[i];
  std::vector<uint64_t> suffix(nseq + 1, 0);
  for (uint32_t i = nseq; i-- > 0;) suffix[i] = suffix[i + 1] + L[i];
  // Tiles of at most R rows and, with a cell bound per step, at most that
  // many cells (a tile holds at least one row): a step that a long job's
  // tile would fill alone then still ends in about the bounded time, so a
  // job that arrives meanwhile does not wait behind it.
  for (uint32_t r0 = 0; r0 < nseq;) {
    uint32_t r1 = r0;
    uint64_t c = 0;
    do {
      c += L[r1] * suffix[r1 + 1];
      ++r1;
    } while (r1 < nseq && r1 - r0 < R && (!s->step_cells || c + L[r1] * suffix[r1 + 1] <= s->step_cells));
    const uint64_t cnt = tri_rows(nseq, r0, r1);
    j->tiles.push_back(Job::T{r0, r1, cnt});
    j->tile_cells.push_back(c);
    j->remaining_cells += c;
    tri += cnt;
    r0 = r1;
  }
  for (const auto& t : j->tiles)
    if (t.count > s->step_values)
      return set_error(FAMSA_LCS_ENOMEM, "a %u-row tile of this job holds %llu values, more than the step buffer's "
                       "%llu; use fewer tile_rows or a larger step_values",
                       s->opt.tile_rows, (unsigned long long)t.count, (unsigned long long)s->step_values);
  // one family-mode unit only if it also keeps within the step's cell bound:
  // a step that such a job fills alone would otherwise run as long as the job
  j->whole = tri <= s->step_values && (!s->step_cells || j->remaining_cells <= s->step_cells);
  j->id = s->next_id++;
  *job_id = j->id;
  if (j->tiles.empty()) {  // an empty job is done at once
    j->state = 2;
  } else {
    s->queue.push_back(j.get());
  }
  s->jobs[j->id] = std::move(j);
  return 0;
}

int famsa_lcs_server_step(famsa_lcs_server_t* s, famsa_lcs_tile_fn fn, void* user, uint32_t* active) {
  clear_error();
  if (!s) return set_error(FAMSA_LCS_EINVAL, "server is NULL");
  FAMSA_HIP(hipSetDevice(s->opt.device));
  int rc = s->admit();
  if (rc) return rc;
  const int cur = (int)(s->step_no & 1), prev = cur ^ 1;
  // this slot's previous step was delivered by the last call, so its buffers are free
  if ((rc = s->issue(cur))) return rc;
  const bool issued = s->slot[cur].busy;
  rc = s->deliver(prev, fn, user);
  if (issued) s->step_no++;
  if (active) *active = (uint32_t)(s->active.size() + s->queue.size());
  return rc;
}

int famsa_lcs_server_job_state(const famsa_lcs_server_t* s, uint32_t id, int* state) {
  clear_error();
  if (!s || !state) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return set_error(FAMSA_LCS_EINVAL, "unknown job %u", id);
  *state = it->second->state;
  return 0;
}

int famsa_lcs_server_memory(const famsa_lcs_server_t* s, uint64_t* in_use, uint64_t* peak) {
  clear_error();
  if (!s) return set_error(FAMSA_LCS_EINVAL, "server is NULL");
  if (in_use) *in_use = s->in_use + s->spare_bytes + s->fixed;
  if (peak) *peak = s->peak;
  return 0;
}

void famsa_lcs_server_destroy(famsa_lcs_server_t* s) { delete s; }

}  // extern "C"
