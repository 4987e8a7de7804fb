// famsa_lcs_plan / famsa_lcs_tiles / famsa_lcs_release: the C-ABI over the
// runtime.  A plan owns the resident batch, the descriptor arrays of every
// launch step, two device step buffers, two pinned host buffers, and (unless
// disabled) instantiated hipGraphs -- one per buffer slot and launch
// signature -- that replay a step's launches.  Steps run on the device's
// shared compute stream (or alternate between two with
// FAMSA_LCS_TWO_STREAMS), while the shared copy stream moves finished steps
// to pinned memory and the caller's thread runs the tile callbacks.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>

#include "runtime.h"

namespace famsa {
const char* last_error_text();
int tune_lookup(const GpuInfo& gi, uint32_t sigma, LaunchParams* lp);
int tune_store(const GpuInfo& gi, uint32_t sigma, const LaunchParams& lp, const char* path);
}  // namespace famsa

using namespace famsa;

struct famsa_lcs_plan_s {
  Opts opt;
  GpuInfo gi;
  DeviceBatchOwner batch;
  std::vector<uint32_t> fam_off;
  struct Tile {
    uint32_t fam, r0, r1, step;
    uint64_t count, out_off;
  };
  std::vector<Tile> tiles;  // delivery order
  struct Step {
    uint64_t tile_begin, tile_end, values;
  };
  std::vector<Step> steps;
  WorkLists wl;
  LaunchParams lp;
  StepExec exec;
  DevMem d_groups, d_lanes, d_items, d_prows, d_colmap, d_rowbase, d_ranges, d_ctl;
  DevMem d_plainwork[2];  // per buffer slot: with two compute streams the slots' steps run concurrently
  DevMem d_carry[2];      // long-row carry scratch, per compute stream
  DevMem d_out[2];
  PinMem h_out[2];
  uint64_t step_cap = 0;  // values per step buffer
  hipStream_t cs[2] = {nullptr, nullptr};  // the device's shared compute streams
  hipStream_t xs = nullptr;                 // and its copy stream
  hipEvent_t ev_comp[2] = {}, ev_copy[2] = {}, ev_s0[2] = {}, ev_s1[2] = {}, ev_user = nullptr;
  hipEvent_t ev_k[2][10] = {};
  std::map<uint64_t, hipGraphExec_t> graphs[2];  // per compute stream, per launch signature
  std::atomic<int> busy{0};
  famsa_lcs_stats stats{};
  uint64_t pairs = 0, cells = 0;

  DeviceWork work() const {
    return DeviceWork{d_groups.as<GroupDesc>(), d_lanes.as<LaneDesc>(), d_items.as<ItemDesc>(),
                      d_prows.as<PlainRow>(), d_colmap.as<uint32_t>(), d_rowbase.as<uint64_t>(),
                      d_ranges.as<StepRange>()};
  }
  StepCtl* ctl(int slot) const { return d_ctl.as<StepCtl>() + slot; }
  bool plain() const { return opt.flags & FAMSA_LCS_PLAIN; }
  // output buffer slots: the plain baseline has one (each launch waits for
  // the previous tile's delivery) unless FAMSA_LCS_PLAIN_ASYNC asks for two
  int slots() const { return plain() && !(opt.flags & FAMSA_LCS_PLAIN_ASYNC) ? 1 : 2; }
  // compute stream of a buffer slot: both slots share stream 0 unless
  // FAMSA_LCS_TWO_STREAMS asks for one stream per slot (never in the plain
  // baseline)
  hipStream_t cstream(int slot) const {
    return (opt.flags & FAMSA_LCS_TWO_STREAMS) && !plain() ? cs[slot] : cs[0];
  }
  // Steps replay captured graphs unless FAMSA_LCS_NO_GRAPH asks for direct
  // launches (which are timed per kernel class with events).
  bool use_graph() const { return !(opt.flags & (FAMSA_LCS_NO_GRAPH | FAMSA_LCS_PLAIN)); }
  ~famsa_lcs_plan_s();
  int build_tiles_and_steps();
  int build_work();
  int host_phase(const uint64_t* seq_off, uint32_t nseq);
  int dump(const char* path) const;
  int setup_device();
  int capture_graphs();
  int capture_on(hipStream_t cap, const DeviceBatch& b, const DeviceWork& w);
  int enqueue_step(uint64_t s, int slot, bool timed);
  int upload_work();
  void drop_graphs() {
    for (auto& m : graphs) {
      for (auto& kv : m) (void)hipGraphExecDestroy(kv.second);
      m.clear();
    }
  }
  int autotune(const char* path);
  int run(uint64_t first_tile, famsa_lcs_tile_fn fn, void* user);
};

famsa_lcs_plan_s::~famsa_lcs_plan_s() {
  // the streams are shared: wait for this plan's own work only
  for (int i = 0; i < 2; ++i) {
    if (ev_comp[i]) (void)hipEventSynchronize(ev_comp[i]);
    if (ev_copy[i]) (void)hipEventSynchronize(ev_copy[i]);
  }
  if (cs[0]) (void)hipStreamSynchronize(cs[0]);  // set-up and tuning work
  drop_graphs();
  for (int i = 0; i < 2; ++i) {
    if (ev_comp[i]) (void)hipEventDestroy(ev_comp[i]);
    if (ev_copy[i]) (void)hipEventDestroy(ev_copy[i]);
    if (ev_s0[i]) (void)hipEventDestroy(ev_s0[i]);
    if (ev_s1[i]) (void)hipEventDestroy(ev_s1[i]);
    for (int j = 0; j < 10; ++j)
      if (ev_k[i][j]) (void)hipEventDestroy(ev_k[i][j]);
  }
  if (ev_user) (void)hipEventDestroy(ev_user);
}

int famsa_lcs_plan_s::build_tiles_and_steps() {
  const uint32_t nfam = (uint32_t)fam_off.size() - 1;
  const uint32_t R = opt.tile_rows;
  // largest tile decides the minimum step size
  uint64_t max_tile = 0;
  for (uint32_t f = 0; f < nfam; ++f) {
    const uint64_t k = fam_off[f + 1] - fam_off[f];
    if (k) max_tile = std::max(max_tile, tri_rows(k, 0, std::min<uint64_t>(R, k)));
  }
  step_cap = std::max<uint64_t>(std::max<uint64_t>(max_tile, 1), plain() ? max_tile : opt.step_values);
  Step cur{0, 0, 0};
  auto close = [&]() {
    if (cur.tile_end > cur.tile_begin) steps.push_back(cur);
    cur = Step{tiles.size(), tiles.size(), 0};
  };
  for (uint32_t f = 0; f < nfam; ++f) {
    const uint32_t k = fam_off[f + 1] - fam_off[f];
    if (k == 0) continue;
    const uint32_t nt = (k + R - 1) / R;
    const uint64_t total = tri_rows(k, 0, k);
    const bool whole = !plain() && total <= step_cap;
    if (whole && cur.values + total > step_cap) close();
    for (uint32_t q = 0; q < nt; ++q) {
      const uint32_t t = (opt.flags & FAMSA_LCS_DESCENDING) ? nt - 1 - q : q;
      const uint32_t r0 = t * R, r1 = std::min<uint32_t>(k, r0 + R);
      const uint64_t cnt = tri_rows(k, r0, r1);
      if (plain() || (!whole && cur.values + cnt > step_cap)) close();
      Tile tl{f, r0, r1, (uint32_t)steps.size(), cnt, cur.values};
      tiles.push_back(tl);
      cur.tile_end = tiles.size();
      cur.values += cnt;
    }
  }
  close();
  for (const Step& s : steps)
    for (uint64_t t = s.tile_begin; t < s.tile_end; ++t) tiles[t].step = (uint32_t)(&s - steps.data());
  return 0;
}

int famsa_lcs_plan_s::build_work() {
  for (uint64_t si = 0; si < steps.size(); ++si) {
    const Step& s = steps[si];
    std::vector<StepFamily> fams;
    for (uint64_t t = s.tile_begin; t < s.tile_end; ++t) {
      const Tile& tl = tiles[t];
      const uint32_t fb = fam_off[tl.fam], k = fam_off[tl.fam + 1] - fb;
      if (fams.empty() || fams.back().fam.fam_base != fb || fams.back().fam.k != k) {
        StepFamily sf;
        sf.fam = FamilyRef{fb, k};
        sf.whole = !plain() && tri_rows(k, 0, k) <= step_cap;
        fams.push_back(sf);
      }
      fams.back().tiles.push_back(TileWork{fb, k, tl.r0, tl.r1, tl.out_off});
    }
    build_step(wl, fams, batch.h_len, batch.h_lenprefix, opt.sigma, lp, plain());
  }
  return 0;
}

// Everything that needs no device: lengths, tiles, steps and work lists.
int famsa_lcs_plan_s::host_phase(const uint64_t* seq_off, uint32_t nseq) {
  batch.h_len.resize(nseq);
  batch.h_lenprefix.assign(nseq + 1, 0);
  for (uint32_t i = 0; i < nseq; ++i) {
    batch.h_len[i] = (uint32_t)(seq_off[i + 1] - seq_off[i]);
    batch.h_lenprefix[i + 1] = batch.h_lenprefix[i] + batch.h_len[i];
  }
  int rc;
  if ((rc = build_tiles_and_steps())) return rc;
  if ((rc = build_work())) return rc;
  for (uint32_t f = 0; f + 1 < fam_off.size(); ++f) {
    const uint64_t k = fam_off[f + 1] - fam_off[f];
    pairs += k * (k ? k - 1 : 0) / 2;
  }
  for (int c = 0; c < 5; ++c) cells += wl.cells[c];
  return 0;
}

template <class T>
static bool put(FILE* f, const std::vector<T>& v) {
  const uint64_t n = v.size(), sz = sizeof(T);
  return fwrite(&n, 8, 1, f) == 1 && fwrite(&sz, 8, 1, f) == 1 && (n == 0 || fwrite(v.data(), sizeof(T), n, f) == n);
}

int famsa_lcs_plan_s::dump(const char* path) const {
  FILE* f = fopen(path, "wb");
  if (!f) return set_error(FAMSA_LCS_EINVAL, "cannot open %s for writing", path);
  const char magic[8] = {'F', 'L', 'C', 'S', 'D', 'M', 'P', '1'};
  bool ok = fwrite(magic, 1, 8, f) == 8;
  ok = ok && put(f, tiles) && put(f, steps) && put(f, wl.ranges) && put(f, wl.groups) && put(f, wl.lanes) &&
       put(f, wl.items) && put(f, wl.prows) && put(f, wl.colmap) && put(f, wl.rowbase) && put(f, batch.h_len) &&
       put(f, fam_off);
  ok = (fclose(f) == 0) && ok;
  return ok ? 0 : set_error(FAMSA_LCS_EINVAL, "short write to %s", path);
}

int famsa_lcs_plan_s::setup_device() {
  int rc;
  if ((rc = lib_stream(opt.device, 0, &cs[0])) || (rc = lib_stream(opt.device, 1, &cs[1])) ||
      (rc = lib_stream(opt.device, kCopyStream, &xs)))
    return rc;
  for (int i = 0; i < 2; ++i) {
    FAMSA_HIP(hipEventCreateWithFlags(&ev_comp[i], hipEventDisableTiming));
    FAMSA_HIP(hipEventCreateWithFlags(&ev_copy[i], hipEventDisableTiming));
    FAMSA_HIP(hipEventCreate(&ev_s0[i]));
    FAMSA_HIP(hipEventCreate(&ev_s1[i]));
    for (int j = 0; j < 10; ++j) FAMSA_HIP(hipEventCreate(&ev_k[i][j]));
  }
  FAMSA_HIP(hipEventCreateWithFlags(&ev_user, hipEventDisableTiming));
  return 0;
}

// One graph per compute stream and distinct launch signature of the plan's
// steps; a replay advances that stream's step counter and runs the step.
int famsa_lcs_plan_s::capture_graphs() {
  const DeviceBatch b = batch.view();
  const DeviceWork w = work();
  // capture on a stream of its own: the shared streams may carry other work
  hipStream_t cap = nullptr;
  FAMSA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  int rc = capture_on(cap, b, w);
  (void)hipStreamDestroy(cap);
  return rc;
}

int famsa_lcs_plan_s::capture_on(hipStream_t cap, const DeviceBatch& b, const DeviceWork& w) {
  for (int slot = 0; slot < 2; ++slot) {
    for (const StepSig& sg : wl.sigs) {
      if (graphs[slot].count(sg.key())) continue;
      hipGraph_t g = nullptr;
      FAMSA_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      int rc = exec.enqueue(sg, b, w, ctl(slot), d_out[slot].as<int32_t>(), d_plainwork[slot].as<uint64_t>(),
                            d_carry[slot].as<uint32_t>(), cap, nullptr);
      hipError_t e = hipStreamEndCapture(cap, &g);  // a graph can be launched on any stream
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return set_error(FAMSA_LCS_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return set_error(FAMSA_LCS_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      graphs[slot][sg.key()] = x;
    }
  }
  return 0;
}

int famsa_lcs_plan_s::enqueue_step(uint64_t s, int slot, bool timed) {
  hipStream_t st = cstream(slot);
  FAMSA_HIP(hipEventRecord(ev_s0[slot], st));
  const StepSig& sg = wl.sigs[s];
  if (use_graph()) {
    auto it = graphs[slot].find(sg.key());
    if (it == graphs[slot].end()) return set_error(FAMSA_LCS_EDEVICE, "no graph for step %llu", (unsigned long long)s);
    FAMSA_HIP(hipGraphLaunch(it->second, st));
  } else {
    int rc = exec.enqueue(sg, batch.view(), work(), ctl(slot), d_out[slot].as<int32_t>(),
                          d_plainwork[slot].as<uint64_t>(), d_carry[slot].as<uint32_t>(), st,
                          timed ? ev_k[slot] : nullptr);
    if (rc) return rc;
  }
  FAMSA_HIP(hipEventRecord(ev_s1[slot], st));
  FAMSA_HIP(hipEventRecord(ev_comp[slot], st));
  return 0;
}

int famsa_lcs_plan_s::upload_work() {
  hipStream_t s = cs[0];
  int rc;
  if ((rc = upload(d_groups, wl.groups, s)) || (rc = upload(d_lanes, wl.lanes, s)) || (rc = upload(d_items, wl.items, s)) ||
      (rc = upload(d_prows, wl.prows, s)) || (rc = upload(d_colmap, wl.colmap, s)) ||
      (rc = upload(d_rowbase, wl.rowbase, s)) || (rc = upload(d_ranges, wl.ranges, s)))
    return rc;
  FAMSA_HIP(hipStreamSynchronize(s));
  return 0;
}

// Time every candidate (columns per item x waves per workgroup of each
// length class) on the plan's first step, one class kernel at a time with
// events around it, keep the fastest, and rebuild the plan with it.
int famsa_lcs_plan_s::autotune(const char* path) {
  if (plain() || steps.empty()) return 0;
  static const uint32_t kCols[] = {64, 128, 256, 512};
  static const uint32_t kWaves[3][3] = {{2, 4, 8}, {4, 8, 16}, {8, 16, 16}};
  hipStream_t st = cs[0];
  hipEvent_t e0 = ev_k[0][0], e1 = ev_k[0][1];
  double best_total = 1e300;
  LaunchParams best = lp;
  std::vector<StepFamily> fams;  // step 0
  for (uint64_t t = steps[0].tile_begin; t < steps[0].tile_end; ++t) {
    const Tile& tl = tiles[t];
    const uint32_t fb = fam_off[tl.fam], k = fam_off[tl.fam + 1] - fb;
    if (fams.empty() || fams.back().fam.fam_base != fb) {
      StepFamily sf;
      sf.fam = FamilyRef{fb, k};
      sf.whole = tri_rows(k, 0, k) <= step_cap;
      fams.push_back(sf);
    }
    fams.back().tiles.push_back(TileWork{fb, k, tl.r0, tl.r1, tl.out_off});
  }
  DevMem tg, tl_, ti, tp, tc, tr, tra;
  for (uint32_t cols : kCols) {
    LaunchParams cand = lp;
    cand.cols_per_item = cols;
    WorkLists w1;
    build_step(w1, fams, batch.h_len, batch.h_lenprefix, opt.sigma, cand, false);
    int rc;
    if ((rc = upload(tg, w1.groups, st)) || (rc = upload(tl_, w1.lanes, st)) || (rc = upload(ti, w1.items, st)) ||
        (rc = upload(tp, w1.prows, st)) || (rc = upload(tc, w1.colmap, st)) || (rc = upload(tr, w1.rowbase, st)) ||
        (rc = upload(tra, w1.ranges, st)))
      return rc;
    const DeviceWork w{tg.as<GroupDesc>(), tl_.as<LaneDesc>(), ti.as<ItemDesc>(), tp.as<PlainRow>(), tc.as<uint32_t>(),
                       tr.as<uint64_t>(), tra.as<StepRange>()};
    double total = 0;
    for (int c = 0; c < 3; ++c) {
      if (!w1.qmax[c]) continue;
      double bc = 1e300;
      uint32_t bw = cand.waves[c];
      for (uint32_t wv : kWaves[c]) {
        int bpc = 0;
        if (fast_prepare(c, opt.sigma, w1.qmax[c], wv, &bpc) || bpc == 0) continue;
        StepCtl hc{};
        hc.next_step = 0;
        hc.stride = 1;
        float best_ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          FAMSA_HIP(hipMemcpyAsync(d_ctl.p, &hc, sizeof hc, hipMemcpyHostToDevice, st));
          if (launch_step_begin(ctl(0), st)) return set_error(FAMSA_LCS_EDEVICE, "step_begin failed");
          FAMSA_HIP(hipEventRecord(e0, st));
          if (launch_fast(c, batch.view(), w, ctl(0), d_out[0].as<int32_t>(), opt.sigma, w1.qmax[c],
                          (uint32_t)(bpc * gi.cus), wv, st))
            return set_error(FAMSA_LCS_EDEVICE, "tuning launch failed");
          FAMSA_HIP(hipEventRecord(e1, st));
          FAMSA_HIP(hipEventSynchronize(e1));
          float ms = 0;
          FAMSA_HIP(hipEventElapsedTime(&ms, e0, e1));
          best_ms = std::min(best_ms, ms);
        }
        if (best_ms < bc) {
          bc = best_ms;
          bw = wv;
        }
      }
      cand.waves[c] = bw;
      total += bc;
    }
    if (total < best_total) {
      best_total = total;
      best = cand;
    }
  }
  // long rows: the lanes-per-row mode at several word widths per lane, or
  // the segmented kernel, each with 8 or 16 waves per workgroup
  {
    std::vector<uint32_t> wls;
    if (!(opt.flags & FAMSA_LCS_LONG_SEGMENTED))
      for (uint32_t wl_ : {28u, 24u, 20u, 16u, 12u})
        if (wl_ <= skew_wl_max(opt.sigma)) wls.push_back(wl_);
    wls.push_back(0);
    double best_long = 1e300;
    LaunchParams lbest = best;
    DevMem carry;
    for (uint32_t lw : wls) {
      LaunchParams cand = best;
      cand.long_wl = lw;
      WorkLists w1;
      build_step(w1, fams, batch.h_len, batch.h_lenprefix, opt.sigma, cand, false);
      if (!w1.has_long) break;  // the first step has no long rows: nothing to choose
      int rc;
      if ((rc = upload(tg, w1.groups, st)) || (rc = upload(tl_, w1.lanes, st)) || (rc = upload(ti, w1.items, st)) ||
          (rc = upload(tp, w1.prows, st)) || (rc = upload(tc, w1.colmap, st)) || (rc = upload(tr, w1.rowbase, st)) ||
          (rc = upload(tra, w1.ranges, st)))
        return rc;
      const DeviceWork w{tg.as<GroupDesc>(), tl_.as<LaneDesc>(), ti.as<ItemDesc>(), tp.as<PlainRow>(),
                         tc.as<uint32_t>(), tr.as<uint64_t>(), tra.as<StepRange>()};
      for (uint32_t wv : {16u, 8u}) {
        int bpc = 0;
        if (long_prepare(opt.sigma, wv, &bpc) || bpc == 0) continue;
        const uint32_t blocks = (uint32_t)bpc * (uint32_t)gi.cus;
        const uint32_t cw = std::max<uint32_t>(1, (w1.long_col_max + 31) / 32);
        const uint64_t cbytes = (uint64_t)blocks * wv * cw * 64u * 4u;
        if (carry.bytes < cbytes && (rc = carry.alloc(cbytes))) return rc;
        StepCtl hc{};
        hc.next_step = 0;
        hc.stride = 1;
        float best_ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          FAMSA_HIP(hipMemcpyAsync(d_ctl.p, &hc, sizeof hc, hipMemcpyHostToDevice, st));
          if (launch_step_begin(ctl(0), st)) return set_error(FAMSA_LCS_EDEVICE, "step_begin failed");
          FAMSA_HIP(hipEventRecord(e0, st));
          if (launch_long(batch.view(), w, ctl(0), d_out[0].as<int32_t>(), opt.sigma, carry.as<uint32_t>(), cw, blocks,
                          wv, st))
            return set_error(FAMSA_LCS_EDEVICE, "tuning launch failed");
          FAMSA_HIP(hipEventRecord(e1, st));
          FAMSA_HIP(hipEventSynchronize(e1));
          float ms = 0;
          FAMSA_HIP(hipEventElapsedTime(&ms, e0, e1));
          best_ms = std::min(best_ms, ms);
        }
        if (best_ms < best_long) {
          best_long = best_ms;
          lbest = cand;
          lbest.waves[3] = wv;
        }
      }
    }
    best = lbest;
  }
  lp = best;
  int rc;
  if ((rc = tune_store(gi, opt.sigma, lp, path))) return rc;
  // rebuild the work lists, launch shapes and graphs with the winner
  drop_graphs();
  wl = WorkLists();
  if ((rc = build_work())) return rc;
  if ((rc = upload_work())) return rc;
  if ((rc = exec.prepare(gi.cus, lp, wl, opt.sigma))) return rc;
  if (exec.w64max_plain > plain_register_w64_limit())
    exec.plain_blocks = std::min<uint32_t>(exec.plain_blocks, (uint32_t)gi.cus * 8u);
  for (int i = 0; i < 2; ++i)
    if (exec.has_long && d_carry[i].bytes < exec.carry_bytes() && (rc = d_carry[i].alloc(exec.carry_bytes())))
      return rc;
  if (use_graph() && (rc = capture_graphs())) return rc;
  return 0;
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int famsa_lcs_plan_s::run(uint64_t first_tile, famsa_lcs_tile_fn fn, void* user) {
  memset(&stats, 0, sizeof stats);
  const uint64_t ntiles = tiles.size();
  if (first_tile >= ntiles) return 0;
  const uint64_t s0 = tiles[first_tile].step, ns = steps.size();
  const bool dev_tiles = opt.flags & FAMSA_LCS_DEVICE_TILES;
  const bool timed = !use_graph();
  const int nslots = slots();
  FAMSA_HIP(hipSetDevice(opt.device));
  // the first step each control block computes, and its stride
  // step s runs on slot s % nslots: seed each slot's control block with the
  // first step it will see
  StepCtl hc[2] = {};
  for (uint64_t s = s0; s < s0 + 2; ++s) {
    hc[s % nslots].next_step = (uint32_t)s;
    hc[s % nslots].stride = (uint32_t)nslots;
    if (nslots == 1) break;
  }
  FAMSA_HIP(hipMemcpy(d_ctl.p, hc, sizeof hc, hipMemcpyHostToDevice));
  if (opt.user_stream) {
    FAMSA_HIP(hipEventRecord(ev_user, opt.user_stream));
    for (int i = 0; i < 2; ++i) FAMSA_HIP(hipStreamWaitEvent(cs[i], ev_user, 0));
  }
  const auto t0 = std::chrono::steady_clock::now();
  auto issue = [&](uint64_t s) -> int {
    const int slot = (int)(s % nslots);
    if (s >= s0 + nslots) FAMSA_HIP(hipStreamWaitEvent(cstream(slot), ev_copy[slot], 0));  // buffer reuse
    int rc = enqueue_step(s, slot, timed);
    if (rc) return rc;
    if (!dev_tiles) {
      FAMSA_HIP(hipStreamWaitEvent(xs, ev_comp[slot], 0));
      FAMSA_HIP(hipMemcpyAsync(h_out[slot].p, d_out[slot].p, steps[s].values * sizeof(int32_t), hipMemcpyDeviceToHost,
                               xs));
      FAMSA_HIP(hipEventRecord(ev_copy[slot], xs));
    } else {
      FAMSA_HIP(hipEventRecord(ev_copy[slot], cstream(slot)));
    }
    return 0;
  };
  auto drain = [&]() {
    for (int i = 0; i < 2; ++i) {
      (void)hipEventSynchronize(ev_comp[i]);
      (void)hipEventSynchronize(ev_copy[i]);
    }
  };
  int rc = 0;
  for (uint64_t s = s0; s < ns && s < s0 + nslots && !rc; ++s) rc = issue(s);
  for (uint64_t s = s0; s < ns && !rc; ++s) {
    const int slot = (int)(s % nslots);
    hipError_t e = hipEventSynchronize(dev_tiles ? ev_comp[slot] : ev_copy[slot]);
    if (e != hipSuccess) {
      rc = set_error(FAMSA_LCS_EDEVICE, "step %llu: %s", (unsigned long long)s, hipGetErrorString(e));
      break;
    }
    float stepms = 0.f;
    if (hipEventElapsedTime(&stepms, ev_s0[slot], ev_s1[slot]) == hipSuccess) stats.step_ms += stepms;
    stats.steps++;
    if (timed) {
      for (int c = 0; c < 5; ++c) {
        float km = 0.f;
        if (wl.sigs[s].has(c) &&
            hipEventElapsedTime(&km, ev_k[slot][2 * c], ev_k[slot][2 * c + 1]) == hipSuccess) {
          stats.kernel_ms[c] += km;
          stats.launches[c] += 1;
        }
      }
    }
    for (uint64_t t = std::max(steps[s].tile_begin, first_tile); t < steps[s].tile_end; ++t) {
      const Tile& tl = tiles[t];
      famsa_lcs_tile tile{};
      tile.tile_index = t;
      tile.family = tl.fam;
      tile.k = fam_off[tl.fam + 1] - fam_off[tl.fam];
      tile.row_begin = tl.r0;
      tile.row_end = tl.r1;
      tile.count = tl.count;
      tile.lcs = (dev_tiles ? d_out[slot].as<int32_t>() : h_out[slot].as<int32_t>()) + tl.out_off;
      tile.stream = cstream(slot);
      tile.values = batch.values;
      if (fn(user, &tile) != 0) {
        rc = set_error(FAMSA_LCS_ECANCELED, "tile callback returned nonzero at tile %llu", (unsigned long long)t);
        break;
      }
      stats.tiles++;
    }
    if (!rc && s + nslots < ns) rc = issue(s + nslots);
  }
  if (rc) {
    drain();
    return rc;
  }
  stats.wall_ms = ms_since(t0);
  for (int c = 0; c < 5; ++c) stats.cells[c] = wl.cells[c];
  if (opt.user_stream) {
    for (int i = 0; i < 2; ++i) {
      FAMSA_HIP(hipEventRecord(ev_comp[i], cs[i]));
      FAMSA_HIP(hipStreamWaitEvent(opt.user_stream, ev_comp[i], 0));
    }
  }
  return 0;
}

// ------------------------------------------------------------------ C-ABI

extern "C" {

void famsa_lcs_default_options(famsa_lcs_options* o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->struct_size = sizeof *o;
  o->alphabet_size = 20;
  o->tile_rows = 1024;
  o->device = 0;
  o->stream = nullptr;
  o->hbm_budget = 0;
  o->flags = 0;
  o->cols_per_item = 0;
  o->step_values = 0;
  o->step_cells = 0;
}

const char* famsa_lcs_last_error(void) { return last_error_text(); }

int famsa_lcs_plan(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, const uint32_t* fam_off,
                   uint32_t nfam, const famsa_lcs_options* opt, famsa_lcs_plan_t** out) {
  clear_error();
  if (!out) return set_error(FAMSA_LCS_EINVAL, "out is NULL");
  *out = nullptr;
  Opts o;
  int rc = normalize_options(opt, &o);
  if (rc) return rc;
  std::vector<uint32_t> fo;
  uint32_t maxlen = 0;
  if ((rc = validate_batch(codes, seq_off, nseq, fam_off, nfam, o.sigma, &fo, &maxlen))) return rc;

  famsa_lcs_plan_s* p = new (std::nothrow) famsa_lcs_plan_s();
  if (!p) return set_error(FAMSA_LCS_ENOMEM, "out of host memory");
  p->opt = o;
  p->fam_off = fo;
  auto fail = [&](int code) {
    delete p;
    return code;
  };
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(set_error(FAMSA_LCS_EDEVICE, "no HIP device available"));
  }
  if (o.device >= ndev) return fail(set_error(FAMSA_LCS_EINVAL, "device %d >= device count %d", o.device, ndev));
  if (hipSetDevice(o.device) != hipSuccess) return fail(set_error(FAMSA_LCS_EDEVICE, "hipSetDevice failed"));
  if ((rc = gpu_info(o.device, &p->gi))) return fail(rc);
  if (!(o.flags & FAMSA_LCS_NO_AUTOTUNE)) tune_lookup(p->gi, o.sigma, &p->lp);
  if (o.cols_per_item) p->lp.cols_per_item = o.cols_per_item;
  if (o.flags & FAMSA_LCS_LONG_SEGMENTED) p->lp.long_wl = 0;

  // budget: batch + descriptors + 2 step buffers (+ plain scratch)
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return fail(set_error(FAMSA_LCS_EDEVICE, "hipMemGetInfo failed"));
  const uint64_t budget = o.hbm_budget ? o.hbm_budget : (uint64_t)(freeb * 0.9);
  const uint64_t fixed = DeviceBatchOwner::footprint(seq_off, nseq, o.sigma);
  if (fixed > budget) return fail(set_error(FAMSA_LCS_ENOMEM, "batch needs %llu bytes, budget is %llu",
                                            (unsigned long long)fixed, (unsigned long long)budget));
  if (!o.hbm_budget || fixed + 2 * o.step_values * 4 > budget)
    p->opt.step_values = std::max<uint64_t>(1, std::min<uint64_t>(o.step_values, (budget - fixed) / 16));

  if ((rc = p->host_phase(seq_off, nseq))) return fail(rc);
  if ((rc = p->setup_device())) return fail(rc);
  if ((rc = p->batch.create(codes, seq_off, nseq, o.sigma, p->cs[0]))) return fail(rc);
  p->batch.values = (o.flags & FAMSA_LCS_OUT_INDEL) ? FAMSA_LCS_VALUES_INDEL
                    : (o.flags & FAMSA_LCS_OUT_SIM) ? FAMSA_LCS_VALUES_SIM
                                                    : FAMSA_LCS_VALUES_LCS;
  hipStream_t s = p->cs[0];
  if ((rc = p->upload_work())) return fail(rc);
  if ((rc = p->d_ctl.alloc(2 * sizeof(StepCtl)))) return fail(rc);
  uint64_t step_max = 0;
  for (const auto& st : p->steps) step_max = std::max(step_max, st.values);
  const int nbuf = p->slots();
  for (int i = 0; i < nbuf; ++i) {
    if ((rc = p->d_out[i].alloc(std::max<uint64_t>(step_max, 1) * 4))) return fail(rc);
    if (!(o.flags & FAMSA_LCS_DEVICE_TILES) && (rc = p->h_out[i].alloc(std::max<uint64_t>(step_max, 1) * 4)))
      return fail(rc);
  }
  if ((rc = p->exec.prepare(p->gi.cus, p->lp, p->wl, o.sigma))) return fail(rc);
  if (p->plain()) p->exec.plain_blocks = p->wl.max_plain_pairs ? (uint32_t)std::min<uint64_t>(
                                                                      (p->wl.max_plain_pairs + kPlainBlock - 1) / kPlainBlock,
                                                                      1u << 20)
                                                                : 0;
  if (p->exec.has_long)
    for (int i = 0; i < nbuf; ++i)
      if ((rc = p->d_carry[i].alloc(p->exec.carry_bytes()))) return fail(rc);
  if (p->exec.w64max_plain > plain_register_w64_limit()) {
    p->exec.plain_blocks = std::min<uint32_t>(p->exec.plain_blocks, (uint32_t)p->gi.cus * 8u);
    const uint64_t thr = (uint64_t)p->exec.plain_blocks * kPlainBlock;
    for (int i = 0; i < nbuf; ++i)
      if ((rc = p->d_plainwork[i].alloc(thr * p->exec.w64max_plain * 8))) return fail(rc);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(set_error(FAMSA_LCS_EDEVICE, "upload failed"));
  // host copies no longer needed on the device side
  if (p->use_graph() && (rc = p->capture_graphs())) return fail(rc);
  *out = p;
  return 0;
}

int famsa_lcs_plan_dry_run(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, const uint32_t* fam_off,
                           uint32_t nfam, const famsa_lcs_options* opt, const char* dump_path,
                           famsa_lcs_plan_info* info) {
  clear_error();
  Opts o;
  int rc = normalize_options(opt, &o);
  if (rc) return rc;
  std::vector<uint32_t> fo;
  uint32_t maxlen = 0;
  if ((rc = validate_batch(codes, seq_off, nseq, fam_off, nfam, o.sigma, &fo, &maxlen))) return rc;
  famsa_lcs_plan_s p;
  p.opt = o;
  p.fam_off = fo;
  if (o.cols_per_item) p.lp.cols_per_item = o.cols_per_item;
  if ((rc = p.host_phase(seq_off, nseq))) return rc;
  p.batch.max_len = maxlen;
  if (dump_path && (rc = p.dump(dump_path))) return rc;
  if (info) famsa_lcs_plan_get_info(&p, info);
  return 0;
}

int famsa_lcs_tiles(famsa_lcs_plan_t* p, uint64_t first_tile, famsa_lcs_tile_fn fn, void* user) {
  clear_error();
  if (!p) return set_error(FAMSA_LCS_EINVAL, "plan is NULL");
  if (!fn) return set_error(FAMSA_LCS_EINVAL, "callback is NULL");
  if (first_tile > p->tiles.size())
    return set_error(FAMSA_LCS_EINVAL, "first_tile %llu > tile count %llu", (unsigned long long)first_tile,
                     (unsigned long long)p->tiles.size());
  int expect = 0;
  if (!p->busy.compare_exchange_strong(expect, 1)) return set_error(FAMSA_LCS_EBUSY, "plan is already running");
  int rc = p->run(first_tile, fn, user);
  p->busy.store(0);
  return rc;
}

void famsa_lcs_release(famsa_lcs_plan_t* p) { delete p; }

int famsa_lcs_autotune(famsa_lcs_plan_t* p, const char* cache_path) {
  clear_error();
  if (!p) return set_error(FAMSA_LCS_EINVAL, "plan is NULL");
  int expect = 0;
  if (!p->busy.compare_exchange_strong(expect, 1)) return set_error(FAMSA_LCS_EBUSY, "plan is already running");
  int rc = p->autotune(cache_path);
  p->busy.store(0);
  return rc;
}

int famsa_lcs_plan_get_info(const famsa_lcs_plan_t* p, famsa_lcs_plan_info* info) {
  clear_error();
  if (!p || !info) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  memset(info, 0, sizeof *info);
  info->ntiles = p->tiles.size();
  info->nsteps = p->steps.size();
  info->pairs = p->pairs;
  info->cells = p->cells;
  info->device_bytes = p->batch.bytes + p->d_groups.bytes + p->d_lanes.bytes + p->d_items.bytes + p->d_prows.bytes +
                       p->d_colmap.bytes + p->d_rowbase.bytes + p->d_ranges.bytes + p->d_ctl.bytes +
                       p->d_plainwork[0].bytes + p->d_plainwork[1].bytes + p->d_carry[0].bytes + p->d_carry[1].bytes + p->d_out[0].bytes + p->d_out[1].bytes;
  info->pinned_bytes = p->h_out[0].bytes + p->h_out[1].bytes;
  for (const auto& t : p->tiles) info->max_tile_values = std::max(info->max_tile_values, t.count);
  info->nfam = (uint32_t)p->fam_off.size() - 1;
  info->max_len = p->batch.max_len;
  info->cols_per_item = p->lp.cols_per_item;
  for (int c = 0; c < 4; ++c) info->waves_per_group[c] = p->exec.waves[c];
  return 0;
}

int famsa_lcs_get_stats(const famsa_lcs_plan_t* p, famsa_lcs_stats* st) {
  clear_error();
  if (!p || !st) return set_error(FAMSA_LCS_EINVAL, "NULL argument");
  *st = p->stats;
  return 0;
}

}  // extern "C"
