// Launch-parameter tuning: candidates (waves per workgroup per length class,
// columns per work item, the long rows' word width per lane) are timed on the
// plan's own first step and the winner is stored in a small text cache keyed
// by GPU architecture and alphabet size.  Parameters only change scheduling,
// never results.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "runtime.h"

namespace famsa {

static std::string cache_key(const GpuInfo& gi, uint32_t sigma) {
  std::string a = gi.arch;
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a.resize(colon);
  return a + "/sigma" + std::to_string(sigma);
}

// Cache format: one line per key,
//   `key waves0 waves1 waves2 cols [long_dwords waves3]`
// (long_dwords: the most dwords per lane of the lanes-per-row mode, 0 for the
// segmented long-row kernel; lines without the last two fields keep the
// defaults for them).
int tune_lookup(const GpuInfo& gi, uint32_t sigma, LaunchParams* lp) {
  const char* path = getenv("FAMSA_LCS_TUNE_CACHE");
  if (!path || !*path) return 0;
  FILE* f = fopen(path, "r");
  if (!f) return 0;
  const std::string key = cache_key(gi, sigma);
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char k[256];
    unsigned w0 = 0, w1 = 0, w2 = 0, c = 0, lw = 0, w3 = 0;
    const int n = sscanf(line, "%255s %u %u %u %u %u %u", k, &w0, &w1, &w2, &c, &lw, &w3);
    if (n < 5 || key != k || !w0 || !w1 || !w2 || !c) continue;
    lp->waves[0] = w0;
    lp->waves[1] = w1;
    lp->waves[2] = w2;
    lp->cols_per_item = c;
    if (n == 7 && w3) {
      lp->long_wl = lw;
      lp->waves[3] = w3;
    }
  }
  fclose(f);
  return 0;
}

int tune_store(const GpuInfo& gi, uint32_t sigma, const LaunchParams& lp, const char* path) {
  if (!path || !*path) path = getenv("FAMSA_LCS_TUNE_CACHE");
  if (!path || !*path) return 0;
  const std::string key = cache_key(gi, sigma);
  std::string keep;
  if (FILE* f = fopen(path, "r")) {
    char line[512];
    while (fgets(line, sizeof line, f)) {
      char k[256];
      if (sscanf(line, "%255s", k) == 1 && key == k) continue;
      keep += line;
    }
    fclose(f);
  }
  FILE* f = fopen(path, "w");
  if (!f) return set_error(FAMSA_LCS_EINVAL, "cannot write tuning cache %s", path);
  fputs(keep.c_str(), f);
  fprintf(f, "%s %u %u %u %u %u %u\n", key.c_str(), lp.waves[0], lp.waves[1], lp.waves[2], lp.cols_per_item,
          lp.long_wl == kLongWlAuto ? skew_wl_max(sigma) : lp.long_wl, lp.waves[3]);
  fclose(f);
  return 0;
}

}  // namespace famsa
