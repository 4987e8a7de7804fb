// Launch-parameter tuning: candidate (waves per workgroup per length class,
// columns per work item) are timed on the plan's own first steps and the
// winner is stored in a small JSON cache keyed by GPU architecture and
// alphabet size.  Parameters only change scheduling, never results.
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

// Cache format: one line per key, `key waves0 waves1 waves2 cols`.
int tune_lookup(const GpuInfo& gi, uint32_t sigma, LaunchParams* lp) {
  const char* path = getenv("FAMSA_LCS_TUNE_CACHE");
  if (!path || !*path) return 0;
  FILE* f = fopen(path, "r");
  if (!f) return 0;
  const std::string key = cache_key(gi, sigma);
  char k[256];
  unsigned w0, w1, w2, c;
  while (fscanf(f, "%255s %u %u %u %u", k, &w0, &w1, &w2, &c) == 5) {
    if (key == k && w0 && w1 && w2 && c) {
      lp->waves[0] = w0;
      lp->waves[1] = w1;
      lp->waves[2] = w2;
      lp->cols_per_item = c;
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
  fprintf(f, "%s %u %u %u %u\n", key.c_str(), lp.waves[0], lp.waves[1], lp.waves[2], lp.cols_per_item);
  fclose(f);
  return 0;
}

}  // namespace famsa
