// Serving loop (placeholder until the scheduler lands).
#include "runtime.h"

extern "C" {
int famsa_lcs_server_create(const famsa_lcs_options*, famsa_lcs_server_t** out) {
  if (out) *out = nullptr;
  return famsa::set_error(FAMSA_LCS_EINVAL, "serving is not available in this build");
}
int famsa_lcs_server_submit(famsa_lcs_server_t*, const uint8_t*, const uint64_t*, uint32_t, uint32_t*) {
  return famsa::set_error(FAMSA_LCS_EINVAL, "serving is not available in this build");
}
int famsa_lcs_server_step(famsa_lcs_server_t*, famsa_lcs_tile_fn, void*, uint32_t*) {
  return famsa::set_error(FAMSA_LCS_EINVAL, "serving is not available in this build");
}
int famsa_lcs_server_job_state(const famsa_lcs_server_t*, uint32_t, int*) {
  return famsa::set_error(FAMSA_LCS_EINVAL, "serving is not available in this build");
}
int famsa_lcs_server_memory(const famsa_lcs_server_t*, uint64_t*, uint64_t*) {
  return famsa::set_error(FAMSA_LCS_EINVAL, "serving is not available in this build");
}
void famsa_lcs_server_destroy(famsa_lcs_server_t*) {}
int famsa_lcs_autotune(famsa_lcs_plan_t*, const char*) {
  return famsa::set_error(FAMSA_LCS_EINVAL, "autotune is not available in this build");
}
}
