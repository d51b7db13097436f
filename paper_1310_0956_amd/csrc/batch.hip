// Batched CGLS over many independent reconstructions (placeholder driver;
// replaced by the shared-work-list batched kernels).
#include "internal.h"
#include "solve.h"

namespace reco {

reco_status solve_batch(int32_t count, const reco_geometry* geoms, const void* const* b,
                        void* const* x, const reco_solve_opts* opts, reco_solve_info* info,
                        hipStream_t st) {
  reco_status worst = RECO_OK;
  for (int i = 0; i < count; ++i) {
    Geometry* g = reinterpret_cast<Geometry*>(geoms[i]);
    reco_status rc = solve_cgls(*g, b[i], x[i], opts[i], info ? &info[i] : nullptr, st);
    if (rc != RECO_OK && worst == RECO_OK) worst = rc;
  }
  return worst;
}

}  // namespace reco

extern "C" {
reco_status reco_server_create(size_t, int32_t, reco_server* out) {
  if (out) *out = nullptr;
  reco::set_error("serving is not available in this build");
  return RECO_EINVAL;
}
reco_status reco_server_destroy(reco_server) { return RECO_OK; }
reco_status reco_submit(reco_server, const reco_geometry_desc*, const void*, void*,
                        const reco_solve_opts*, uint64_t*) {
  reco::set_error("serving is not available in this build");
  return RECO_EINVAL;
}
reco_status reco_poll(reco_server, uint64_t, reco_solve_info*, double*) {
  reco::set_error("serving is not available in this build");
  return RECO_EINVAL;
}
}
