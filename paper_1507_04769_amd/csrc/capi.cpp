// C ABI glue: status strings, version and the sparse-grid object
// (Sec. 3.2).  The BVP and interpolant entry points live next to their
// kernels (bvp.hip, interp.hip).
#include <cstring>
#include <new>

#include "sgcm_internal.h"

extern "C" const char* sgcm_strerror(int code) {
  switch (code) {
    case SGCM_OK: return "success";
    case SGCM_EINVAL: return "invalid argument";
    case SGCM_ENOMEM: return "out of memory";
    case SGCM_EDEVICE: return "HIP device or launch failure";
    case SGCM_EUNSUPPORTED: return "not supported by this library";
    case SGCM_ENOTCONVERGED: return "node values from a BVP that did not converge";
    default: return "unknown status";
  }
}

extern "C" int sgcm_version(void) { return 20000; }

extern "C" int sgcm_grid_create(int32_t d, int32_t level, const double* lo, const double* hi,
                                sgcm_grid** out) {
  if (!out) return SGCM_EINVAL;
  *out = nullptr;
  if (d < 1 || d > sgcm::kMaxDim || level < 0) return SGCM_EINVAL;
  if (level > sgcm::kMaxLevel) return SGCM_EUNSUPPORTED;
  sgcm_grid* g = new (std::nothrow) sgcm_grid();
  if (!g) return SGCM_ENOMEM;
  int rc;
  try {
    rc = sgcm::build_grid(d, level, lo, hi, &g->g);
  } catch (const std::bad_alloc&) {
    rc = SGCM_ENOMEM;
  }
  if (rc != SGCM_OK) {
    delete g;
    return rc;
  }
  *out = g;
  return SGCM_OK;
}

extern "C" int64_t sgcm_grid_size(const sgcm_grid* g) { return g ? g->g.M : -1; }

extern "C" int sgcm_grid_nodes(const sgcm_grid* gh, double* nodes_host) {
  if (!gh || !nodes_host) return SGCM_EINVAL;
  const sgcm::Grid& g = gh->g;
  for (int64_t a = 0; a < g.M; ++a)
    for (int j = 0; j < g.d; ++j)
      nodes_host[a * g.d + j] = g.lo[j] + (g.hi[j] - g.lo[j]) * g.xi[a * g.d + j];
  return SGCM_OK;
}

extern "C" int sgcm_grid_keys(const sgcm_grid* gh, int32_t* keys_host) {
  if (!gh || !keys_host) return SGCM_EINVAL;
  std::memcpy(keys_host, gh->g.keys.data(), gh->g.keys.size() * sizeof(int32_t));
  return SGCM_OK;
}

extern "C" void sgcm_grid_destroy(sgcm_grid* g) {
  if (!g) return;
  sgcm::free_device_tables(g->g);
  delete g;
}
