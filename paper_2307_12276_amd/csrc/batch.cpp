// Batched momentum bins (first version): every bin advanced by its own
// exponential midpoint step, one after the other.
#include "internal.h"
#include "adl.h"

#include <new>
#include <vector>

struct adl_batch {
  std::vector<adl_op*> ops;
};

extern "C" {

size_t adl_batch_workspace_bytes(int nbins, adl_op* const* ops, int max_degree) {
  (void)max_degree;
  if (nbins < 1 || !ops) return 0;
  return 256;
}

int adl_batch_create(int nbins, adl_op* const* ops, void* workspace, size_t ws_bytes, int tile_rows,
                     adl_batch** out) {
  (void)workspace;
  (void)ws_bytes;
  (void)tile_rows;
  if (!out || nbins < 1 || !ops) return ADL_EINVAL;
  adl_batch* b = new (std::nothrow) adl_batch();
  if (!b) return ADL_EINVAL;
  b->ops.assign(ops, ops + nbins);
  *out = b;
  return ADL_OK;
}

int adl_batch_destroy(adl_batch* b) {
  delete b;
  return ADL_OK;
}

int adl_batch_midpoint_step(adl_batch* b, double* const* u, const double* const* S_half, double dt, double tol,
                            int use_graph, adl_stats* per_bin, void* stream) {
  (void)use_graph;
  if (!b || !u) return ADL_EINVAL;
  int rc = ADL_OK;
  for (size_t i = 0; i < b->ops.size(); ++i) {
    const int r = adl_exp_midpoint_step(b->ops[i], u[i], S_half ? S_half[i] : nullptr, dt, tol,
                                        per_bin ? &per_bin[i] : nullptr, stream);
    if (r != ADL_OK && rc == ADL_OK) rc = r;
  }
  return rc;
}

}  // extern "C"
