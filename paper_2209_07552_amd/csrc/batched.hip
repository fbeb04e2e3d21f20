#include "common.hpp"
using namespace msrep;
extern "C" size_t msrep_plan_ws_bytes(int32_t, const msrep_mat *, const msrep_tune *) { return 0; }
extern "C" msrep_status msrep_plan_create(int32_t, const msrep_mat *, const msrep_tune *, double,
                                          double, void *, size_t, void *, msrep_plan *) {
  return fail(MSREP_ERR_UNSUPPORTED, "msrep_plan_create: not built yet");
}
extern "C" msrep_status msrep_spmv_batched(msrep_plan, const void *const *, void *const *, void *) {
  return fail(MSREP_ERR_UNSUPPORTED, "msrep_spmv_batched: not built yet");
}
extern "C" int64_t msrep_plan_items(msrep_plan) { return 0; }
extern "C" msrep_status msrep_plan_destroy(msrep_plan) { return MSREP_OK; }
