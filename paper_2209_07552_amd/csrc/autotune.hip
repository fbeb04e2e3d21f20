#include "common.hpp"
using namespace msrep;
extern "C" size_t msrep_autotune_ws_bytes(const msrep_mat *) { return 0; }
extern "C" msrep_status msrep_autotune(const msrep_mat *, const void *, void *, size_t, msrep_tune *, void *) {
  return fail(MSREP_ERR_UNSUPPORTED, "msrep_autotune: not built yet");
}
