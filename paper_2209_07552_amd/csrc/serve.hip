#include "common.hpp"
using namespace msrep;
extern "C" msrep_status msrep_serve(const msrep_serve_cfg *, const msrep_host_mat *, int32_t,
                                    const msrep_request *, int64_t, msrep_result *, msrep_serve_stats *) {
  return fail(MSREP_ERR_UNSUPPORTED, "msrep_serve: not built yet");
}
