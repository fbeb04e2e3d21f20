// msrep_convert (placeholder until the conversion kernels land).
#include "common.hpp"
using namespace msrep;
extern "C" size_t msrep_convert_ws_bytes(const msrep_mat *src, int32_t dst_fmt) {
  (void)src; (void)dst_fmt; return 0;
}
extern "C" msrep_status msrep_convert(const msrep_mat *src, msrep_mat *dst, void *ws_d,
                                      size_t ws_bytes, void *stream) {
  (void)src; (void)dst; (void)ws_d; (void)ws_bytes; (void)stream;
  return fail(MSREP_ERR_UNSUPPORTED, "msrep_convert: not built yet");
}
