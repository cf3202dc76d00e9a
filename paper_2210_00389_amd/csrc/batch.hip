// batch.hip -- many small graphs in one persistent launch (placeholder until
// the persistent kernel lands; reports an explicit error).
#include "tc_internal.h"

namespace tc {

size_t batch_ws_bytes(int64_t total_n, int64_t total_nnz, int32_t num_graphs) {
  (void)total_n;
  (void)total_nnz;
  (void)num_graphs;
  return 256;
}

int batch_run(const tc_batch*, const tc_tuning*, uint32_t, int64_t*, int64_t*, int32_t*, void*, size_t,
              hipStream_t) {
  return fail(TC_ERR_INVALID_ARG, "tc_count_batch: not available in this build");
}

}  // namespace tc
