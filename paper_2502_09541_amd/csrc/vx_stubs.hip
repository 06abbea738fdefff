// Entry points not built yet.
#include "vx_table.h"

namespace vx {
vx_status join_batch(vx_ctx*, const vx_batch_join*, vx_join_out*) {
  set_error("vx_join_agg: BATCH not built");
  return VX_EUNSUPPORTED;
}
}  // namespace vx
