// Entry points not built yet.
#include "vx_table.h"

namespace vx {
vx_status join_batch(vx_ctx*, const vx_batch_join*, vx_join_out*) {
  set_error("vx_join_agg: BATCH not built");
  return VX_EUNSUPPORTED;
}
vx_status join_partitioned(vx_ctx*, const vx_partitioned_join*, vx_join_out*) {
  set_error("vx_join_agg: PARTITIONED not built");
  return VX_EUNSUPPORTED;
}
}  // namespace vx

extern "C" vx_status vx_partition(vx_ctx*, const vx_partition_desc*, vx_partition_out*) {
  vx::set_error("vx_partition not built");
  return VX_EUNSUPPORTED;
}
