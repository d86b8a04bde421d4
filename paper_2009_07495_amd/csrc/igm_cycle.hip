// The int-GMRES(m) kernels (igm_cycle.hpp) with the SELL-64 SpMV, and the
// lookup over every SpMV mapping; the kernels with lanes per row and with the
// merge-based split are built in igm_cycle_lanes.hip and igm_cycle_merge.hip.
#include "igm_cycle.hpp"

namespace igm {

template const void *cycle_kernel_for<kMapSell>(int, int, int);
extern template const void *cycle_kernel_for<kMapLanes>(int, int, int);
extern template const void *cycle_kernel_for<kMapMerge>(int, int, int);

const void *cycle_kernel(int block, int R, int pre, int spmv_lanes) {
  if (spmv_lanes == IGM_SPMV_MERGE) return cycle_kernel_for<kMapMerge>(block, R, pre);
  if (spmv_lanes > 1) return cycle_kernel_for<kMapLanes>(block, R, pre);
  return cycle_kernel_for<kMapSell>(block, R, pre);
}

size_t cycle_smem_bytes(int m) { return sizeof(int64_t) * (4 * (size_t)m + 2) + sizeof(double) * (size_t)m; }

}  // namespace igm
