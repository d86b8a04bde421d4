// The int-GMRES(m) kernels (igm_cycle.hpp) whose SpMV runs 4, 16 or 64 lanes
// per row over the CSR layout.
#include "igm_cycle.hpp"

namespace igm {

template const void *cycle_kernel_for<kMapLanes>(int, int, int);

}  // namespace igm
