// The int-GMRES(m) kernels (igm_cycle.hpp) whose SpMV splits each
// workgroup's chunk of rows evenly by entries (merge-based partition).
#include "igm_cycle.hpp"

namespace igm {

template const void *cycle_kernel_for<kMapMerge>(int, int, int);

}  // namespace igm
