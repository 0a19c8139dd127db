// Sweep kernels along xi reconstructing component by component (all
// modes, precisions, schemes and boundary kinds).
#include "ocfd_sweep.h"

namespace ocfd {
template hipError_t launch_sweep_dc<0, false>(int mode, const SweepArgs& a, hipStream_t st);
}  // namespace ocfd
