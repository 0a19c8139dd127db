// Sweep kernels along xi (all modes, precisions, schemes and boundary kinds).
#include "ocfd_sweep.h"

namespace ocfd {
template hipError_t launch_sweep_d<0>(int mode, const SweepArgs& a, hipStream_t st);
}  // namespace ocfd
