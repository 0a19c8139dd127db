// Sweep kernels along zeta (all modes, precisions, schemes and boundary kinds).
#include "ocfd_sweep.h"

namespace ocfd {
template hipError_t launch_sweep_d<2>(int mode, const SweepArgs& a, hipStream_t st);
}  // namespace ocfd
