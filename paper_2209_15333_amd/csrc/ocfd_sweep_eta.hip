// Sweep kernels along eta (all modes, precisions, schemes and boundary kinds).
#include "ocfd_sweep.h"

namespace ocfd {
template hipError_t launch_sweep_d<1>(int mode, const SweepArgs& a, hipStream_t st);
}  // namespace ocfd
