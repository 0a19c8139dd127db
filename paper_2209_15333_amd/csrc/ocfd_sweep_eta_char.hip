// Sweep kernels along eta reconstructing in characteristic variables (all
// modes, precisions, schemes and boundary kinds).
#include "ocfd_sweep.h"

namespace ocfd {
template hipError_t launch_sweep_dc<1, true>(int mode, const SweepArgs& a, hipStream_t st);
}  // namespace ocfd
