// Mixed-precision walk kernel (int32 voxel index + fp32 offset).
#include "rms_internal.h"

namespace rms {

hipError_t launch_walk_mixed(const WalkPlan&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace rms
