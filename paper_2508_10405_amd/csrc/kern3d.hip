// 3D stencil kernels (placeholder until the 3D propagator lands).
#include "common.h"
#include "kernels.h"

namespace lsrtm {

const int kTiles3[][3] = {{64, 4, 32}, {64, 8, 32}, {64, 8, 64}, {32, 8, 64}, {128, 4, 64}, {64, 4, 64}};
const int kNumTiles3 = 6;

hipError_t launch3d(int, int, int, hipStream_t, const Slot*, const int4*, const Coef&, int, int, int) {
    return hipErrorNotSupported;
}

}  // namespace lsrtm
