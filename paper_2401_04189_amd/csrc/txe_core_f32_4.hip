// FP32 MFMA instances of the core kernel: four rank tiles.
#include "txe_core.h"

namespace txe {
template hipError_t launch_core_for_mt<float, 4>(const Tables<float> &, const ChunkArgs<float> &, bool, hipStream_t);
}  // namespace txe
