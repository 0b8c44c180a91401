// FP32 MFMA instances of the core kernel: one to three rank tiles.
#include "txe_core.h"

namespace txe {
template hipError_t launch_core_for_mt<float, 1>(const Tables<float> &, const ChunkArgs<float> &, bool, hipStream_t);
template hipError_t launch_core_for_mt<float, 2>(const Tables<float> &, const ChunkArgs<float> &, bool, hipStream_t);
template hipError_t launch_core_for_mt<float, 3>(const Tables<float> &, const ChunkArgs<float> &, bool, hipStream_t);
}  // namespace txe
