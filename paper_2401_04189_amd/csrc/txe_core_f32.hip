// FP32 MFMA instances of the core kernel.
#include "txe_core.h"

namespace txe {
template hipError_t launch_core<float>(const Tables<float> &, const ChunkArgs<float> &, bool, hipStream_t);
}  // namespace txe
