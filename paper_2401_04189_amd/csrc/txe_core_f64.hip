// FP64 MFMA instances of the core kernel.
#include "txe_core.h"

namespace txe {
template hipError_t launch_core<double>(const Tables<double> &, const ChunkArgs<double> &, bool, hipStream_t);
}  // namespace txe
