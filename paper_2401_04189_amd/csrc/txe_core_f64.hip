// FP64 MFMA instances of the core kernel: one to three rank tiles.
#include "txe_core.h"

namespace txe {
template hipError_t launch_core_for_mt<double, 1>(const Tables<double> &, const ChunkArgs<double> &, bool, hipStream_t);
template hipError_t launch_core_for_mt<double, 2>(const Tables<double> &, const ChunkArgs<double> &, bool, hipStream_t);
template hipError_t launch_core_for_mt<double, 3>(const Tables<double> &, const ChunkArgs<double> &, bool, hipStream_t);
}  // namespace txe
