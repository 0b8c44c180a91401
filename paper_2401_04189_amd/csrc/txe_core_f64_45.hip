// FP64 MFMA instances of the core kernel: four and five rank tiles.
#include "txe_core.h"

namespace txe {
template hipError_t launch_core_for_mt<double, 4>(const Tables<double> &, const ChunkArgs<double> &, bool, hipStream_t);
template hipError_t launch_core_for_mt<double, 5>(const Tables<double> &, const ChunkArgs<double> &, bool, hipStream_t);
}  // namespace txe
