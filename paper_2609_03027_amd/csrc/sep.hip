// Separable DFT-as-GEMM (EPIC_XFORM_DFT_SEPARABLE): Eq. 1's outer sum for one
// sample's grid G as F G F^T, F the centred DFT matrix restricted to the
// gridded region's columns.
#include "internal.h"

namespace epic {

epic_status sep_build(epic_plan, const std::vector<int> &, const std::vector<double> &,
                      hipStream_t) {
    return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM is not built yet");
}

epic_status sep_accumulate(epic_plan, epic_acc, const uint8_t *, int, hipStream_t) {
    return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM is not built yet");
}

}  // namespace epic
