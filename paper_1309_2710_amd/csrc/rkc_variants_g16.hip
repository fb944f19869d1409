// Kernel variants with 16 lanes per cell.
#include "rkc_integrate.h"
#include "rkc_internal.h"

namespace rkchost {

static const VariantDesc kTable[] = {RKC_VARIANT(16, 1, 2), RKC_VARIANT_PD(16, 1), RKC_VARIANT_PD(16, 2)};

const VariantDesc *variants_g16(int *n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace rkchost
