// Kernel variants with 8 lanes per cell.
#include "rkc_integrate.h"
#include "rkc_internal.h"

namespace rkchost {

static const VariantDesc kTable[] = {RKC_VARIANT(8, 2, 3), RKC_VARIANT(8, 2, 4), RKC_VARIANT_PD(8, 2), RKC_VARIANT_PD(8, 4)};

const VariantDesc *variants_g8(int *n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace rkchost
