// Kernel variants with 64 lanes per cell.
#include "rkc_integrate.h"
#include "rkc_internal.h"

namespace rkchost {

static const VariantDesc kTable[] = {RKC_VARIANT(64, 1, 5), RKC_VARIANT_PD(64, 1), RKC_VARIANT_PD(64, 2), RKC_VARIANT_PD(64, 4),
                                     RKC_VARIANT_PD_GLOBAL(64, 2), RKC_VARIANT_PD_GLOBAL(64, 4)};

const VariantDesc *variants_g64(int *n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace rkchost
