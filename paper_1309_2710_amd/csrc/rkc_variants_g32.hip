// Kernel variants with 32 lanes per cell.
#include "rkc_integrate.h"
#include "rkc_internal.h"

namespace rkchost {

static const VariantDesc kTable[] = {RKC_VARIANT_PD(32, 1), RKC_VARIANT_PD(32, 2)};

const VariantDesc *variants_g32(int *n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace rkchost
