// Kernel variants with one lane per cell, by the capacity NMAX of the state
// vectors (N = n_species + 1 <= NMAX elements per lane).
#include "rkc_internal.h"
#include "rkc_lane.h"

#define RKC_LANE_VARIANT(NMAX_)                                                                \
    rkchost::VariantDesc {                                                                     \
        1, NMAX_, 0, 256,                                                                      \
            reinterpret_cast<const void *>(&rkcdev::rkc_lane_kernel<NMAX_, false>),            \
            reinterpret_cast<const void *>(&rkcdev::rkck_lane_kernel<NMAX_, false>),           \
            reinterpret_cast<const void *>(&rkcdev::rhs_lane_kernel<NMAX_, false>),            \
            reinterpret_cast<const void *>(&rkcdev::rkc_lane_kernel<NMAX_, true>),             \
            reinterpret_cast<const void *>(&rkcdev::rkck_lane_kernel<NMAX_, true>),            \
            reinterpret_cast<const void *>(&rkcdev::rhs_lane_kernel<NMAX_, true>)              \
    }

namespace rkchost {

static const VariantDesc kTable[] = {RKC_LANE_VARIANT(10), RKC_LANE_VARIANT(14), RKC_LANE_VARIANT(16),
                                     RKC_LANE_VARIANT(24), RKC_LANE_VARIANT(32)};

const VariantDesc *variants_lane(int *n) {
    *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace rkchost
