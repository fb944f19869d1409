// Internal declarations shared by the host runtime and the kernel variants.
#pragma once

#include <hip/hip_runtime.h>

#include "rkc_device.h"

namespace rkchost {

// One compiled kernel variant: G lanes per cell, NSL state elements per lane,
// RUC reaction units per lane held in registers (0: parameters read from LDS,
// any number of units).
struct VariantDesc {
    int G, NSL, RUC;
    int max_threads;
    const void *k_rkc;
    const void *k_rkck;
    const void *k_rhs;
};

const VariantDesc *variants_g64(int *n);
const VariantDesc *variants_g32(int *n);
const VariantDesc *variants_g16(int *n);
const VariantDesc *variants_g8(int *n);

}  // namespace rkchost

#define RKC_VARIANT(G_, NSL_, RUC_)                                                            \
    rkchost::VariantDesc {                                                                     \
        G_, NSL_, RUC_, (rkcdev::Occ<RUC_, NSL_>::threads),                                          \
            reinterpret_cast<const void *>(&rkcdev::rkc_kernel<G_, NSL_, RUC_>),               \
            reinterpret_cast<const void *>(&rkcdev::rkck_kernel<G_, NSL_, RUC_>),              \
            reinterpret_cast<const void *>(&rkcdev::rhs_kernel<G_, NSL_, RUC_>)                \
    }
