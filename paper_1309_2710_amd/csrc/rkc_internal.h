// Internal declarations shared by the host runtime and the kernel variants.
#pragma once

#include <hip/hip_runtime.h>

#include "rkc.h"
#include "rkc_device.h"

namespace rkchost {

// One compiled kernel variant: G lanes per cell, NSL state elements per lane,
// RUC reaction units per lane held in registers (0: parameters read from LDS,
// -1: from global memory, any number of units).
struct VariantDesc {
    int G, NSL, RUC;
    int max_threads;
    const void *k_rkc;
    const void *k_rkck;
    const void *k_rhs;
    // the same kernels with the third-body/falloff rounds (null: not built)
    const void *k_rkc_pd;
    const void *k_rkck_pd;
    const void *k_rhs_pd;
};

const VariantDesc *variants_g64(int *n);
const VariantDesc *variants_g32(int *n);
const VariantDesc *variants_g16(int *n);
const VariantDesc *variants_g8(int *n);
// one lane per cell (G = 1, NSL = the state capacity NMAX of the kernel)
const VariantDesc *variants_lane(int *n);

// Aggregate counters per launch (n_rhs, n_steps, n_reject, n_sigma,
// n_power_iter, s_max_used, n_failed, worst_status, issued slots; rest spare).
constexpr int AGG_N = 16;

// What one integrator launch ran (for rkc_stats).
struct LaunchInfo {
    int G = 0, RUC = 0, blocks = 0, threads = 0;
    bool persistent = false;
    size_t lds = 0;
};

}  // namespace rkchost


namespace rkchost {

// Validate the scalar arguments and options of an integration.
int check_integrate_args(double dt, double rtol, double atol, const rkc_opts &o);

// Enqueue one integration of n cells whose arrays are device pointers on the
// mechanism's device, with the launch's own scratch (aggregate counters
// [16], work-queue head): launches that use distinct scratch may run
// concurrently on different streams.  Not thread-safe for one mechanism
// (its per-shape table cache is filled on first use).  With may_build false
// nothing is allocated: RKC_ENOTSUP if the tables of the selected variant
// have not been built by an earlier call.
int enqueue_integrate(rkc_mech *m, size_t n, double *Td, const double *Pd, double *Yd, double dt,
                      double rtol, double atol, const rkc_opts &o, int32_t *sd, int32_t *cd,
                      unsigned long long *agg_d, int *queue_d, hipStream_t st, LaunchInfo *li,
                      bool may_build = true);

// Select the variant and build the device tables a later enqueue_integrate
// with these options will use (so that concurrent launches only read them);
// with n_cells > 0 also fix the kernels' launch attributes for that size.
int prepare(rkc_mech *m, const rkc_opts &o, size_t n_cells);
int mech_species(const rkc_mech *m);
int mech_device(const rkc_mech *m);

// Statistics of one launch from its aggregate counters ([16], see the kernels).
void fill_stats(const unsigned long long *agg, const LaunchInfo &li, rkc_stats *stats);

}  // namespace rkchost

// A variant with plain-reaction kernels only (register-resident parameters).
#define RKC_VARIANT(G_, NSL_, RUC_)                                                            \
    rkchost::VariantDesc {                                                                     \
        G_, NSL_, RUC_, (rkcdev::Occ<RUC_, NSL_>::threads),                                    \
            reinterpret_cast<const void *>(&rkcdev::rkc_kernel<G_, NSL_, RUC_, false>),        \
            reinterpret_cast<const void *>(&rkcdev::rkck_kernel<G_, NSL_, RUC_, false>),       \
            reinterpret_cast<const void *>(&rkcdev::rhs_kernel<G_, NSL_, RUC_, false>),        \
            nullptr, nullptr, nullptr                                                          \
    }

// A variant with both kernel sets (parameters in LDS).
// Plain and pressure-dependent kernels with the reaction parameters and the
// species table in global memory (RUC = -1).
#define RKC_VARIANT_PD_GLOBAL(G_, NSL_)                                                        \
    rkchost::VariantDesc {                                                                     \
        G_, NSL_, -1, (rkcdev::Occ<-1, NSL_>::threads),                                        \
            reinterpret_cast<const void *>(&rkcdev::rkc_kernel<G_, NSL_, -1, false>),          \
            reinterpret_cast<const void *>(&rkcdev::rkck_kernel<G_, NSL_, -1, false>),         \
            reinterpret_cast<const void *>(&rkcdev::rhs_kernel<G_, NSL_, -1, false>),          \
            reinterpret_cast<const void *>(&rkcdev::rkc_kernel<G_, NSL_, -1, true>),           \
            reinterpret_cast<const void *>(&rkcdev::rkck_kernel<G_, NSL_, -1, true>),          \
            reinterpret_cast<const void *>(&rkcdev::rhs_kernel<G_, NSL_, -1, true>)            \
    }

#define RKC_VARIANT_PD(G_, NSL_)                                                               \
    rkchost::VariantDesc {                                                                     \
        G_, NSL_, 0, (rkcdev::Occ<0, NSL_>::threads),                                          \
            reinterpret_cast<const void *>(&rkcdev::rkc_kernel<G_, NSL_, 0, false>),           \
            reinterpret_cast<const void *>(&rkcdev::rkck_kernel<G_, NSL_, 0, false>),          \
            reinterpret_cast<const void *>(&rkcdev::rhs_kernel<G_, NSL_, 0, false>),           \
            reinterpret_cast<const void *>(&rkcdev::rkc_kernel<G_, NSL_, 0, true>),            \
            reinterpret_cast<const void *>(&rkcdev::rkck_kernel<G_, NSL_, 0, true>),           \
            reinterpret_cast<const void *>(&rkcdev::rhs_kernel<G_, NSL_, 0, true>)             \
    }
