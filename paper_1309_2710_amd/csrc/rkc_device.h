// Device code of the batched chemical-kinetics integrator (gfx950, FP64).
//
// One cell (an independent kinetics ODE, Sec. 2.2) is owned by a group of G
// lanes of a 64-wide wavefront (G = 8, 16, 32 or 64).  Inside a group:
//   - state element k of y = {T, Y_1..Y_nS} lives on lane k % G, slot k / G;
//   - reaction unit p (a forward/reverse pair, or one unpaired reaction) is
//     evaluated by lane p % G, round p / G;
//   - the net production sum (E:spec-rate) is a load-balanced gather in two
//     levels of fixed shape: each species' nonzero terms, split by the sign
//     of nu'' - nu', are cut into chunks of at most SEGL terms; chunk c goes
//     to lane c % G, segment c / G, and every lane runs the same NSEG
//     segments of SEGL terms (short chunks padded with a zero term), so the
//     loop has no divergence and a segment's loads issue back to back.  A
//     term is the 16-bit byte offset of a unit's net rate q (|nu''-nu'| = 2
//     or 3 repeats the term).  Each segment's sum is a "piece"; then the lane
//     of state index k adds the L2P positive and subtracts the L2N negative
//     pieces of species k (16-bit offsets into the piece array, padded with
//     its zero slot), again the same count in every lane;
//   - norms and mixture sums are reductions over the G lanes by DPP exchanges
//     inside 16-lane rows and DPP row broadcasts across them, so every lane of
//     a group holds bitwise identical scalars and takes the same decisions.
//     (ds_swizzle butterflies issue fewer vector instructions but lengthen
//     the dependent chain; measured slower at four waves per SIMD.)
// The integrator is written as a state machine in which every iteration of
// the main loop performs exactly one source-term evaluation for every group
// of the wave, whatever phase (power iteration, initial step, Chebyshev stage,
// error check, Cash-Karp stage) each group is in.  The expensive part of the
// loop therefore never diverges; only the cheap per-phase bookkeeping does.
// A group that finishes its cell pulls the next one from a device queue.
//
// Mechanism tables are staged once per workgroup into LDS (species thermo,
// the gather table and, for large mechanisms, the reaction parameters); for
// small enough mechanisms the reaction parameters of a lane's units are held
// in registers for the lifetime of the wave.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rkcdev {

constexpr double R_ERG = 8.31446261815324e7;   // erg/(mol K)
constexpr double KAPPA = 2.0 / 13.0;           // RKC damping (Sec. 2.4)

// Species table fields, stored field-major as spec[field * NK + k] where k is
// the state index (k = 0 is temperature: all fields zero).
enum {
    F_W = 0, F_INVW = 1, F_TMID = 2,
    F_CPLO = 3,   // a1..a5 of the low range (Cp/R Horner)
    F_HLO = 8,    // a1, a2/2, a3/3, a4/4, a5/5, a6 of the low range (H/(RT))
    F_CPHI = 14,
    F_HHI = 19,
    NFIELD = 25
};

// Reaction unit record: 8 doubles.
//   [0..2] log2 A, beta, theta' = (Ea/R) log2(e) of the forward reaction
//   [3..5] the same for the reverse reaction (log2 A = -1e4 for an unpaired
//          reaction, so its reverse rate underflows to exactly zero)
//   [6]    bit pattern: forward reactant slots, three 16-bit byte offsets
//          into the concentration array (bits 0..47); an empty slot points
//          at C[n_species], which holds 1.0
//   [7]    bit pattern: the reverse reaction's reactant slots, same layout
constexpr int UNIT_DOUBLES = 8;

// Pressure-dependent unit record (third body and falloff), 12 doubles:
//   [0] bit pattern: kind (bits 0..7; 1 third body, 2 Lindemann, 3 Troe) and
//       efficiency set (bits 8..15)
//   [1..3] log2 A0, beta0, theta0' of the forward low-pressure limit k_0
//   [4..6] the same for the reverse reaction (log2 A0 = -1e4 if unpaired)
//   [7] unused; [8..11] Troe a, log2(e)/T***, log2(e)/T*, T** log2(e)
//       (T** <= 0: term absent)
// Units of the rounds that hold pressure-dependent units have one record each
// (kind 0 for the plain ones there), lane-interleaved like the unit records.
constexpr int PDEP_DOUBLES = 12;
constexpr int MAX_EFFSETS = 16;

struct Tables {
    const double *units;     // [RU * G][8]
    const double *units_il;  // [RU + 1][4][G] double2: the same records lane-interleaved
                             // as in LDS, one zero round after the last (read from
                             // global memory by the RUC = -1 kernels)
    const double *pdep;      // [NPR * G][12], interleaved by lane (rounds RUp..RU-1)
    const double *eff;       // [NMS][NK] third-body efficiencies by state index
    const double *spec;      // [NFIELD][NK]
    const uint32_t *gather;  // [NSEG * SEGL / 2][G]: two 16-bit terms per word
    const uint32_t *gather2; // [NSL * (L2P + L2N) / 2][G]: pieces of state index
                             // k = s G + g, positive then negative, two per word
};

// A gather term is the byte offset, inside the group's rate array, of a unit's
// net rate q (RU G entries plus one slot that is always zero, for padding).
constexpr uint32_t TERM_MAX_BYTES = 0xffffu;

struct Params {
    int nS, N, NK, nU, RU, NSEG, SEGL, L2P, L2N;
    int RUp, NPR, NMS;               // first round with pressure-dependent units, their
                                     // rounds (RUp + NPR = RU), efficiency sets
    int RU2;                         // rounds [0, RU2): no side has a third reactant slot
    double invTmax;                  // bound on the 1/T of the Arrhenius factors (keeps
                                     // every base-2 exponent below 2^30 in magnitude)
    Tables tab;
    int n_cells;
    double *T;
    const double *P;
    double *Y;
    double *F;                       // source-term output [n][N] (rhs kernel only)
    double dt, rtol, atol;
    int s_max, max_steps;
    int32_t *cell_status;            // optional
    int32_t *cell_counters;          // optional [n][8]
    unsigned long long *agg;         // [16] aggregate counters
    const double *coef;              // RKC stage coefficients for s <= coef_smax (see
                                     // coef_offset), or null
    int coef_smax;
    double invN;                     // 1 / N
    int *queue;                      // persistent work-queue head
    int persistent;
    int groups_total;                // groups in the launched grid
    // element (cell, i) of Y is Y[cell * ycs + i * yss] and element (cell, k)
    // of F is F[cell * fcs + k * fss]: (n_species, 1) and (N, 1) for
    // cell-major arrays, (1, n_cells) for species-major (cell-fastest) ones
    long long ycs, yss, fcs, fss;
    // one-lane-per-cell kernels (rkc_lane.h): wave-uniform tables read with
    // scalar loads, and the LDS rows of one wave
    const double *l_spec;            // [nS][LS_FIELDS] species records
    const double *l_units;           // [nU][LU_DOUBLES] unit records with their terms
    const double *l_pdep;            // [units past n_plain][PDEP_DOUBLES], unit order
    const double *l_eff;             // [NMS][nS] third-body efficiencies
    int n_plain;                     // units [0, n_plain) have no pressure dependence
    int lane_rows;                   // LDS rows of 64 doubles per wave
};

// RKC stage coefficients (E:rkc1, E:rkcj) depend on the stage count s and
// the stage j only.  For s <= coef_smax they are read from a table of 4
// doubles per (s, j), j = 1..s, starting at entry coef_offset(s): entry j = 1
// holds (mu~_1, 0, 0, 0), entry j >= 2 (mu_j, nu_j, mu~_j, gamma~_j).
__host__ __device__ inline int coef_offset(int s) { return (s - 1) * s / 2 - 1; }

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)v, lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// DPP controls: quad_perm [1,0,3,2] (xor 1), [2,3,0,1] (xor 2), row_half_mirror
// (lane i <-> 7-i within 8), row_mirror (lane i <-> 15-i within 16).  After the
// four exchanges every lane of a 16-lane row holds the row sum, computed as
// a + b in one lane and b + a in its partner (identical in IEEE arithmetic).
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

// DPP row broadcasts (wave64): lane 15 of each row into the whole next row
// (row 0 has no source), and lane 31 into rows 2 and 3.  Lanes without a
// source keep an unspecified value; the reductions below never read them.
constexpr int DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

// Sum over the G lanes of a group (G = 8, 16, 32, 64); every lane of the
// group receives the bitwise same value.  With row sums r0..r3, a 64-lane
// group gets (r0 + r1) + (r2 + r3) and a 32-lane group r0 + r1 or r2 + r3:
// row 1 adds row 0's sum and row 3 row 2's, row 3 then adds row 1's, and the
// totals are read from lanes 31 and 63.
template <int G>
__device__ __forceinline__ double gsum(double x) {
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "group size");
    x += dpp_f64<DPP_XOR1>(x);
    x += dpp_f64<DPP_XOR2>(x);
    x += dpp_f64<DPP_HALF_MIRROR>(x);
    if constexpr (G >= 16) x += dpp_f64<DPP_MIRROR>(x);
    if constexpr (G >= 32) x += dpp_f64<DPP_BCAST15>(x);
    if constexpr (G == 32) {
        const double lo = readlane_f64(x, 31), hi = readlane_f64(x, 63);
        x = (__lane_id() < 32) ? lo : hi;
    } else if constexpr (G == 64) {
        x += dpp_f64<DPP_BCAST31>(x);
        x = readlane_f64(x, 63);
    }
    return x;
}

// Two sums at once.  For a 64-lane group the upper half of a trades places
// with the lower half of b (v_permlane32_swap), so that one addition leaves
// a's half-sums (a_l + a_{l+32}) in lanes 0..31 and b's in lanes 32..63; the
// row reductions and one row broadcast then serve both, and the totals are
// read from lanes 31 and 63.  Every lane receives the bitwise same values.
template <int G>
__device__ __forceinline__ void gsum2(double &a, double &b) {
    if constexpr (G == 64) {
        const long long va = __double_as_longlong(a), vb = __double_as_longlong(b);
        const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)va, (unsigned)vb, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(va >> 32), (unsigned)(vb >> 32),
                                                         false, false);
        const double a2 = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
        const double b2 = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
        double x = a2 + b2;
        x += dpp_f64<DPP_XOR1>(x);
        x += dpp_f64<DPP_XOR2>(x);
        x += dpp_f64<DPP_HALF_MIRROR>(x);
        x += dpp_f64<DPP_MIRROR>(x);
        x += dpp_f64<DPP_BCAST15>(x);
        a = readlane_f64(x, 31);
        b = readlane_f64(x, 63);
    } else {
        a = gsum<G>(a);
        b = gsum<G>(b);
    }
}

// Maximum over the group's lanes, combined in the same pattern as gsum.
template <int G>
__device__ __forceinline__ double gmax(double x) {
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "group size");
    x = fmax(x, dpp_f64<DPP_XOR1>(x));
    x = fmax(x, dpp_f64<DPP_XOR2>(x));
    x = fmax(x, dpp_f64<DPP_HALF_MIRROR>(x));
    if constexpr (G >= 16) x = fmax(x, dpp_f64<DPP_MIRROR>(x));
    if constexpr (G >= 32) x = fmax(x, dpp_f64<DPP_BCAST15>(x));
    if constexpr (G == 32) {
        const double lo = readlane_f64(x, 31), hi = readlane_f64(x, 63);
        x = (__lane_id() < 32) ? lo : hi;
    } else if constexpr (G == 64) {
        x = fmax(x, dpp_f64<DPP_BCAST31>(x));
        x = readlane_f64(x, 63);
    }
    return x;
}

// Logical OR over the group's lanes (lanes of other groups are masked off).
template <int G>
__device__ __forceinline__ int gor(int x) {
    const unsigned long long b = __ballot(x != 0);
    if constexpr (G == 64) {
        return b != 0ull;
    } else {
        const int base = (int)(__lane_id() / G) * G;
        return ((b >> base) & ((1ull << G) - 1ull)) != 0ull;
    }
}

// Value of lane 0 of the group.
template <int G>
__device__ __forceinline__ double gbcast0(double x) {
    if constexpr (G == 64) return readlane_f64(x, 0);
    else return __shfl(x, 0, G);
}

// Registers holding the reaction parameters of a lane's units (RUC > 0).
template <int RUC>
struct UnitRegs {
    double l2Af[RUC], bf[RUC], tf[RUC], l2Ar[RUC], br[RUC], tr[RUC];
    uint32_t idf[RUC], idr[RUC];
};
template <>
struct UnitRegs<0> {};
template <>
struct UnitRegs<-1> {};

struct GroupLds {
    const double *spec;
    const double *tmid;    // [NK] range switch temperatures (LDS in every variant)
    const uint32_t *gather;
    const uint32_t *gather2;
    const double *units;   // interleaved records: LDS (RUC == 0) or global (RUC == -1)
    const double *pdep;    // pressure-dependent records of rounds RUp.. (LDS)
    const double *eff;     // [NMS][NK] efficiency sets (LDS)
    double *Mv;            // [NMS] third-body concentrations of the sets
    double *C;             // [NK] concentrations, C[nS] == 1.0
    double *Q;             // [RU G + 2]: net rates q, then a zero slot
    double *piece;         // [NSEG * G + 2]: partial sums of the gather, then a zero slot
};

// log2 k = log2 A + beta log2 T - theta' / T (E:rxn-const in base 2, with
// theta' = theta log2(e) and log2 A stored per reaction) and the net rate of
// a forward/reverse pair, each with its roundings written out as FMAs: left
// to the compiler, the contraction of a sum of products may differ between
// kernel variants, and every variant must form the same values.
__device__ __forceinline__ double arrhenius_arg(double l2A, double beta, double theta2,
                                                double l2T, double invT) {
    return __builtin_fma(-theta2, invT, __builtin_fma(beta, l2T, l2A));
}

__device__ __forceinline__ double net_rate(double kf, double cf, double kr, double cr) {
    return __builtin_fma(kf, cf, -(kr * cr));
}

__device__ __forceinline__ double unpack_c(const double *C, uint32_t id, int s) {
    return C[(id >> (10 * s)) & 1023u];
}

// 2^y: y = n + f with n = round(y), rounded by adding 1.5 * 2^52, and
// f = y - n, which is exact (|f| <= 1/2); then 2^f = 1 + f (L + f q(f)) with
// L = ln 2 and q a degree-9 Chebyshev fit of (2^f - 1 - f ln 2)/f^2 on
// [-1/2, 1/2] (relative error below 2.7e-17; fit_exp_poly.py prints the
// coefficients), by Horner, scaled by 2^n.  Within about one ulp; every
// Horner step is one FMA.  The rate constants are exponentials of sums that
// already carry a rounding of order |y| 2^-53, so a base-2 argument formed
// from base-2 parameters loses nothing against a two-part ln 2 reduction of
// a natural-log argument, and saves its extra FMA.
//
// Two ways of applying 2^n:
// * exp2_sat: n converted to int32 with saturation (v_cvt_i32_f64 clamps),
//   so every |y| < 2^51 gives 0 below about -1075, +inf above 1024 (and
//   larger |y| keep f within a few units, the polynomial positive for
//   positive f, so the result still saturates); NaN propagates.
// * exp2_b31: the exponent is the low word of y + 1.5 * 2^52, which holds n
//   in two's complement while |n| < 2^31, without a conversion.  Callers
//   keep |y| below 2^30: the Arrhenius factors do through the bound on 1/T
//   that the host derives from the mechanism's largest log2 A, |beta| and
//   theta' (|log2 T| <= 1075 for any positive double).
struct ExpK {
    double shift, ln2, c[10];
};

__host__ __device__ constexpr ExpK exp_k() {
    return ExpK{0x1.8p52, 0.6931471805599453,
                {4.45410341058704e-10, 7.070977866508138e-09, 1.0178067267449427e-07,
                 1.3215451633221434e-06, 1.5252733820795803e-05, 0.00015403530424776529,
                 0.0013333558146423213, 0.009618129107618665, 0.05550410866482158,
                 0.24022650695910075}};
}

// n (an integral double) to int32, saturating at the int32 range (the
// hardware conversion clamps; NaN gives 0).
__device__ __forceinline__ int cvt_sat_i32(double n) {
    int i;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(i) : "v"(n));
    return i;
}

__device__ __forceinline__ double exp2_frac(double f, const ExpK &k) {
    double q = k.c[0];
#pragma unroll
    for (int i = 1; i < 10; ++i) q = __builtin_fma(q, f, k.c[i]);
    q = __builtin_fma(q, f, k.ln2);
    return __builtin_fma(q, f, 1.0);
}

__device__ __forceinline__ double exp2_sat(double y, const ExpK &k) {
    const double t = y + k.shift;
    const double n = t - k.shift;
    return __builtin_ldexp(exp2_frac(y - n, k), cvt_sat_i32(n));
}

__device__ __forceinline__ double exp2_b31(double y, const ExpK &k) {
    const double t = y + k.shift;
    const double n = t - k.shift;
    return __builtin_ldexp(exp2_frac(y - n, k), (int)(uint32_t)__double_as_longlong(t));
}

__device__ __forceinline__ double exp2_sat(double y) { return exp2_sat(y, exp_k()); }

// The same constants as values the compiler cannot see through, so that they
// are materialised where a source-term evaluation starts and do not occupy
// registers across the integrator's bookkeeping.  All are scalar but the
// second polynomial coefficient, which meets the first in one FMA
// (c0 f + c1): an instruction reads at most one scalar register.
__device__ __forceinline__ double opaque_sd(double v) {
    asm volatile("" : "+s"(v));
    return v;
}

__device__ __forceinline__ double opaque_vd(double v) {
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ ExpK exp_k_local() {
    constexpr ExpK c = exp_k();
    ExpK k;
    k.shift = opaque_sd(c.shift);
    k.ln2 = opaque_sd(c.ln2);
#pragma unroll
    for (int i = 0; i < 10; ++i) k.c[i] = (i == 1) ? opaque_vd(c.c[i]) : opaque_sd(c.c[i]);
    return k;
}

constexpr double LOG2E = 1.44269504088896340736;     // log2(e)

// Base-2 logarithm of a positive finite double (NaN otherwise).  With
// x = m 2^e, m in [1/2, 1), the hardware single-precision log2 m (relative
// error ~1e-7) is the estimate l0, corrected exactly: d = m 2^(-l0) - 1 is
// tiny (|d| < 1e-6), log2 m = l0 + ln(1 + d) log2(e), and the series
// d - d^2/2 + d^3/3 of ln(1 + d) leaves a truncation below d^4/4.  The error
// is that of the exponential (about 1e-16 absolute) plus the final rounding.
// No division and no polynomial table beyond the exponential's.
__device__ __forceinline__ double log2_pos(double x, const ExpK &k) {
    int e;
    const double m = frexp(x, &e);
    const double l0 = (double)__builtin_amdgcn_logf((float)m);
    const double d = __builtin_fma(m, exp2_b31(-l0, k), -1.0);
    const double l1 = d * __builtin_fma(d, __builtin_fma(d, 1.0 / 3.0, -0.5), 1.0);
    const double r = (double)e + __builtin_fma(l1, LOG2E, l0);
    return (x > 0.0 && x <= 0x1.fffffffffffffp+1023) ? r : __builtin_nan("");
}

__device__ __forceinline__ double log2_pos(double x) { return log2_pos(x, exp_k()); }

// x^(-1/6) for a positive finite x.  With x = m 2^e and e = 6q + t,
// t in 0..5: x^(-1/6) = a^(-1/6) 2^(-q), a = m 2^t in [1/2, 32).  A
// single-precision seed of a^(-1/6) (hardware log2 and exp2) is refined by two
// Newton steps for y^-6 = a, y <- y (7 - a y^6)/6, which take the relative
// error e to about 3.5 e^2 each (2e-7 -> 2e-13 -> below rounding).  Within a
// few ulps.
__device__ __forceinline__ double rsixth_pos(double x) {
    int e;
    const double m = frexp(x, &e);
    const int q = (e >= 0) ? e / 6 : -((5 - e) / 6);
    const double a = __builtin_ldexp(m, e - 6 * q);
    double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)a) * (-1.0f / 6.0f));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double y3 = y * y * y;
        y = y * __builtin_fma(-a, y3 * y3, 7.0) * (1.0 / 6.0);
    }
    return __builtin_ldexp(y, -q);
}

// 1/x for a positive normal x: hardware reciprocal refined by two Newton
// steps (each doubles the correct bits; the result is within an ulp).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// A zero the compiler cannot see through.  Adding it to loop-invariant table
// indices keeps the (cheap) address arithmetic inside the integration loop
// instead of pinning one register per address for the lifetime of the wave.
__device__ __forceinline__ uint32_t opaque_zero() {
    uint32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

constexpr double LOG10_2 = 0.30102999566398119521;    // log10(2)
constexpr double LOG2_10 = 3.32192809488736234787;    // log2(10)

// Falloff rate k_inf Pr/(1 + Pr) F with Pr = k_0 [M] / k_inf (Chemkin form);
// F = 1 (Lindemann) or the Troe factor with log10 F = lFc / (1 + f^2),
// f = (log10 Pr + c) / (n - 0.14 (log10 Pr + c)), c = -0.4 - 0.67 lFc,
// n = 0.75 - 1.27 lFc, lFc = log10 F_cent.  Zero if k_inf or k_0 [M] is 0.
__device__ __forceinline__ double falloff_rate(double kinf, double k0M, double lFc, bool troe,
                                               const ExpK &K) {
    if (!(kinf > 0.0) || !(k0M > 0.0)) return 0.0;
    const double Pr = k0M / kinf;
    double F = 1.0;
    if (troe) {
        const double x = log2_pos(Pr, K) * LOG10_2 + (-0.4 - 0.67 * lFc);
        const double f = x / ((0.75 - 1.27 * lFc) - 0.14 * x);
        F = exp2_sat(lFc / (1.0 + f * f) * LOG2_10, K);
    }
    return kinf * (Pr / (1.0 + Pr)) * F;
}

// One lane's gather segments of SL terms each (SL even): all of a segment's
// words and rates are loaded before they are summed (in term order, the same
// sum as a running accumulator), so the loads overlap instead of each waiting
// for the previous add.
template <int G, int SL>
__device__ __forceinline__ void gather_segments(const uint32_t *tw, const unsigned char *Qb,
                                                double *__restrict__ piece, int NSEG, int go) {
    constexpr int H = SL / 2;
    for (int sg = 0; sg < NSEG; ++sg) {
        uint32_t w[H];
#pragma unroll
        for (int e = 0; e < H; ++e) w[e] = tw[(sg * H + e) * G];
        double v[SL];
#pragma unroll
        for (int e = 0; e < H; ++e) {
            v[2 * e] = *reinterpret_cast<const double *>(Qb + (w[e] & 0xffffu));
            v[2 * e + 1] = *reinterpret_cast<const double *>(Qb + (w[e] >> 16));
        }
        double acc = v[0];
#pragma unroll
        for (int e = 1; e < SL; ++e) acc += v[e];
        piece[sg * G + go] = acc;
    }
}

// Sum of N2 (even) terms of one lane: 16-bit byte offsets into base, two per
// word at tw[e * G]; all loads are issued before the adds (in term order).
template <int G, int N2>
__device__ __forceinline__ double sum_terms(const uint32_t *tw, const unsigned char *base) {
    constexpr int H = N2 / 2;
    uint32_t w[H];
#pragma unroll
    for (int e = 0; e < H; ++e) w[e] = tw[e * G];
    double v[N2];
#pragma unroll
    for (int e = 0; e < H; ++e) {
        v[2 * e] = *reinterpret_cast<const double *>(base + (w[e] & 0xffffu));
        v[2 * e + 1] = *reinterpret_cast<const double *>(base + (w[e] >> 16));
    }
    double acc = v[0];
#pragma unroll
    for (int e = 1; e < N2; ++e) acc += v[e];
    return acc;
}

// Second gather level: the net production of each of the lane's state slots,
// its LP positive pieces minus its LN negative ones.
template <int G, int NSL, int LP, int LN>
__device__ __forceinline__ void piece_sums(const uint32_t *tw2, const unsigned char *Pb,
                                           double (&w)[NSL]) {
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const uint32_t *t = tw2 + (size_t)s * ((LP + LN) / 2) * G;
        w[s] = sum_terms<G, LP>(t, Pb) - sum_terms<G, LN>(t + (LP / 2) * G, Pb);
    }
}

// The same for piece counts without an unrolled instance.
template <int G, int NSL>
__device__ __forceinline__ void piece_sums_any(const uint32_t *tw2, const unsigned char *Pb,
                                               int LP, int LN, double (&w)[NSL]) {
    const int H = (LP + LN) / 2;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const uint32_t *t = tw2 + (size_t)s * H * G;
        double wp = 0.0, wn = 0.0;
        for (int e = 0; e < LP / 2; ++e) {
            const uint32_t x = t[e * G];
            wp += *reinterpret_cast<const double *>(Pb + (x & 0xffffu));
            wp += *reinterpret_cast<const double *>(Pb + (x >> 16));
        }
        for (int e = LP / 2; e < H; ++e) {
            const uint32_t x = t[e * G];
            wn += *reinterpret_cast<const double *>(Pb + (x & 0xffffu));
            wn += *reinterpret_cast<const double *>(Pb + (x >> 16));
        }
        w[s] = wp - wn;
    }
}

// Source term of E:mass and E:energy for the group's cell at state z.
// z/fz hold this lane's NSL elements (index k = s * G + g).
template <int G, int NSL, int RUC, bool PD>
__device__ __forceinline__ void rhs_eval(const double (&z)[NSL], double P10, double invP10,
                                         double (&fz)[NSL], const GroupLds &L,
                                         const UnitRegs<RUC> &ur, int g, int N, int RU, int NSEG,
                                         int SEGL, int L2P, int L2N, int RUp, int NMS,
                                         int RU2, double invTmax) {
    constexpr int NK = NSL * G;
    const uint32_t oz = opaque_zero();
    const int go = g + (int)oz;
    const ExpK K = exp_k_local();
    const double T = gbcast0<G>(z[0]);
    const double invT = rcp_nr(T);
    const double l2T = log2_pos(T, K);
    const double invTa = fmin(invT, invTmax);   // 1/T of the Arrhenius factors

    double sYW = 0.0, sYcp = 0.0;
    double hRT[NSL], invW[NSL];
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + go;
        const double Y = (k == 0) ? 0.0 : z[s];
        invW[s] = L.spec[F_INVW * NK + k];
        const bool hi = T >= L.tmid[k];
        const double *a = L.spec + (hi ? F_CPHI : F_CPLO) * NK + k;
        const double *b = L.spec + (hi ? F_HHI : F_HLO) * NK + k;
        const double cpR = a[0] + T * (a[NK] + T * (a[2 * NK] + T * (a[3 * NK] + T * a[4 * NK])));
        hRT[s] = b[0] + T * (b[NK] + T * (b[2 * NK] + T * (b[3 * NK] + T * b[4 * NK])))
               + b[5 * NK] * invT;
        const double YW = Y * invW[s];
        sYW += YW;
        sYcp += YW * cpR;
    }
    gsum2<G>(sYW, sYcp);
    const double RTW = R_ERG * T * sYW;
    const double rho = P10 * rcp_nr(RTW);  // ideal gas, g/cm^3
    const double inv_rho = RTW * invP10;

    // The C, Q and piece arrays never overlap; telling the compiler so lets it
    // issue the loads of one unit or segment before the stores of the last.
    double *__restrict__ C = L.C;
    double *__restrict__ Q = L.Q;
    double *__restrict__ piece = L.piece;

    wave_sync();   // previous evaluation's readers of C are done
    double Ck[NSL];
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + go;
        Ck[s] = (k >= 1 && k < N) ? rho * z[s] * invW[s] : 0.0;
        if (k >= 1 && k < N) C[k - 1] = Ck[s];
    }
    // third-body concentration of each efficiency set, [M] = sum_i alpha_i C_i
    if constexpr (PD)
    for (int q = 0; q < NMS; q += 2) {
        double p0 = 0.0, p1 = 0.0;
        const bool two = q + 1 < NMS;
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
            p0 += L.eff[q * NK + s * G + go] * Ck[s];
            if (two) p1 += L.eff[(q + 1) * NK + s * G + go] * Ck[s];
        }
        if (two) {
            gsum2<G>(p0, p1);
        } else {
            p0 = gsum<G>(p0);
        }
        if (g == 0) {
            L.Mv[q] = p0;
            if (two) L.Mv[q + 1] = p1;
        }
    }
    wave_sync();

    // Rates of progress (E:rxn-rate) with Arrhenius coefficients (E:rxn-const),
    // net of each forward/reverse pair.
    if constexpr (RUC > 0) {
        double q[RUC];
#pragma unroll
        for (int r = 0; r < RUC; ++r) {
            const double kf = exp2_b31(arrhenius_arg(ur.l2Af[r], ur.bf[r], ur.tf[r], l2T, invTa), K);
            const double kr = exp2_b31(arrhenius_arg(ur.l2Ar[r], ur.br[r], ur.tr[r], l2T, invTa), K);
            const uint32_t a = ur.idf[r] + oz, b = ur.idr[r] + oz;
            // the same operations in the same order as the LDS path below, so
            // the placement of the parameters never changes a result
            const double cf = unpack_c(C, a, 0) * unpack_c(C, a, 1) * unpack_c(C, a, 2);
            const double cr = unpack_c(C, b, 0) * unpack_c(C, b, 1) * unpack_c(C, b, 2);
            q[r] = net_rate(kf, cf, kr, cr);
        }
#pragma unroll
        for (int r = 0; r < RUC; ++r) Q[r * G + go] = q[r];
    } else {
        // LDS copy is lane-interleaved: 16-byte piece q of unit r * G + g at
        // double2 index (4 r + q) G + g, so a wave's reads are contiguous.  The
        // reactant slots (piece 3) of the next unit are loaded one iteration
        // ahead; the load after the last unit reads the group arrays that
        // follow the table in LDS and is not used.
        const double2 *ub = reinterpret_cast<const double2 *>(L.units) + g;
        const unsigned char *Cb = reinterpret_cast<const unsigned char *>(C);
        auto cat = [&](uint64_t o, int sl) {
            return *reinterpret_cast<const double *>(Cb + ((o >> (16 * sl)) & 0xffffu));
        };
        // one unit from its slots u3 (loaded one unit ahead); returns the next
        // unit's slots.  Reactant slots first: the concentration products load
        // and multiply while the two exponentials are computed.  In rounds
        // [0, RU2) no side has a third reactant, whose slot names the 1.0
        // entry, so the third factor is left out (multiplying by 1.0 is
        // exact: the products are the same).
        auto unit = [&](int r, const double2 u3, auto three) {
            const double2 *u = ub + (size_t)(4 * r) * G;
            const double2 u0 = u[0], u1 = u[G], u2 = u[2 * G];
            const double2 u3n = u[7 * G];
            const uint64_t a = __double_as_longlong(u3.x), b = __double_as_longlong(u3.y);
            double cf = cat(a, 0) * cat(a, 1);
            double cr = cat(b, 0) * cat(b, 1);
            if constexpr (decltype(three)::value) {
                cf *= cat(a, 2);
                cr *= cat(b, 2);
            }
            const double kf = exp2_b31(arrhenius_arg(u0.x, u0.y, u1.x, l2T, invTa), K);
            const double kr = exp2_b31(arrhenius_arg(u1.y, u2.x, u2.y, l2T, invTa), K);
            Q[r * G + g] = net_rate(kf, cf, kr, cr);
            return u3n;
        };
        const std::integral_constant<bool, false> two_slots;
        const std::integral_constant<bool, true> three_slots;
        const int r_fast = PD ? RUp : RU;
        if constexpr (RUC < 0) {
            // records in global memory: the whole record of the next unit is
            // loaded before this unit is computed, so the cache latency runs
            // under a unit's arithmetic (the table ends with a zero round)
            struct Rec {
                double2 a, b, c, d;
            };
            auto load = [&](int r) {
                const double2 *u = ub + (size_t)(4 * r) * G;
                return Rec{u[0], u[G], u[2 * G], u[3 * G]};
            };
            auto unitg = [&](int r, const Rec cur, auto three) {
                const Rec nxt = load(r + 1);
                const uint64_t a = __double_as_longlong(cur.d.x), b = __double_as_longlong(cur.d.y);
                double cf = cat(a, 0) * cat(a, 1);
                double cr = cat(b, 0) * cat(b, 1);
                if constexpr (decltype(three)::value) {
                    cf *= cat(a, 2);
                    cr *= cat(b, 2);
                }
                const double kf = exp2_b31(arrhenius_arg(cur.a.x, cur.a.y, cur.b.x, l2T, invTa), K);
                const double kr = exp2_b31(arrhenius_arg(cur.b.y, cur.c.x, cur.c.y, l2T, invTa), K);
                Q[r * G + g] = net_rate(kf, cf, kr, cr);
                return nxt;
            };
            Rec ra = load(0);
            int r = 0;
            for (; r + 1 < RU2; r += 2) {
                const Rec rb = unitg(r, ra, two_slots);
                ra = unitg(r + 1, rb, two_slots);
            }
            if (r < RU2) ra = unitg(r++, ra, two_slots);
            for (; r + 1 < r_fast; r += 2) {
                const Rec rb = unitg(r, ra, three_slots);
                ra = unitg(r + 1, rb, three_slots);
            }
            if (r < r_fast) (void)unitg(r, ra, three_slots);
        } else {
        // two units per iteration, so that the prefetched slots alternate
        // between two registers instead of being copied every unit
        double2 u3a = ub[3 * G];
        int r = 0;
        for (; r + 1 < RU2; r += 2) {
            const double2 u3b = unit(r, u3a, two_slots);
            u3a = unit(r + 1, u3b, two_slots);
        }
        if (r < RU2) u3a = unit(r++, u3a, two_slots);
        for (; r + 1 < r_fast; r += 2) {
            const double2 u3b = unit(r, u3a, three_slots);
            u3a = unit(r + 1, u3b, three_slots);
        }
        if (r < r_fast) (void)unit(r, u3a, three_slots);
        }
        // rounds with pressure-dependent units: third body and falloff (only
        // in the kernels built for mechanisms that have them)
        if constexpr (PD)
        for (int rp = RUp; rp < RU; ++rp) {
            const int p = rp * G + g;
            const double2 *u = ub + (size_t)(4 * rp) * G;
            const double2 u0 = u[0], u1 = u[G], u2 = u[2 * G], u3 = u[3 * G];
            const uint64_t a = __double_as_longlong(u3.x), b = __double_as_longlong(u3.y);
            const double cf = cat(a, 0) * cat(a, 1) * cat(a, 2);
            const double cr = cat(b, 0) * cat(b, 1) * cat(b, 2);
            double kf = exp2_b31(arrhenius_arg(u0.x, u0.y, u1.x, l2T, invTa), K);
            double kr = exp2_b31(arrhenius_arg(u1.y, u2.x, u2.y, l2T, invTa), K);
            const double2 *pd = reinterpret_cast<const double2 *>(L.pdep) +
                                (size_t)(6 * (rp - RUp)) * G + g;
            const double2 d0 = pd[0];
            const uint64_t tag = __double_as_longlong(d0.x);
            const int kind = (int)(tag & 0xffu);
            if (kind != 0) {
                const double M = L.Mv[(tag >> 8) & 0xffu];
                if (kind == 1) {
                    kf *= M;
                    kr *= M;
                } else {
                    const double2 d1 = pd[G], d2 = pd[2 * G], d3 = pd[3 * G];
                    const double k0f = exp2_b31(arrhenius_arg(d0.y, d1.x, d1.y, l2T, invTa), K);
                    const double k0r = exp2_b31(arrhenius_arg(d2.x, d2.y, d3.x, l2T, invTa), K);
                    double lFc = 0.0;   // log10 of the Troe centre value (Lindemann: F = 1)
                    if (kind == 3) {
                        const double2 d4 = pd[4 * G], d5 = pd[5 * G];
                        // exp(-T/T***), exp(-T/T*), exp(-T**/T) in base 2
                        // (the host stores log2(e)/T***, log2(e)/T*, T** log2(e))
                        const double Fc = (1.0 - d4.x) * exp2_sat(-T * d4.y, K) +
                                          d4.x * exp2_sat(-T * d5.x, K) +
                                          (d5.y > 0.0 ? exp2_sat(-d5.y * invT, K) : 0.0);
                        lFc = log2_pos(Fc, K) * LOG10_2;
                    }
                    kf = falloff_rate(kf, k0f * M, lFc, kind == 3, K);
                    kr = falloff_rate(kr, k0r * M, lFc, kind == 3, K);
                }
            }
            Q[p] = net_rate(kf, cf, kr, cr);
        }
    }
    wave_sync();

    // Net production (E:spec-rate), species equations (E:mass) and the
    // enthalpy sum of the energy equation (E:energy).
    {
        const unsigned char *Qb = reinterpret_cast<const unsigned char *>(Q);
        const uint32_t *tw = L.gather + go;
        switch (SEGL) {   // uniform; the common segment lengths are unrolled
        case 2: gather_segments<G, 2>(tw, Qb, piece, NSEG, go); break;
        case 4: gather_segments<G, 4>(tw, Qb, piece, NSEG, go); break;
        case 6: gather_segments<G, 6>(tw, Qb, piece, NSEG, go); break;
        case 8: gather_segments<G, 8>(tw, Qb, piece, NSEG, go); break;
        case 10: gather_segments<G, 10>(tw, Qb, piece, NSEG, go); break;
        case 12: gather_segments<G, 12>(tw, Qb, piece, NSEG, go); break;
        default: {
            const int half = SEGL >> 1;
            for (int sg = 0; sg < NSEG; ++sg) {
                double acc = 0.0;
#pragma unroll 4
                for (int e2 = 0; e2 < half; ++e2) {
                    const uint32_t w = tw[(sg * half + e2) * G];
                    acc += *reinterpret_cast<const double *>(Qb + (w & 0xffffu));
                    acc += *reinterpret_cast<const double *>(Qb + (w >> 16));
                }
                piece[sg * G + go] = acc;
            }
        }
        }
    }
    wave_sync();
    double w[NSL];
    {
        const unsigned char *Pb = reinterpret_cast<const unsigned char *>(piece);
        const uint32_t *tw2 = L.gather2 + go;
        switch (L2P * 16 + L2N) {   // uniform; the common piece counts are unrolled
#define RKC_PIECES(LP, LN) \
        case LP * 16 + LN: piece_sums<G, NSL, LP, LN>(tw2, Pb, w); break;
        RKC_PIECES(2, 2) RKC_PIECES(2, 4) RKC_PIECES(2, 6) RKC_PIECES(2, 8)
        RKC_PIECES(4, 2) RKC_PIECES(4, 4) RKC_PIECES(4, 6) RKC_PIECES(4, 8)
        RKC_PIECES(6, 2) RKC_PIECES(6, 4) RKC_PIECES(6, 6) RKC_PIECES(6, 8)
        RKC_PIECES(8, 2) RKC_PIECES(8, 4) RKC_PIECES(8, 6) RKC_PIECES(8, 8)
#undef RKC_PIECES
        default: piece_sums_any<G, NSL>(tw2, Pb, L2P, L2N, w);
        }
    }
    double hs = 0.0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + go;
        fz[s] = L.spec[F_W * NK + k] * w[s] * inv_rho;
        hs += hRT[s] * w[s];
    }
    hs = gsum<G>(hs);
    // dT/dt = -sum_i H_i omega_i / (rho cp); R cancels between H and cp.
    const double fT = -T * hs * inv_rho * rcp_nr(sYcp);
    if (g == 0) fz[0] = fT;
}

// ---------------------------------------------------------------- staging

template <int RUC>
__device__ __forceinline__ void load_unit_regs(const Params &p, UnitRegs<RUC> &ur, int g, int G) {
    if constexpr (RUC > 0) {
#pragma unroll
        for (int r = 0; r < RUC; ++r) {
            const double *u = p.tab.units + (size_t)(r * G + g) * UNIT_DOUBLES;
            ur.l2Af[r] = u[0]; ur.bf[r] = u[1]; ur.tf[r] = u[2];
            ur.l2Ar[r] = u[3]; ur.br[r] = u[4]; ur.tr[r] = u[5];
            // 16-bit byte offsets -> three 10-bit indices
            const uint64_t bf = __double_as_longlong(u[6]), br = __double_as_longlong(u[7]);
            uint32_t f = 0, v = 0;
            for (int sl = 0; sl < 3; ++sl) {
                f |= (uint32_t)(((bf >> (16 * sl)) & 0xffffu) >> 3) << (10 * sl);
                v |= (uint32_t)(((br >> (16 * sl)) & 0xffffu) >> 3) << (10 * sl);
            }
            ur.idf[r] = f;
            ur.idr[r] = v;
        }
    }
}

// Bytes of per-group control state kept in LDS by the integrator kernels.
constexpr int STATE_BYTES = 320;

// Sizes that fix the LDS layout of a workgroup.
struct Shape {
    int NK, RU, G, NSEG, SEGL, L2, NPR, NMS;   // L2 = L2P + L2N
    bool units_in_lds, spec_in_lds;
};

// Where a kernel variant keeps the reaction parameters: RUC > 0 registers,
// RUC = 0 LDS, RUC = -1 global memory (read through the caches, with the
// species table, so that large mechanisms leave LDS to more lane groups).
__device__ __forceinline__ Shape shape_of(const Params &p, int G, int RUC) {
    return Shape{p.NK, p.RU, G, p.NSEG, p.SEGL, p.L2P + p.L2N, p.NPR, p.NMS, RUC == 0, RUC >= 0};
}

// Doubles of per-group LDS: concentrations, net rates (+ zero slot, padded to
// even), gather pieces (+ zero slot, padded to even), third-body
// concentrations of the efficiency sets (padded to even).
__host__ __device__ inline size_t group_doubles(const Shape &s) {
    return (size_t)s.NK + (size_t)s.RU * s.G + 2 + (size_t)s.NSEG * s.G + 2 +
           (size_t)((s.NMS + 1) & ~1);
}

// Bytes of dynamic LDS for a workgroup of `groups` groups.  With the species
// table in global memory its T_mid row is still staged, so that choosing a
// NASA range does not wait for a global load before the coefficient loads.
__host__ __device__ inline size_t lds_bytes(const Shape &s, int groups) {
    size_t b = (size_t)(s.spec_in_lds ? NFIELD : 1) * s.NK * 8;
    if (s.units_in_lds) b += (size_t)s.RU * s.G * UNIT_DOUBLES * 8;
    b += (size_t)s.NPR * s.G * PDEP_DOUBLES * 8;
    b += (size_t)s.NMS * s.NK * 8;
    b += (size_t)groups * group_doubles(s) * 8;
    b += (size_t)groups * STATE_BYTES;
    b += (size_t)s.NSEG * (s.SEGL / 2) * s.G * 4 + (size_t)s.NK * (s.L2 / 2) * 4;
    return b;
}

struct LdsPtrs {
    double *spec, *units, *pdep, *eff;
    uint32_t *gather, *gather2;
    double *groups;
    unsigned char *states;
};

__device__ __forceinline__ LdsPtrs carve(unsigned char *base, const Shape &s, int groups) {
    LdsPtrs l;
    size_t off = 0;
    l.spec = reinterpret_cast<double *>(base + off);
    off += (size_t)(s.spec_in_lds ? NFIELD : 1) * s.NK * 8;
    l.units = reinterpret_cast<double *>(base + off);
    if (s.units_in_lds) off += (size_t)s.RU * s.G * UNIT_DOUBLES * 8;
    l.pdep = reinterpret_cast<double *>(base + off); off += (size_t)s.NPR * s.G * PDEP_DOUBLES * 8;
    l.eff = reinterpret_cast<double *>(base + off); off += (size_t)s.NMS * s.NK * 8;
    l.groups = reinterpret_cast<double *>(base + off);
    off += (size_t)groups * group_doubles(s) * 8;
    l.states = base + off;
    off += (size_t)groups * STATE_BYTES;
    l.gather = reinterpret_cast<uint32_t *>(base + off); off += (size_t)s.NSEG * (s.SEGL / 2) * s.G * 4;
    l.gather2 = reinterpret_cast<uint32_t *>(base + off);
    return l;
}

// Per-group LDS views and their one-time initialisation (absent-slot
// concentration 1.0, the zero slot of the signed rates).
__device__ __forceinline__ GroupLds group_view(const LdsPtrs &lp, const Shape &s, int gib) {
    GroupLds L;
    L.spec = lp.spec; L.gather = lp.gather; L.gather2 = lp.gather2;
    L.tmid = s.spec_in_lds ? lp.spec + F_TMID * s.NK : lp.spec;
    L.units = lp.units;
    L.pdep = lp.pdep;
    L.eff = lp.eff;
    L.C = lp.groups + (size_t)gib * group_doubles(s);
    L.Q = L.C + s.NK;
    L.piece = L.Q + s.RU * s.G + 2;
    L.Mv = L.piece + s.NSEG * s.G + 2;
    return L;
}

__device__ __forceinline__ void stage_tables(const Params &p, int G, const LdsPtrs &lp,
                                             int n_units_l, bool spec_l) {
    double *spec_lp = lp.spec, *units_l = lp.units;
    uint32_t *gather_l = lp.gather;
    const int tid = threadIdx.x, nt = blockDim.x;
    // pressure-dependent records (already interleaved) and efficiency sets
    for (int i = tid; i < p.NPR * G * PDEP_DOUBLES; i += nt) lp.pdep[i] = p.tab.pdep[i];
    for (int i = tid; i < p.NMS * p.NK; i += nt) lp.eff[i] = p.tab.eff[i];
    if (spec_l)
        for (int i = tid; i < NFIELD * p.NK; i += nt) spec_lp[i] = p.tab.spec[i];
    else
        for (int i = tid; i < p.NK; i += nt) spec_lp[i] = p.tab.spec[F_TMID * p.NK + i];
    for (int i = tid; i < p.NSEG * (p.SEGL / 2) * G; i += nt) gather_l[i] = p.tab.gather[i];
    for (int i = tid; i < p.NK * ((p.L2P + p.L2N) / 2); i += nt) lp.gather2[i] = p.tab.gather2[i];
    // unit records, lane-interleaved in 16-byte pieces (see rhs_eval)
    const double2 *ug = reinterpret_cast<const double2 *>(p.tab.units);
    double2 *ul = reinterpret_cast<double2 *>(units_l);
    for (int i = tid; i < n_units_l * (UNIT_DOUBLES / 2); i += nt) {
        const int unit = i / (UNIT_DOUBLES / 2), q = i % (UNIT_DOUBLES / 2);
        ul[((unit / G) * (UNIT_DOUBLES / 2) + q) * G + unit % G] = ug[i];
    }
}

// The RUC = -1 kernels read the species table and the lane-interleaved unit
// records from global memory.
__device__ __forceinline__ void global_tables(GroupLds &L, const Params &p) {
    L.spec = p.tab.spec;
    L.units = p.tab.units_il;
}

__device__ __forceinline__ void group_init(const GroupLds &L, const Params &p, int G, int g) {
    for (int k = g; k < p.NK; k += G) L.C[k] = (k == p.nS) ? 1.0 : 0.0;
    if (g == 0) {
        L.Q[p.RU * G] = 0.0; L.Q[p.RU * G + 1] = 0.0;
        L.piece[p.NSEG * G] = 0.0; L.piece[p.NSEG * G + 1] = 0.0;
    }
}

// ------------------------------------------------------- source-term kernel

// Occupancy targets (waves per SIMD; a workgroup holds one wave per SIMD per
// target wave): register-resident reaction parameters, or four state slots
// per lane, need the register file of two waves; two slots fit three waves
// (168 VGPRs) and one slot fits four (128 VGPRs), all without spilling.
template <int RUC, int NSL>
struct Occ {
    static constexpr int waves = (RUC > 0 || NSL > 2) ? 2 : (NSL == 2 ? 3 : 4);
    static constexpr int threads = waves * 256;
};

template <int G, int NSL, int RUC, bool PD>
__global__ __launch_bounds__((Occ<RUC, NSL>::threads), (Occ<RUC, NSL>::waves)) void rhs_kernel(Params p) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int groups = blockDim.x / G;
    const int gib = threadIdx.x / G;
    const int g = threadIdx.x % G;
    const Shape sh = shape_of(p, G, RUC);
    LdsPtrs lp = carve(lds_raw, sh, groups);
    stage_tables(p, G, lp, RUC == 0 ? p.RU * G : 0, RUC >= 0);
    GroupLds L = group_view(lp, sh, gib);
    if constexpr (RUC < 0) global_tables(L, p);
    group_init(L, p, G, g);
    __syncthreads();
    UnitRegs<RUC> ur;
    load_unit_regs<RUC>(p, ur, g, G);

    const int cell = blockIdx.x * groups + gib;
    const bool active = cell < p.n_cells;
    double z[NSL], fz[NSL];
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        double v = 0.0;
        if (active) {
            if (k == 0) v = p.T[cell];
            else if (k < p.N) v = p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss];
        }
        z[s] = v;
    }
    if (!active) z[0] = (g == 0) ? 1000.0 : z[0];
    const double P10 = active ? p.P[cell] * 10.0 : 1e6;
    rhs_eval<G, NSL, RUC, PD>(z, P10, 1.0 / P10, fz, L, ur, g, p.N, p.RU, p.NSEG, p.SEGL, p.L2P,
                              p.L2N, p.RUp, p.NMS, p.RU2, p.invTmax);
    if (active) {
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
            const int k = s * G + g;
            if (k < p.N) p.F[(long long)cell * p.fcs + (long long)k * p.fss] = fz[s];
        }
    }
}

}  // namespace rkcdev
