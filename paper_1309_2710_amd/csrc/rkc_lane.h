// One lane per cell: device code for small mechanisms (Sec. 3 runs one
// thread per ODE).
//
// Every lane of a wavefront integrates its own cell, and all 64 cells share
// the mechanism, so everything that describes the mechanism is wave-uniform:
// reaction parameters, reactant species, the species records and the terms of
// the net production sum are read with scalar loads (constant address space)
// into scalar registers, and the loops over reactions and species are scalar
// loops with no divergence at all.  Per-lane data whose index comes from the
// mechanism (concentrations and net production rates by species) sit in LDS
// rows of 64 doubles, one double per lane, so a row access is one
// conflict-free ds_read_b64 whose address is the lane's base plus a uniform
// row offset; no lane ever reads another lane's column, so the rows need no
// barriers.  The state vectors of the integrator stay in VGPRs (NMAX elements
// per vector, NMAX >= N = n_species + 1).
//
// The integrator is the same state machine as the lane-group kernels: every
// iteration of the main loop performs exactly one source-term evaluation in
// every lane, whatever phase the lane's cell is in; a lane that finishes takes
// the next cell from the work queue (wave-aggregated claims), so lanes refill
// independently and the wave keeps all 64 lanes busy until the queue drains.
// Every scalar of the method (norms, mixture sums) is a plain sum over the
// lane's own elements in index order.
#pragma once

#include "rkc_integrate.h"

namespace rkcdev {

constexpr int LROW = 64 * 8;   // bytes of one LDS row: a double per lane of a wave

// Species record of the lane kernels (LS_FIELDS doubles per species, so one
// species is a few scalar loads): W, 1/W, T_mid, then the Cp/R and H/(RT)
// Horner coefficients of the low and the high range (same values as the
// F_* fields of the lane-group table).
enum {
    LS_W = 0, LS_INVW = 1, LS_TMID = 2, LS_CPLO = 3, LS_HLO = 8, LS_CPHI = 14, LS_HHI = 19,
    LS_FIELDS = 32
};

typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) uint32_t cuint;

__device__ __forceinline__ cdouble *cptr(const double *p) { return (cdouble *)p; }
__device__ __forceinline__ cuint *cptr(const uint32_t *p) { return (cuint *)p; }

// Row access: lane base (VGPR) plus a row byte offset (uniform).
__device__ __forceinline__ double &lrow_at(unsigned char *base, uint32_t off) {
    return *reinterpret_cast<double *>(base + off);
}

// Horner forms of Cp/R and H/(RT) from a species record (uniform pointer a or
// b at the first coefficient of one range); the same expressions as the
// lane-group kernels.
__device__ __forceinline__ double cp_horner(cdouble *a, double T) {
    return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}
__device__ __forceinline__ double h_horner(cdouble *b, double T, double invT) {
    return b[0] + T * (b[1] + T * (b[2] + T * (b[3] + T * b[4]))) + b[5] * invT;
}

// LDS rows of one wave (each LROW bytes: a double per lane):
//   [0, nS)            concentrations C_k
//   nS                 1.0 (the empty reactant slot)
//   [nS + 1, 2 nS + 1) net production rates omega_k
//   2 nS + 1           discard row (target of a unit's unused term slots)
//   [2 nS + 2, ...)    third-body concentrations of the efficiency sets
__host__ __device__ inline int lane_row_one(int nS) { return nS; }
__host__ __device__ inline int lane_row_omega(int nS) { return nS + 1; }
__host__ __device__ inline int lane_row_discard(int nS) { return 2 * nS + 1; }
__host__ __device__ inline int lane_row_mset(int nS) { return 2 * nS + 2; }

// Unit record of the lane kernels: LU_DOUBLES doubles (two 64-byte scalar
// loads).
//   [0..7]   as the lane-group unit record (log2 A, beta, theta' forward and
//            reverse; forward and reverse reactant slots as 16-bit byte
//            offsets k * 8, the empty slot at n_species * 8, i.e. the row
//            of ones)
//   [8], [9] the LDS rows of the unit's net-production terms, six 16-bit
//            row indices (terms 0-3 in [8], 4-5 in [9]); unused slots name
//            the discard row
//   [10..15] nu'' - nu' of terms 0..5 (0 for unused slots)
constexpr int LU_DOUBLES = 16;
constexpr int LU_TERMS = 6;

// A unit record in scalar registers.
struct LaneUnit {
    double l2Af, bf, tf, l2Ar, br, tr;
    uint64_t sf, sr, t03, t45;
    double dnu[LU_TERMS];
};

__device__ __forceinline__ LaneUnit lane_unit(cdouble *r) {
    LaneUnit u;
    u.l2Af = r[0]; u.bf = r[1]; u.tf = r[2]; u.l2Ar = r[3]; u.br = r[4]; u.tr = r[5];
    u.sf = __double_as_longlong(r[6]);
    u.sr = __double_as_longlong(r[7]);
    u.t03 = __double_as_longlong(r[8]);
    u.t45 = __double_as_longlong(r[9]);
#pragma unroll
    for (int t = 0; t < LU_TERMS; ++t) u.dnu[t] = r[10 + t];
    return u;
}

__device__ __forceinline__ uint32_t slot_off(uint64_t slots, int s) {
    return (uint32_t)((slots >> (16 * s)) & 0xffffu) << 6;   // k * 8 -> row k
}
__device__ __forceinline__ uint32_t term_off(const LaneUnit &u, int t) {
    return (uint32_t)(((t < 4 ? u.t03 : u.t45) >> (16 * (t & 3))) & 0xffffu) * LROW;
}

// Source term of E:mass and E:energy for the lane's cell at state z, lb the
// lane's base in the wave's LDS rows.  The net production sum (E:spec-rate)
// is accumulated unit by unit: each unit's net rate of progress q is added,
// times nu'' - nu', to the omega row of each of its species.  Every row
// access of a unit is unconditional (empty reactant slots read the row of
// ones, unused term slots the discard row), so a unit's reads issue back to
// back, and the next unit's record is loaded while this one's exponentials
// are evaluated.
template <int NMAX, bool PD>
__device__ __forceinline__ void rhs_lane(const double (&z)[NMAX], double P10, double invP10,
                                         double (&fz)[NMAX], unsigned char *lb,
                                         ParamsK &pk) {
    const ExpK K = exp_k_local();
    const int N = pk.N, nS = pk.nS;
    cdouble *spec = cptr(pk.l_spec);
    const double T = z[0];
    const double invT = rcp_nr(T);
    const double l2T = log2_pos(T, K);
    const double invTa = fmin(invT, pk.invTmax);   // 1/T of the Arrhenius factors
    const uint32_t orow0 = (uint32_t)lane_row_omega(nS) * LROW;

    // mixture sums (E:mass): sum Y/W and sum (Y/W) Cp/R
    double sYW = 0.0, sYcp = 0.0;
#pragma unroll
    for (int k = 1; k < NMAX; ++k) {
        if (k < N) {
            cdouble *sp = spec + (k - 1) * LS_FIELDS;
            const double YW = z[k] * sp[LS_INVW];
            double cpR;
            if (T >= sp[LS_TMID]) cpR = cp_horner(sp + LS_CPHI, T);
            else cpR = cp_horner(sp + LS_CPLO, T);
            sYW += YW;
            sYcp += YW * cpR;
        }
    }
    const double RTW = R_ERG * T * sYW;
    const double rho = P10 * rcp_nr(RTW);   // ideal gas, g/cm^3
    const double inv_rho = RTW * invP10;

    // concentrations and cleared production rows, then the third-body
    // concentration of each efficiency set
#pragma unroll
    for (int k = 1; k < NMAX; ++k) {
        if (k < N) {
            lrow_at(lb, (uint32_t)(k - 1) * LROW) = rho * z[k] * spec[(k - 1) * LS_FIELDS + LS_INVW];
            lrow_at(lb, orow0 + (uint32_t)(k - 1) * LROW) = 0.0;
        }
    }
    const int nU = pk.nU;
    if constexpr (PD) {
        const int NMS = pk.NMS;
        cdouble *eff = cptr(pk.l_eff);
        const uint32_t mrow0 = (uint32_t)lane_row_mset(nS) * LROW;
        for (int q = 0; q < NMS; ++q) {
            double M = 0.0;
#pragma unroll
            for (int k = 1; k < NMAX; ++k)
                if (k < N) M += eff[q * nS + k - 1] * lrow_at(lb, (uint32_t)(k - 1) * LROW);
            lrow_at(lb, mrow0 + (uint32_t)q * LROW) = M;
        }
    }

    // Rates of progress (E:rxn-rate) with Arrhenius coefficients (E:rxn-const),
    // net of each forward/reverse pair, one unit per iteration for every lane.
    cdouble *units = cptr(pk.l_units);
    const int n_plain = PD ? pk.n_plain : nU;
    LaneUnit un = lane_unit(units);
    for (int u = 0; u < nU; ++u) {
        const LaneUnit cu = un;
        const double cf = lrow_at(lb, slot_off(cu.sf, 0)) * lrow_at(lb, slot_off(cu.sf, 1)) *
                          lrow_at(lb, slot_off(cu.sf, 2));
        const double cr = lrow_at(lb, slot_off(cu.sr, 0)) * lrow_at(lb, slot_off(cu.sr, 1)) *
                          lrow_at(lb, slot_off(cu.sr, 2));
        double om[LU_TERMS];
#pragma unroll
        for (int t = 0; t < LU_TERMS; ++t) om[t] = lrow_at(lb, term_off(cu, t));
        // the next unit's record (the last unit reloads its own)
        un = lane_unit(units + (size_t)(u + 1 < nU ? u + 1 : u) * LU_DOUBLES);
        double kf = exp2_b31(arrhenius_arg(cu.l2Af, cu.bf, cu.tf, l2T, invTa), K);
        double kr = exp2_b31(arrhenius_arg(cu.l2Ar, cu.br, cu.tr, l2T, invTa), K);
        if (PD && u >= n_plain) {
            cdouble *d = cptr(pk.l_pdep) + (size_t)(u - n_plain) * PDEP_DOUBLES;
            const uint64_t tag = __double_as_longlong(d[0]);
            const int kind = (int)(tag & 0xffu);
            if (kind != 0) {
                const double M = lrow_at(lb, (uint32_t)(lane_row_mset(nS) + (int)((tag >> 8) & 0xffu)) * LROW);
                if (kind == 1) {
                    kf *= M;
                    kr *= M;
                } else {
                    const double k0f = exp2_b31(arrhenius_arg(d[1], d[2], d[3], l2T, invTa), K);
                    const double k0r = exp2_b31(arrhenius_arg(d[4], d[5], d[6], l2T, invTa), K);
                    double lFc = 0.0;
                    if (kind == 3) {
                        const double Fc = (1.0 - d[8]) * exp2_sat(-T * d[9], K) +
                                          d[8] * exp2_sat(-T * d[10], K) +
                                          (d[11] > 0.0 ? exp2_sat(-d[11] * invT, K) : 0.0);
                        lFc = log2_pos(Fc, K) * LOG10_2;
                    }
                    kf = falloff_rate(kf, k0f * M, lFc, kind == 3, K);
                    kr = falloff_rate(kr, k0r * M, lFc, kind == 3, K);
                }
            }
        }
        const double q = net_rate(kf, cf, kr, cr);
#pragma unroll
        for (int t = 0; t < LU_TERMS; ++t)
            lrow_at(lb, term_off(cu, t)) = __builtin_fma(cu.dnu[t], q, om[t]);
    }

    // species equations (E:mass) and the enthalpy sum of the energy equation
    // (E:energy)
    double w[NMAX];
#pragma unroll
    for (int k = 1; k < NMAX; ++k) w[k] = (k < N) ? lrow_at(lb, orow0 + (uint32_t)(k - 1) * LROW) : 0.0;
    double hs = 0.0;
#pragma unroll
    for (int k = 1; k < NMAX; ++k) {
        if (k < N) {
            cdouble *sp = spec + (k - 1) * LS_FIELDS;
            fz[k] = sp[LS_W] * w[k] * inv_rho;
            double hRT;
            if (T >= sp[LS_TMID]) hRT = h_horner(sp + LS_HHI, T, invT);
            else hRT = h_horner(sp + LS_HLO, T, invT);
            hs += hRT * w[k];
        } else {
            fz[k] = 0.0;
        }
    }
    // dT/dt = -sum_i H_i omega_i / (rho cp); R cancels between H and cp.
    fz[0] = -T * hs * inv_rho * rcp_nr(sYcp);
}

// The row of ones of the lane's wave (written once; nothing else writes it).
__device__ __forceinline__ void lane_init_rows(unsigned char *lb, int nS) {
    lrow_at(lb, (uint32_t)lane_row_one(nS) * LROW) = 1.0;
}

// ----------------------------------------------------------- lane helpers

// Load the state of `cell` into y; false (and nothing to integrate) for a
// non-positive or non-finite T or P, or a non-finite mass fraction.
template <int NMAX>
__device__ __forceinline__ bool load_lane(const Params &p, int cell, double (&y)[NMAX],
                                          double &P10) {
    int bad = 0;
    const double T = p.T[cell];
    bad |= !(T > 0.0) || !isfinite(T);
    y[0] = T;
#pragma unroll
    for (int k = 1; k < NMAX; ++k) {
        double v = 0.0;
        if (k < p.N) {
            v = p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss];
            bad |= !isfinite(v);
        }
        y[k] = v;
    }
    const double P = p.P[cell];
    bad |= !(P > 0.0) || !isfinite(P);
    P10 = P * 10.0;
    return bad == 0;
}

template <int NMAX>
__device__ __forceinline__ void store_lane(const Params &p, int cell, const double (&y)[NMAX]) {
    p.T[cell] = y[0];
#pragma unroll
    for (int k = 1; k < NMAX; ++k)
        if (k < p.N) p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss] = y[k];
}

__device__ __forceinline__ void store_counts_lane(const Params &p, int cell, const Counts &c,
                                                  int status) {
    if (p.cell_status) p.cell_status[cell] = status;
    if (p.cell_counters) {
        int32_t *o = p.cell_counters + (size_t)cell * 8;
        o[0] = c.n_rhs; o[1] = c.n_steps; o[2] = c.n_reject; o[3] = c.n_sigma;
        o[4] = c.s_max_used; o[5] = c.s_hash; o[6] = status; o[7] = c.n_piter;
    }
}

// The power-method direction of Sec. 2.4 is kept between calls of the power
// method in the cell's own input row (T[cell], Y[cell][*]): the row is read
// once when the cell starts and written with the final state when it ends,
// and nothing else reads it in between, so the direction needs no registers
// of its own while the source term is evaluated.
template <int NMAX>
__device__ __forceinline__ void park_direction(const Params &p, int cell, const double (&y)[NMAX],
                                               const double (&z)[NMAX]) {
    p.T[cell] = z[0] - y[0];
#pragma unroll
    for (int k = 1; k < NMAX; ++k)
        if (k < p.N) p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss] = z[k] - y[k];
}

template <int NMAX>
__device__ __forceinline__ void fetch_direction(const Params &p, int cell, double (&v)[NMAX]) {
    v[0] = p.T[cell];
#pragma unroll
    for (int k = 1; k < NMAX; ++k)
        v[k] = (k < p.N) ? p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss] : 0.0;
}

// Per-lane aggregate statistics in 32 bits (flushed into the 64-bit launch
// totals before any lane's evaluation count could wrap).
struct AggL {
    unsigned rhs, steps, rej, sig, piter;
    int smax, failed, worst;
};

__device__ __forceinline__ void agg_lane(AggL &a, const Counts &c, int status) {
    a.rhs += (unsigned)c.n_rhs;
    a.steps += (unsigned)c.n_steps;
    a.rej += (unsigned)c.n_reject;
    a.sig += (unsigned)c.n_sigma;
    a.piter += (unsigned)c.n_piter;
    a.smax = max(a.smax, c.s_max_used);
    a.failed += (status != ST_OK);
    a.worst = max(a.worst, status);
}

__device__ __forceinline__ void flush_lane(const Params &p, AggL &a, unsigned long long slots) {
    flush_agg(p, Agg{a.rhs, a.steps, a.rej, a.sig, a.piter, a.smax, a.failed, a.worst}, true,
              slots);
    a = AggL{0, 0, 0, 0, 0, a.smax, 0, a.worst};
}

// Before a cell's counts are added: flush every lane's totals when one of
// them has passed 2^30 evaluations (a cell adds fewer than 2^31).
__device__ __forceinline__ void agg_guard(const Params &p, AggL &a) {
    if (__any(a.rhs >= 0x40000000u || a.steps >= 0x40000000u || a.piter >= 0x40000000u))
        flush_lane(p, a, 0ull);
}

// Cells for the lanes that ask (want): the first pass gives every lane its
// own cell of the launch (`first`), later passes claim the next cells of the
// work queue together, one atomic per wave (persistent launches), or none
// (plain launches: the grid covers every cell).  A lane whose claim is past
// the last cell gets -1.
__device__ __forceinline__ int claim_lane(const Params &p, bool want) {
    const unsigned long long m = __ballot(want);
    if (!p.persistent || m == 0ull) return -1;
    const int lead = __builtin_ctzll(m);
    int base = 0;
    if ((int)__lane_id() == lead) base = atomicAdd(p.queue, __popcll(m));
    base = __shfl(base, lead, 64);
    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    const long long c = (long long)p.groups_total + base + rank;
    return want && c < p.n_cells ? (int)c : -1;
}

// Chebyshev values of Sec. 2.4 at w0 for the coefficients of stage j >= 2 of
// an s-stage step, by the same recurrence (and the same roundings) as the
// lane-group kernels advance one stage at a time: T_{j-1}, T_{j-2} and their
// first and second derivatives, b_{j-1} and the reciprocals 1/b_{j-1},
// 1/b_{j-2} as those kernels carry them (1/b_1 = w0, 1/b_0 = 1/b_2).
struct ChebPrev {
    double Tm1, Tm2, Tpm1, Tpm2, Tppm1, Tppm2, bm1, ibm1, ibm2;
};

__device__ __forceinline__ ChebPrev cheb_prev(double w0, int j) {
    ChebPrev c;
    c.Tm1 = w0; c.Tm2 = 1.0; c.Tpm1 = 1.0; c.Tpm2 = 0.0; c.Tppm1 = 0.0; c.Tppm2 = 0.0;
    c.bm1 = 1.0 / w0;
    c.ibm1 = w0;
    // 1/b_0 = 1/b_2 with b_2 from the degree-2 values
    {
        const double P2 = 2.0 * w0 * 1.0 - 0.0 + 2.0 * w0;
        const double Q2 = 2.0 * w0 * 0.0 - 0.0 + 4.0 * 1.0;
        c.ibm2 = 1.0 / (Q2 / (P2 * P2));
    }
    for (int jj = 2; jj < j; ++jj) {
        const double Tj = 2.0 * w0 * c.Tm1 - c.Tm2;
        const double Tpj = 2.0 * w0 * c.Tpm1 - c.Tpm2 + 2.0 * c.Tm1;
        const double Tppj = 2.0 * w0 * c.Tppm1 - c.Tppm2 + 4.0 * c.Tpm1;
        const double bj = Tppj / (Tpj * Tpj);
        c.Tm2 = c.Tm1; c.Tm1 = Tj; c.Tpm2 = c.Tpm1; c.Tpm1 = Tpj; c.Tppm2 = c.Tppm1;
        c.Tppm1 = Tppj;
        c.bm1 = bj; c.ibm2 = c.ibm1; c.ibm1 = 1.0 / bj;
    }
    return c;
}

// ------------------------------------------------------------------- RKC

template <int NMAX, bool PD>
__global__ __launch_bounds__(256) void rkc_lane_kernel(Params p) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    unsigned char *lb = lds_raw + (size_t)(threadIdx.x >> 6) * p.lane_rows * LROW +
                        (threadIdx.x & 63) * 8;
    lane_init_rows(lb, p.nS);
    const int N = p.N;
    const double u_round = 0x1p-53;
    const double t_end = p.dt;
    const double h_min = 10.0 * u_round * t_end;
    const double sqrt_u = sqrt(u_round);

    // w1 is both the latest stage and the point where the source term is
    // evaluated next (the probe of the power method, the tentative initial
    // step, the first stage)
    double y[NMAX], f0[NMAX], w1[NMAX], w2[NMAX], fz[NMAX];
    // control state of the lane's cell (the lane-group kernels' RkcState).
    // aux0/aux1 hold delta and the previous estimate during the power method,
    // then the tentative step during the initial-step phase, then w0 and w1
    // of Sec. 2.4 during the stages of a step whose coefficients are not
    // tabulated: the three uses never overlap in time.
    double t = 0.0, h = 0.0, sigma = 0.0, aux0 = 0.0, aux1 = 0.0, h_prev = 0.0, rprev = 0.0,
           P10 = 1e6, invP10 = 1e-6;
    int cell = -1, phase = PH_F0, k_pow = 0, s = 0, j = 0, last = 0, need_sigma = 0,
        since_sigma = 0, predictive = 0, after = AFTER_INIT, tab = 0;
    // action decided after an evaluation that sets up the next evaluation
    // point (start of a power method, or stage count and first stage); it is
    // carried out at the top of the next iteration, where the source-term
    // output is dead, so that it does not share registers with it
    int pending = ACT_NONE;
    Counts c{0, 0, 0, 0, 0, 0, 0};
    AggL agg{0, 0, 0, 0, 0, 0, 0, 0};

    // Take cells until one has valid input (bad ones are marked and skipped)
    // or the work runs out; `first` is the lane's cell of the launch.
    auto acquire = [&](bool want, int first) {
        int cand = first;
        for (;;) {
            if (want && cand >= 0) {
                double P10n;
                if (load_lane<NMAX>(p, cand, y, P10n)) {
                    cell = cand;
                    P10 = P10n;
                    invP10 = 1.0 / P10n;
                    c = Counts{0, 0, 0, 0, 0, 0, 0};
                    t = 0.0; need_sigma = 0; since_sigma = 0; predictive = 0;
                    h_prev = 0.0; rprev = 0.0;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) w1[i] = y[i];
                    phase = PH_F0;
                    pending = ACT_NONE;
                    want = false;
                } else {
                    const Counts zc{0, 0, 0, 0, 0, 0, 0};
                    store_counts_lane(p, cand, zc, ST_BADINPUT);
                    agg_lane(agg, zc, ST_BADINPUT);
                }
            } else if (want) {
                want = false;   // nothing left for this lane
                cell = -1;
            }
            if (!__any(want)) break;
            cand = claim_lane(p, want);
        }
    };

#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        y[i] = f0[i] = w2[i] = fz[i] = 0.0;
        w1[i] = (i == 0) ? 1000.0 : 0.0;
    }
    {
        const long long first = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        acquire(true, first < p.n_cells ? (int)first : -1);
    }

    unsigned iters = 0;
    for (;;) {
        if (!__any(cell >= 0)) break;
        ++iters;
        if (cell >= 0 && pending != ACT_NONE) {
            ParamsK &pk = *params_k();
            if (pending == ACT_POWER_INIT || pending == ACT_POWER_STEP) {
                double v[NMAX];
                if (pending == ACT_POWER_INIT) {
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) v[i] = f0[i];
                } else {
                    fetch_direction<NMAX>(p, cell, v);
                }
                double ny2 = 0.0, nv2 = 0.0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) { ny2 += y[i] * y[i]; nv2 += v[i] * v[i]; }
                const double ny = sqrt(ny2);
                const double delta = (ny > 0.0) ? sqrt_u * ny : sqrt_u;
                double nv = sqrt(nv2);
                if (!(nv > 0.0)) {
                    double o2 = 0.0;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        v[i] = (i < N) ? 1.0 : 0.0;
                        o2 += v[i] * v[i];
                    }
                    nv = sqrt(o2);
                }
                const double q = delta / nv;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) w1[i] = y[i] + q * v[i];
                aux0 = delta;
                k_pow = 1;
                aux1 = 0.0;
                after = (pending == ACT_POWER_INIT) ? AFTER_INIT : AFTER_STEP;
                phase = PH_POWER;
            } else if (pending == ACT_AFTER_SIGMA) {
                // stage count from the spectral radius, then the first stage (E:rkc1)
                double hh = h;
                int lst = (hh >= t_end - t);
                if (lst) hh = t_end - t;
                const double sq = floor(sqrt(1.0 + 1.54 * hh * sigma));
                int ss;
                if (1.0 + sq > (double)pk.s_max) {
                    ss = pk.s_max;
                    hh = ((double)(pk.s_max - 1) * (double)(pk.s_max - 1) - 1.0) / (1.54 * sigma);
                    lst = 0;
                } else {
                    ss = 1 + (int)sq;
                }
                c.s_hash = (int)((unsigned)c.s_hash * 31u + (unsigned)ss);
                c.s_max_used = max(c.s_max_used, ss);
                double mu_t1;
                if (ss <= pk.coef_smax) {
                    mu_t1 = pk.coef[4 * coef_offset(ss)];
                    tab = 1;
                } else {
                    // w1 = T'_s / T''_s at w0 = 1 + kappa/s^2; the stages
                    // recompute the recurrences up to their own index
                    tab = 0;
                    const double w0 = 1.0 + KAPPA / ((double)ss * (double)ss);
                    double T0 = 1.0, T1 = w0, Pa = 0.0, Pb = 1.0, Qa = 0.0, Qb = 0.0;
                    for (int jj = 2; jj <= ss; ++jj) {
                        const double Tn = 2.0 * w0 * T1 - T0;
                        const double Pn = 2.0 * w0 * Pb - Pa + 2.0 * T1;
                        const double Qn = 2.0 * w0 * Qb - Qa + 4.0 * Pb;
                        T0 = T1; T1 = Tn; Pa = Pb; Pb = Pn; Qa = Qb; Qb = Qn;
                    }
                    aux0 = w0;
                    aux1 = Pb / Qb;
                    mu_t1 = (1.0 / w0) * aux1;   // b_1 w1 with b_1 = 1/w0
                }
                h = hh; last = lst; s = ss; j = 2;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    w2[i] = y[i];
                    w1[i] = y[i] + mu_t1 * hh * f0[i];
                }
                phase = PH_STAGE;
            }
            pending = ACT_NONE;
        }
        {
            ParamsK &pk = *params_k();
            rhs_lane<NMAX, PD>(w1, P10, invP10, fz, lb, pk);
        }
        bool fin_now = false;
        int fin = ST_OK;
        if (cell >= 0) {
            ParamsK &pk = *params_k();
            c.n_rhs += 1;
            int act = ACT_NONE;
            if (phase == PH_STAGE) {
                // (E:rkcj): tabulated coefficients of (s, j), or the
                // recurrences of Sec. 2.4 recomputed up to stage j
                double mu, nu, mut, gam;
                if (tab) {
                    const double4 cf =
                        *reinterpret_cast<const double4 *>(pk.coef + 4 * (coef_offset(s) + j - 1));
                    mu = cf.x; nu = cf.y; mut = cf.z; gam = cf.w;
                } else {
                    const double w0 = aux0;
                    const ChebPrev q = cheb_prev(w0, j);
                    const double Tpj = 2.0 * w0 * q.Tpm1 - q.Tpm2 + 2.0 * q.Tm1;
                    const double Tppj = 2.0 * w0 * q.Tppm1 - q.Tppm2 + 4.0 * q.Tpm1;
                    const double bj = Tppj / (Tpj * Tpj);
                    mu = 2.0 * bj * w0 * q.ibm1;
                    nu = -bj * q.ibm2;
                    mut = 2.0 * bj * aux1 * q.ibm1;
                    gam = -(1.0 - q.bm1 * q.Tm1) * mut;
                }
                const double c0 = 1.0 - mu - nu, ch1 = mut * h, ch2 = gam * h;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const double wj = c0 * y[i] + mu * w1[i] + nu * w2[i] + ch1 * fz[i] + ch2 * f0[i];
                    w2[i] = w1[i];
                    w1[i] = wj;
                }
                if (j == s) phase = PH_ERR;
                else j = j + 1;
            } else if (phase == PH_ERR) {
                // error estimate, weighted RMS norm (E:rmsE) and step control
                double e2 = 0.0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    if (i < N) {
                        const double d = 0.8 * (y[i] - w1[i]) + 0.4 * h * (f0[i] + fz[i]);
                        const double m = fmax(fabs(y[i]), fabs(w1[i]));
                        const double w = pk.atol + pk.rtol * m;
                        const double sc = (w < 0x1p-900) ? 0x1p200 : 1.0;
                        const double q = (d * sc) * rcp_nr(w * sc);
                        e2 += q * q;
                    }
                }
                e2 *= pk.invN;
                if (e2 <= NORM2_ACCEPT) {
                    c.n_steps += 1;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) { y[i] = w1[i]; f0[i] = fz[i]; }
                    if (last) {
                        fin_now = true;
                        fin = ST_OK;
                    } else {
                        t = t + h;
                        since_sigma += 1;
                        need_sigma = (since_sigma >= 25);
                        double fac, r = 0.0;
                        if (e2 == 0.0) {
                            fac = 10.0;
                        } else {
                            r = rsixth_pos(e2);
                            if (!predictive) fac = 0.8 * r;
                            else if (rprev == 0.0) fac = 0.0;
                            else fac = 0.8 * h * r * r * rcp_nr(h_prev * rprev);
                        }
                        if (fac > 10.0) fac = 10.0;
                        if (fac < 0.1) fac = 0.1;
                        h_prev = h;
                        rprev = r;
                        predictive = 1;
                        h = h * fac;
                        act = ACT_BEGIN_STEP;
                    }
                } else {
                    c.n_reject += 1;
                    double fac = isfinite(e2) ? 0.8 * rsixth_pos(e2) : 0.1;
                    if (fac < 0.1) fac = 0.1;
                    h = h * fac;
                    need_sigma = 1;
                    predictive = 0;
                    act = ACT_BEGIN_STEP;
                }
                if (act == ACT_BEGIN_STEP && h < h_min) { act = ACT_NONE; fin_now = true; fin = ST_UNDERFLOW; }
            } else if (phase == PH_POWER) {
                // nonlinear power method: one difference quotient per iteration
                c.n_piter += 1;
                double ng2 = 0.0, dz2 = 0.0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const double gv = fz[i] - f0[i];
                    const double dd = w1[i] - y[i];
                    ng2 += gv * gv;
                    dz2 += dd * dd;
                }
                const double ng = sqrt(ng2);
                double sig = ng / sqrt(dz2);
                bool stop = false;
                if (k_pow >= 2 && fabs(sig - aux1) <= 0.01 * sig) stop = true;
                else if (ng == 0.0) { sig = 0.0; stop = true; }
                else if (k_pow == 50) stop = true;
                if (stop) {
                    park_direction<NMAX>(p, cell, y, w1);
                    c.n_sigma += 1;
                    sigma = 1.2 * sig;
                    if (!isfinite(sigma)) {
                        fin_now = true;
                        fin = ST_NONFINITE;
                    } else if (after == AFTER_INIT) {
                        // tentative initial step 1/sigma, capped at dt
                        double htt = (sigma > 0.0) ? 1.0 / sigma : t_end;
                        if (htt > t_end) htt = t_end;
                        aux0 = htt;
#pragma unroll
                        for (int i = 0; i < NMAX; ++i) w1[i] = y[i] + htt * f0[i];
                        phase = PH_INIT;
                    } else {
                        need_sigma = 0;
                        since_sigma = 0;
                        act = ACT_AFTER_SIGMA;
                    }
                } else {
                    const double q = aux0 / ng;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) w1[i] = y[i] + q * (fz[i] - f0[i]);
                    aux1 = sig;
                    k_pow = k_pow + 1;
                }
            } else if (phase == PH_INIT) {
                // initial step from the error of the tentative step
                const double ht = aux0;
                double e2 = 0.0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    if (i < N) {
                        const double d = ht * (fz[i] - f0[i]);
                        const double m = fabs(y[i]);
                        const double w = pk.atol + pk.rtol * m;
                        const double sc = (w < 0x1p-900) ? 0x1p200 : 1.0;
                        const double q = (d * sc) * rcp_nr(w * sc);
                        e2 += q * q;
                    }
                }
                const double e0 = sqrt(e2 * pk.invN);
                if (!isfinite(e0)) {
                    fin_now = true;
                    fin = ST_NONFINITE;
                } else {
                    double hh = (e0 > 0.0) ? 0.1 * ht / sqrt(e0) : ht;
                    if (hh < h_min) hh = h_min;
                    if (hh > t_end) hh = t_end;
                    h = hh;
                    t = 0.0;
                    act = ACT_BEGIN_STEP;
                }
            } else {   // PH_F0: f(y0)
                bool bad = false;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    f0[i] = fz[i];
                    bad |= (i < N) && !isfinite(fz[i]);
                }
                if (bad) {
                    fin_now = true;
                    fin = ST_NONFINITE;
                } else {
                    act = ACT_POWER_INIT;   // first direction: f(y0)
                }
            }

            if (act == ACT_BEGIN_STEP) {
                if (c.n_steps + c.n_reject >= pk.max_steps) { act = ACT_NONE; fin_now = true; fin = ST_MAXSTEPS; }
                else if (need_sigma) act = ACT_POWER_STEP;
                else act = ACT_AFTER_SIGMA;
            }
            if (act == ACT_POWER_INIT || act == ACT_POWER_STEP || act == ACT_AFTER_SIGMA)
                pending = act;
            if (fin_now) {
                store_lane<NMAX>(p, cell, y);
                store_counts_lane(p, cell, c, fin);
                // the lane's next cell starts from the safe dummy state until
                // it is loaded (a lane without a cell keeps evaluating it)
#pragma unroll
                for (int i = 0; i < NMAX; ++i) w1[i] = (i == 0) ? 1000.0 : 0.0;
                P10 = 1e6;
                invP10 = 1e-6;
                cell = -1;
            }
        }
        if (__any(fin_now)) {
            agg_guard(p, agg);
            if (fin_now) agg_lane(agg, c, fin);
            acquire(fin_now, claim_lane(p, fin_now));
        }
    }
    flush_lane(p, agg, (unsigned long long)iters * 64ull);
}

// ------------------------------------------------------------------ RKCK

template <int NMAX, bool PD>
__global__ __launch_bounds__(256) void rkck_lane_kernel(Params p) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    unsigned char *lb = lds_raw + (size_t)(threadIdx.x >> 6) * p.lane_rows * LROW +
                        (threadIdx.x & 63) * 8;
    lane_init_rows(lb, p.nS);
    const int N = p.N;
    const double u_round = 0x1p-53;
    const double t_end = p.dt;
    const double h_min = 10.0 * u_round * t_end;

    double y[NMAX], k1[NMAX], k2[NMAX], k3[NMAX], k4[NMAX], k5[NMAX], z[NMAX], fz[NMAX];
    double t = 0.0, h = 0.0, P10 = 1e6, invP10 = 1e-6;
    int cell = -1, phase = CK_K1, last = 0;
    Counts c{0, 0, 0, 0, 0, 0, 0};
    AggL agg{0, 0, 0, 0, 0, 0, 0, 0};

    auto acquire = [&](bool want, int first) {
        int cand = first;
        for (;;) {
            if (want && cand >= 0) {
                double P10n;
                if (load_lane<NMAX>(p, cand, y, P10n)) {
                    cell = cand;
                    P10 = P10n;
                    invP10 = 1.0 / P10n;
                    c = Counts{0, 0, 0, 0, 0, 0, 0};
                    t = 0.0;
                    // first trial step is the whole interval; the last step lands on dt
                    h = t_end;
                    last = 1;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) z[i] = y[i];
                    phase = CK_K1;
                    want = false;
                } else {
                    const Counts zc{0, 0, 0, 0, 0, 0, 0};
                    store_counts_lane(p, cand, zc, ST_BADINPUT);
                    agg_lane(agg, zc, ST_BADINPUT);
                }
            } else if (want) {
                want = false;
                cell = -1;
            }
            if (!__any(want)) break;
            cand = claim_lane(p, want);
        }
    };

#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        y[i] = k1[i] = k2[i] = k3[i] = k4[i] = k5[i] = fz[i] = 0.0;
        z[i] = (i == 0) ? 1000.0 : 0.0;
    }
    {
        const long long first = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        acquire(true, first < p.n_cells ? (int)first : -1);
    }

    unsigned iters = 0;
    for (;;) {
        if (!__any(cell >= 0)) break;
        ++iters;
        {
            ParamsK &pk = *params_k();
            rhs_lane<NMAX, PD>(z, P10, invP10, fz, lb, pk);
        }
        bool fin_now = false;
        int fin = ST_OK;
        if (cell >= 0) {
            c.n_rhs += 1;
            switch (phase) {
            case CK_K1:
#pragma unroll
                for (int i = 0; i < NMAX; ++i) { k1[i] = h * fz[i]; z[i] = y[i] + CK_B21 * k1[i]; }
                phase = CK_K2;
                break;
            case CK_K2:
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    k2[i] = h * fz[i];
                    z[i] = y[i] + CK_B31 * k1[i] + CK_B32 * k2[i];
                }
                phase = CK_K3;
                break;
            case CK_K3:
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    k3[i] = h * fz[i];
                    z[i] = y[i] + CK_B41 * k1[i] + CK_B42 * k2[i] + CK_B43 * k3[i];
                }
                phase = CK_K4;
                break;
            case CK_K4:
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    k4[i] = h * fz[i];
                    z[i] = y[i] + CK_B51 * k1[i] + CK_B52 * k2[i] + CK_B53 * k3[i] + CK_B54 * k4[i];
                }
                phase = CK_K5;
                break;
            case CK_K5:
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    k5[i] = h * fz[i];
                    z[i] = y[i] + CK_B61 * k1[i] + CK_B62 * k2[i] + CK_B63 * k3[i]
                         + CK_B64 * k4[i] + CK_B65 * k5[i];
                }
                phase = CK_K6;
                break;
            default: {   // CK_K6: embedded error estimate and step control (E:hnew)
                double y5[NMAX];
                double emax = 0.0;
                bool bad = false;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const double k6 = h * fz[i];
                    y5[i] = y[i] + CK_C1 * k1[i] + CK_C3 * k3[i] + CK_C4 * k4[i] + CK_C6 * k6;
                    const double del = CK_D1 * k1[i] + 0.0 * k2[i] + CK_D3 * k3[i] + CK_D4 * k4[i]
                                     + CK_D5 * k5[i] + CK_D6 * k6;
                    if (i < N) {
                        const double d0 = p.rtol * (fabs(y[i]) + fabs(k1[i]) + 1e-30);
                        const double r = fabs(del / d0);
                        if (!isfinite(r)) bad = true;
                        else emax = fmax(emax, r);
                    }
                }
                const double errmax = bad ? __builtin_inf() : emax;
                double hn = h;
                int f = -1;
                if (errmax <= 1.0) {
                    c.n_steps += 1;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) y[i] = y5[i];
                    if (last) {
                        f = ST_OK;
                    } else {
                        t = t + h;
                        double fac = (errmax == 0.0) ? 5.0 : 0.9 * exp2_sat(-0.2 * log2_pos(errmax));
                        if (fac > 5.0) fac = 5.0;
                        hn = h * fac;
                    }
                } else {
                    c.n_reject += 1;
                    double fac = isfinite(errmax) ? 0.9 * exp2_sat(-0.25 * log2_pos(errmax)) : 0.1;
                    if (fac < 0.1) fac = 0.1;
                    hn = h * fac;
                }
                if (f < 0) {
                    if (hn < h_min) f = ST_UNDERFLOW;
                    else if (c.n_steps + c.n_reject >= p.max_steps) f = ST_MAXSTEPS;
                    else {
                        const int lst = (hn >= t_end - t);
                        if (lst) hn = t_end - t;
                        last = lst;
                        h = hn;
#pragma unroll
                        for (int i = 0; i < NMAX; ++i) z[i] = y[i];
                        phase = CK_K1;
                    }
                }
                if (f >= 0) { fin_now = true; fin = f; }
            }
            }
            if (fin_now) {
                store_lane<NMAX>(p, cell, y);
                store_counts_lane(p, cell, c, fin);
#pragma unroll
                for (int i = 0; i < NMAX; ++i) z[i] = (i == 0) ? 1000.0 : 0.0;
                P10 = 1e6;
                invP10 = 1e-6;
                cell = -1;
            }
        }
        if (__any(fin_now)) {
            agg_guard(p, agg);
            if (fin_now) agg_lane(agg, c, fin);
            acquire(fin_now, claim_lane(p, fin_now));
        }
    }
    flush_lane(p, agg, (unsigned long long)iters * 64ull);
}

// ------------------------------------------------------- source-term kernel

template <int NMAX, bool PD>
__global__ __launch_bounds__(256) void rhs_lane_kernel(Params p) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    unsigned char *lb = lds_raw + (size_t)(threadIdx.x >> 6) * p.lane_rows * LROW +
                        (threadIdx.x & 63) * 8;
    lane_init_rows(lb, p.nS);
    const long long cl = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = cl < p.n_cells;
    const int cell = active ? (int)cl : 0;
    double z[NMAX], fz[NMAX];
    double P10 = 1e6;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) z[i] = (i == 0) ? 1000.0 : 0.0;
    if (active) {
        z[0] = p.T[cell];
#pragma unroll
        for (int k = 1; k < NMAX; ++k)
            if (k < p.N) z[k] = p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss];
        P10 = p.P[cell] * 10.0;
    }
    rhs_lane<NMAX, PD>(z, P10, 1.0 / P10, fz, lb, *params_k());
    if (active) {
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k < p.N) p.F[(long long)cell * p.fcs + (long long)k * p.fss] = fz[k];
    }
}

}  // namespace rkcdev
