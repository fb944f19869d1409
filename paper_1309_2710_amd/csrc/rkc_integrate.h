// Integrator kernels: RKC (Sec. 2.4) and RKCK (Sec. 2.3) as RHS-synchronous
// state machines over lane groups (see rkc_device.h for the data layout).
//
// Control flow follows the paper's algorithm with these readings of points it
// leaves open: b_1 = 1/omega_0 as printed and a_j = 1 - b_j T_j(omega_0);
// stage count 1 + floor(sqrt(1 + 1.54 h sigma)) capped at s_max; initial
// tentative step min(1/sigma, dt); predictive step controller with factor
// 0.8 (h_n/h_{n-1}) err_n^{1/3} / err_{n+1}^{2/3} (non-predictive 0.8/err^{1/3}
// on the first accepted step and after a rejection), clamped to [0.1, 10];
// spectral radius by a nonlinear power method (delta = sqrt(u) |y|, stop when
// two successive estimates agree to 1 %, at most 50 iterations, safety factor
// 1.2), recomputed every 25 accepted steps and after each rejection,
// warm-started from the saved direction; the last step lands exactly on dt; a
// trial step with a non-finite error estimate is rejected with factor 0.1.
#pragma once

#include "rkc_device.h"

namespace rkcdev {

enum { PH_F0 = 0, PH_POWER = 1, PH_INIT = 2, PH_STAGE = 3, PH_ERR = 4 };
enum { CK_K1 = 10, CK_K2, CK_K3, CK_K4, CK_K5, CK_K6 };
enum { ST_OK = 0, ST_UNDERFLOW = 1, ST_MAXSTEPS = 2, ST_NONFINITE = 3, ST_BADINPUT = 4 };
enum { AFTER_INIT = 0, AFTER_STEP = 1 };

struct Counts {
    int n_rhs, n_steps, n_reject, n_sigma, s_max_used, s_hash, n_piter;
};

// Per-group aggregate statistics, kept in the group's LDS state record until
// the kernel ends (they would otherwise hold a dozen registers for its whole
// lifetime).
struct Agg {
    unsigned long long rhs, steps, rej, sig, piter;
    int smax, failed, worst;
};

__device__ __forceinline__ void agg_cell(Agg &a, const Counts &c, int status) {
    a.rhs += (unsigned)c.n_rhs;
    a.steps += (unsigned)c.n_steps;
    a.rej += (unsigned)c.n_reject;
    a.sig += (unsigned)c.n_sigma;
    a.piter += (unsigned)c.n_piter;
    a.smax = max(a.smax, c.s_max_used);
    a.failed += (status != ST_OK);
    a.worst = max(a.worst, status);
}

__device__ __forceinline__ unsigned long long wsum_u64(unsigned long long x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}
__device__ __forceinline__ int wmax_i(int x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m, 64));
    return x;
}

// `slots` is the number of source-term evaluations the wave issued (loop
// iterations times groups per wave); with n_rhs it gives the fraction of
// issued evaluations that advanced a cell.
__device__ __forceinline__ void flush_agg(const Params &p, Agg a, bool leader,
                                          unsigned long long slots) {
    if (!leader) a = Agg{0, 0, 0, 0, 0, 0, 0, 0};
    const unsigned long long r = wsum_u64(a.rhs), s = wsum_u64(a.steps), j = wsum_u64(a.rej),
                             g = wsum_u64(a.sig), pi = wsum_u64(a.piter),
                             f = wsum_u64((unsigned long long)a.failed);
    const int sm = wmax_i(a.smax), w = wmax_i(a.worst);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(p.agg + 0, r);
        atomicAdd(p.agg + 1, s);
        atomicAdd(p.agg + 2, j);
        atomicAdd(p.agg + 3, g);
        atomicAdd(p.agg + 4, pi);
        atomicMax(p.agg + 5, (unsigned long long)sm);
        atomicAdd(p.agg + 6, f);
        atomicMax(p.agg + 7, (unsigned long long)w);
        atomicAdd(p.agg + 8, slots);
    }
}

template <int G>
__device__ __forceinline__ int next_cell(const Params &p, int g) {
    if (!p.persistent) return p.n_cells;
    int c = 0;
    if (g == 0) c = atomicAdd(p.queue, 1);
    c = __shfl(c, 0, G);
    return p.groups_total + c;
}

template <int G, int NSL>
__device__ __forceinline__ bool load_state(const Params &p, int cell, int g, double (&y)[NSL],
                                           double &P10) {
    int bad = 0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        double v = 0.0;
        if (k == 0) {
            v = p.T[cell];
            bad |= !(v > 0.0) || !isfinite(v);
        } else if (k < p.N) {
            v = p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss];
            bad |= !isfinite(v);
        }
        y[s] = v;
    }
    const double P = p.P[cell];
    bad |= !(P > 0.0) || !isfinite(P);
    bad = gor<G>(bad);
    P10 = P * 10.0;
    return bad == 0;
}

template <int G, int NSL>
__device__ __forceinline__ void store_state(const Params &p, int cell, int g, const double (&y)[NSL]) {
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        if (k == 0) p.T[cell] = y[s];
        else if (k < p.N) p.Y[(long long)cell * p.ycs + (long long)(k - 1) * p.yss] = y[s];
    }
}

__device__ __forceinline__ void store_counts(const Params &p, int cell, int g, const Counts &c,
                                             int status) {
    if (g != 0) return;
    if (p.cell_status) p.cell_status[cell] = status;
    if (p.cell_counters) {
        int32_t *o = p.cell_counters + (size_t)cell * 8;
        o[0] = c.n_rhs; o[1] = c.n_steps; o[2] = c.n_reject; o[3] = c.n_sigma;
        o[4] = c.s_max_used; o[5] = c.s_hash; o[6] = status; o[7] = c.n_piter;
    }
}

// The kernel's parameter block (the only kernel argument, at the start of
// the kernarg segment) through a pointer the compiler cannot see through:
// fields read through it are loaded with scalar loads where they are used,
// instead of occupying scalar registers for the whole kernel.
typedef const __attribute__((address_space(4))) Params ParamsK;
__device__ __forceinline__ ParamsK *params_k() {
    ParamsK *k = (ParamsK *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(k));
    return k;
}

// Square of the weighted RMS norm (E:rmsE) over the N state components of
// the group (the mean of the squared weighted components).
template <int G, int NSL>
__device__ __forceinline__ double rms_norm2(const double (&d)[NSL], const double (&ya)[NSL],
                                            const double (&yb)[NSL], double rtol, double atol,
                                            int g, int N, double invN) {
    double s2 = 0.0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        if (k < N) {
            const double m = fmax(fabs(ya[s]), fabs(yb[s]));
            const double w = atol + rtol * m;
            // d / w by a refined reciprocal; tiny weights (only possible with
            // atol = 0) are scaled by 2^200 first, exactly, so that the
            // reciprocal stays in range.  A zero weight (atol = 0 and y = 0)
            // gives a non-finite norm.
            const double sc = (w < 0x1p-900) ? 0x1p200 : 1.0;
            const double q = (d[s] * sc) * rcp_nr(w * sc);
            s2 += q * q;
        }
    }
    s2 = gsum<G>(s2);
    return s2 * invN;
}

// The correctly rounded square root of m is at most 1 exactly when m is at
// most the double that follows 1 (sqrt(1 + 2^-52) rounds to 1).
constexpr double NORM2_ACCEPT = 0x1.0000000000001p0;

#define RKC_KERNEL_PROLOGUE                                                                  \
    extern __shared__ __align__(16) unsigned char lds_raw[];                                 \
    const int groups = blockDim.x / G;                                                       \
    const int gib = threadIdx.x / G;                                                         \
    const int g = threadIdx.x % G;                                                           \
    const Shape sh = shape_of(p, G, RUC);                                                    \
    LdsPtrs lp = carve(lds_raw, sh, groups);                                                 \
    stage_tables(p, G, lp, RUC == 0 ? p.RU * G : 0, RUC >= 0);                               \
    GroupLds L = group_view(lp, sh, gib);                                                    \
    if constexpr (RUC < 0) global_tables(L, p);                                              \
    group_init(L, p, G, g);                                                                  \
    __syncthreads();                                                                         \
    UnitRegs<RUC> ur;                                                                        \
    load_unit_regs<RUC>(p, ur, g, G);                                                        \
    const int N = p.N;                                                                       \
    const double u_round = 0x1p-53;                                                          \
    const double t_end = p.dt;                                                               \
    const double h_min = 10.0 * u_round * t_end;

// Per-group control state of the RKC machine, kept in LDS: it is only used
// between source-term evaluations, so it does not occupy registers while the
// evaluation runs.  Every lane of the group writes identical values.
struct RkcState {
    double t, h, sigma, sigma_prev, delta, ht, h_prev, rprev, P10, invP10;
    double w0, w1, Tm1, Tm2, Tpm1, Tpm2, Tppm1, Tppm2, bm1, ibm1, ibm2;
    int cell, phase, k_pow, s, j, last, need_sigma, since_sigma, predictive, after, tab;
    Counts c;
    Agg agg;
};
static_assert(sizeof(RkcState) <= STATE_BYTES, "RKC state exceeds its LDS slot");

// Actions that follow the phase-specific part of one loop iteration.
enum { ACT_NONE = 0, ACT_BEGIN_STEP, ACT_AFTER_SIGMA, ACT_POWER_INIT, ACT_POWER_STEP, ACT_FINISH };

// ------------------------------------------------------------------- RKC

template <int G, int NSL, int RUC, bool PD>
__global__ __launch_bounds__((Occ<RUC, NSL>::threads), (Occ<RUC, NSL>::waves)) void rkc_kernel(Params p) {
    RKC_KERNEL_PROLOGUE
    const double sqrt_u = sqrt(u_round);
    RkcState &S = *reinterpret_cast<RkcState *>(lp.states + (size_t)gib * STATE_BYTES);

    double y[NSL], f0[NSL], wm1[NSL], wm2[NSL], z[NSL], fz[NSL], v[NSL];
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
        y[i] = f0[i] = wm1[i] = wm2[i] = fz[i] = v[i] = 0.0;
        z[i] = (i == 0 && g == 0) ? 1000.0 : 0.0;
    }
    S.P10 = 1e6;
    S.agg = Agg{0, 0, 0, 0, 0, 0, 0, 0};
    S.invP10 = 1e-6;

    // Take the next valid cell starting at `first` (cells with bad input are
    // marked and skipped); S.cell = -1 when the queue is exhausted.
    auto acquire = [&](int first) {
        int cell = first;
        while (cell < p.n_cells) {
            double P10;
            if (load_state<G, NSL>(p, cell, g, y, P10)) {
                S.cell = cell;
                S.P10 = P10;
                S.invP10 = 1.0 / P10;
                S.c = Counts{0, 0, 0, 0, 0, 0, 0};
                S.t = 0.0; S.need_sigma = 0; S.since_sigma = 0; S.predictive = 0;
                S.h_prev = 0.0; S.rprev = 0.0;
#pragma unroll
                for (int i = 0; i < NSL; ++i) z[i] = y[i];
                S.phase = PH_F0;
                return;
            }
            Counts zc{0, 0, 0, 0, 0, 0, 0};
            store_counts(p, cell, g, zc, ST_BADINPUT);
            agg_cell(S.agg, zc, ST_BADINPUT);
            cell = next_cell<G>(p, g);
        }
        S.cell = -1;
    };

    acquire(blockIdx.x * groups + gib);

    unsigned iters = 0;
    for (;;) {
        if (!__any(S.cell >= 0)) break;   // a wave whose groups hold no cell issues nothing
        ++iters;
        {
            ParamsK &pr = *params_k();
            rhs_eval<G, NSL, RUC, PD>(z, S.P10, S.invP10, fz, L, ur, g, N, pr.RU, pr.NSEG, pr.SEGL,
                                      pr.L2P, pr.L2N, pr.RUp, pr.NMS, pr.RU2, pr.invTmax);
        }
        if (S.cell >= 0) {
            ParamsK &pk = *params_k();
            Counts c = S.c;
            c.n_rhs += 1;
            int act = ACT_NONE, fin = ST_OK;
            const int phase = S.phase;
            if (phase == PH_STAGE && S.tab) {
                // (E:rkcj) with the tabulated coefficients of (s, j)
                const int j = S.j;
                const double4 cf =
                    *reinterpret_cast<const double4 *>(pk.coef + 4 * (coef_offset(S.s) + j - 1));
                const double h = S.h;
                const double c0 = 1.0 - cf.x - cf.y, ch1 = cf.z * h, ch2 = cf.w * h;
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    const double wj = c0 * y[i] + cf.x * wm1[i] + cf.y * wm2[i] + ch1 * fz[i] +
                                      ch2 * f0[i];
                    wm2[i] = wm1[i];
                    wm1[i] = wj;
                    z[i] = wj;
                }
                if (j == S.s) S.phase = PH_ERR;
                else S.j = j + 1;
            } else if (phase == PH_STAGE) {
                // (E:rkcj) with the coefficient recurrences advanced one stage;
                // 1/b_{j-1} and 1/b_{j-2} are carried, so a stage needs two
                // divisions (b_j and 1/b_j)
                const double w0 = S.w0, Tm1 = S.Tm1, Tpm1 = S.Tpm1, Tppm1 = S.Tppm1, bm1 = S.bm1;
                const double ibm1 = S.ibm1;
                const double Tj = 2.0 * w0 * Tm1 - S.Tm2;
                const double Tpj = 2.0 * w0 * Tpm1 - S.Tpm2 + 2.0 * Tm1;
                const double Tppj = 2.0 * w0 * Tppm1 - S.Tppm2 + 4.0 * Tpm1;
                const double bj = Tppj / (Tpj * Tpj);
                const double mu = 2.0 * bj * w0 * ibm1;
                const double nu = -bj * S.ibm2;
                const double mut = 2.0 * bj * S.w1 * ibm1;
                const double gam = -(1.0 - bm1 * Tm1) * mut;
                const double h = S.h;
                const double c0 = 1.0 - mu - nu, ch1 = mut * h, ch2 = gam * h;
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    const double wj = c0 * y[i] + mu * wm1[i] + nu * wm2[i] + ch1 * fz[i] + ch2 * f0[i];
                    wm2[i] = wm1[i];
                    wm1[i] = wj;
                    z[i] = wj;
                }
                S.Tm2 = Tm1; S.Tm1 = Tj; S.Tpm2 = Tpm1; S.Tpm1 = Tpj; S.Tppm2 = Tppm1; S.Tppm1 = Tppj;
                S.bm1 = bj; S.ibm2 = ibm1; S.ibm1 = 1.0 / bj;
                const int j = S.j;
                if (j == S.s) S.phase = PH_ERR;
                else S.j = j + 1;
            } else if (phase == PH_ERR) {
                // error estimate, weighted RMS norm (E:rmsE) and step control
                const double h = S.h;
                double d[NSL];
#pragma unroll
                for (int i = 0; i < NSL; ++i)
                    d[i] = 0.8 * (y[i] - wm1[i]) + 0.4 * h * (f0[i] + fz[i]);
                // err = sqrt(e2) is only compared with 1 and raised to -1/3,
                // so the square root is not formed
                const double e2 = rms_norm2<G, NSL>(d, y, wm1, pk.rtol, pk.atol, g, N, pk.invN);
                if (e2 <= NORM2_ACCEPT) {
                    c.n_steps += 1;
#pragma unroll
                    for (int i = 0; i < NSL; ++i) { y[i] = wm1[i]; f0[i] = fz[i]; }
                    if (S.last) {
                        act = ACT_FINISH;
                        fin = ST_OK;
                    } else {
                        S.t = S.t + h;
                        const int ss = S.since_sigma + 1;
                        S.since_sigma = ss;
                        S.need_sigma = (ss >= 25);
                        // with r = err^(-1/3) and r_prev = err_prev^(-1/3) the
                        // predictive factor is 0.8 (h/h_prev) r^2 / r_prev; an
                        // err_prev of 0 is kept as r_prev = 0 (factor 0)
                        double fac, r = 0.0;
                        if (e2 == 0.0) {
                            fac = 10.0;
                        } else {
                            r = rsixth_pos(e2);
                            if (!S.predictive) fac = 0.8 * r;
                            else if (S.rprev == 0.0) fac = 0.0;
                            else fac = 0.8 * h * r * r * rcp_nr(S.h_prev * S.rprev);
                        }
                        if (fac > 10.0) fac = 10.0;
                        if (fac < 0.1) fac = 0.1;
                        S.h_prev = h;
                        S.rprev = r;
                        S.predictive = 1;
                        S.h = h * fac;
                        act = ACT_BEGIN_STEP;
                    }
                } else {
                    c.n_reject += 1;
                    double fac = isfinite(e2) ? 0.8 * rsixth_pos(e2) : 0.1;
                    if (fac < 0.1) fac = 0.1;
                    S.h = h * fac;
                    S.need_sigma = 1;
                    S.predictive = 0;
                    act = ACT_BEGIN_STEP;
                }
                if (act == ACT_BEGIN_STEP && S.h < h_min) { act = ACT_FINISH; fin = ST_UNDERFLOW; }
            } else if (phase == PH_POWER) {
                // nonlinear power method: one difference quotient per iteration
                c.n_piter += 1;
                double gv[NSL];
                double ng2 = 0.0, dz2 = 0.0;
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    gv[i] = fz[i] - f0[i];
                    const double dd = z[i] - y[i];
                    ng2 += gv[i] * gv[i];
                    dz2 += dd * dd;
                }
                gsum2<G>(ng2, dz2);
                const double ng = sqrt(ng2);
                double sig = ng / sqrt(dz2);
                const int k_pow = S.k_pow;
                bool stop = false;
                if (k_pow >= 2 && fabs(sig - S.sigma_prev) <= 0.01 * sig) stop = true;
                else if (ng == 0.0) { sig = 0.0; stop = true; }
                else if (k_pow == 50) stop = true;
                if (stop) {
#pragma unroll
                    for (int i = 0; i < NSL; ++i) v[i] = z[i] - y[i];
                    c.n_sigma += 1;
                    const double sigma = 1.2 * sig;
                    S.sigma = sigma;
                    if (!isfinite(sigma)) {
                        act = ACT_FINISH;
                        fin = ST_NONFINITE;
                    } else if (S.after == AFTER_INIT) {
                        // tentative initial step 1/sigma, capped at dt
                        double ht = (sigma > 0.0) ? 1.0 / sigma : t_end;
                        if (ht > t_end) ht = t_end;
                        S.ht = ht;
#pragma unroll
                        for (int i = 0; i < NSL; ++i) z[i] = y[i] + ht * f0[i];
                        S.phase = PH_INIT;
                    } else {
                        S.need_sigma = 0;
                        S.since_sigma = 0;
                        act = ACT_AFTER_SIGMA;
                    }
                } else {
                    const double q = S.delta / ng;
#pragma unroll
                    for (int i = 0; i < NSL; ++i) z[i] = y[i] + q * gv[i];
                    S.sigma_prev = sig;
                    S.k_pow = k_pow + 1;
                }
            } else if (phase == PH_INIT) {
                // initial step from the error of the tentative step
                const double ht = S.ht;
                double d[NSL];
#pragma unroll
                for (int i = 0; i < NSL; ++i) d[i] = ht * (fz[i] - f0[i]);
                const double e0 = sqrt(rms_norm2<G, NSL>(d, y, y, pk.rtol, pk.atol, g, N, pk.invN));
                if (!isfinite(e0)) {
                    act = ACT_FINISH;
                    fin = ST_NONFINITE;
                } else {
                    double h = (e0 > 0.0) ? 0.1 * ht / sqrt(e0) : ht;
                    if (h < h_min) h = h_min;
                    if (h > t_end) h = t_end;
                    S.h = h;
                    S.t = 0.0;
                    act = ACT_BEGIN_STEP;
                }
            } else {   // PH_F0: f(y0)
                int bad = 0;
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    f0[i] = fz[i];
                    bad |= (i * G + g < N) && !isfinite(fz[i]);
                }
                bad = gor<G>(bad);
                if (bad) {
                    act = ACT_FINISH;
                    fin = ST_NONFINITE;
                } else {
#pragma unroll
                    for (int i = 0; i < NSL; ++i) v[i] = f0[i];
                    act = ACT_POWER_INIT;
                }
            }

            if (act == ACT_BEGIN_STEP) {
                if (c.n_steps + c.n_reject >= pk.max_steps) { act = ACT_FINISH; fin = ST_MAXSTEPS; }
                else if (S.need_sigma) act = ACT_POWER_STEP;
                else act = ACT_AFTER_SIGMA;
            }
            if (act == ACT_POWER_INIT || act == ACT_POWER_STEP) {
                double ny2 = 0.0, nv2 = 0.0;
#pragma unroll
                for (int i = 0; i < NSL; ++i) { ny2 += y[i] * y[i]; nv2 += v[i] * v[i]; }
                gsum2<G>(ny2, nv2);
                const double ny = sqrt(ny2);
                const double delta = (ny > 0.0) ? sqrt_u * ny : sqrt_u;
                double nv = sqrt(nv2);
                if (!(nv > 0.0)) {
                    double o2 = 0.0;
#pragma unroll
                    for (int i = 0; i < NSL; ++i) {
                        v[i] = (i * G + g < N) ? 1.0 : 0.0;
                        o2 += v[i] * v[i];
                    }
                    nv = sqrt(gsum<G>(o2));
                }
                const double q = delta / nv;
#pragma unroll
                for (int i = 0; i < NSL; ++i) z[i] = y[i] + q * v[i];
                S.delta = delta;
                S.k_pow = 1;
                S.sigma_prev = 0.0;
                S.after = (act == ACT_POWER_INIT) ? AFTER_INIT : AFTER_STEP;
                S.phase = PH_POWER;
            } else if (act == ACT_AFTER_SIGMA) {
                // stage count from the spectral radius, then the first stage (E:rkc1)
                const double sigma = S.sigma, t = S.t;
                double h = S.h;
                int last = (h >= t_end - t);
                if (last) h = t_end - t;
                const double sq = floor(sqrt(1.0 + 1.54 * h * sigma));
                int s;
                if (1.0 + sq > (double)pk.s_max) {
                    s = pk.s_max;
                    h = ((double)(pk.s_max - 1) * (double)(pk.s_max - 1) - 1.0) / (1.54 * sigma);
                    last = 0;
                } else {
                    s = 1 + (int)sq;
                }
                c.s_hash = (int)((unsigned)c.s_hash * 31u + (unsigned)s);
                c.s_max_used = max(c.s_max_used, s);
                double mu_t1;
                if (s <= pk.coef_smax) {
                    mu_t1 = pk.coef[4 * coef_offset(s)];
                    S.tab = 1;
                } else {
                    // Chebyshev values at w0 = 1 + kappa/s^2 up to degree s, for
                    // w1 = T'_s/T''_s; the stages then advance the recurrences
                    S.tab = 0;
                    const double w0 = 1.0 + KAPPA / ((double)s * (double)s);
                    double T0 = 1.0, T1 = w0, P0 = 0.0, P1 = 1.0, Q0 = 0.0, Q1 = 0.0;
                    double P2 = 0.0, Q2 = 0.0;
                    for (int jj = 2; jj <= s; ++jj) {
                        const double Tn = 2.0 * w0 * T1 - T0;
                        const double Pn = 2.0 * w0 * P1 - P0 + 2.0 * T1;
                        const double Qn = 2.0 * w0 * Q1 - Q0 + 4.0 * P1;
                        if (jj == 2) { P2 = Pn; Q2 = Qn; }
                        T0 = T1; T1 = Tn; P0 = P1; P1 = Pn; Q0 = Q1; Q1 = Qn;
                    }
                    const double w1 = P1 / Q1;
                    const double b1 = 1.0 / w0;
                    const double b2 = Q2 / (P2 * P2);
                    S.w0 = w0; S.w1 = w1;
                    S.Tm1 = w0; S.Tm2 = 1.0; S.Tpm1 = 1.0; S.Tpm2 = 0.0; S.Tppm1 = 0.0;
                    S.Tppm2 = 0.0;
                    S.bm1 = b1; S.ibm1 = w0; S.ibm2 = 1.0 / b2;   // b_1 = 1/w0, b_0 = b_2
                    mu_t1 = b1 * w1;
                }
                S.h = h; S.last = last; S.s = s; S.j = 2;
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    wm2[i] = y[i];
                    wm1[i] = y[i] + mu_t1 * h * f0[i];
                    z[i] = wm1[i];
                }
                S.phase = PH_STAGE;
            }
            S.c = c;
            if (act == ACT_FINISH) {
                store_state<G, NSL>(p, S.cell, g, y);
                store_counts(p, S.cell, g, c, fin);
                agg_cell(S.agg, c, fin);
                acquire(next_cell<G>(p, g));
            }
        }
    }
    flush_agg(p, S.agg, g == 0, (unsigned long long)iters * (64 / G));
}

// ------------------------------------------------------------------ RKCK

// Table 1 (Sec. 2.3): Cash-Karp coefficients.
#define CK_B21 (1.0 / 5.0)
#define CK_B31 (3.0 / 40.0)
#define CK_B32 (9.0 / 40.0)
#define CK_B41 (3.0 / 10.0)
#define CK_B42 (-9.0 / 10.0)
#define CK_B43 (6.0 / 5.0)
#define CK_B51 (-11.0 / 54.0)
#define CK_B52 (5.0 / 2.0)
#define CK_B53 (-70.0 / 27.0)
#define CK_B54 (35.0 / 27.0)
#define CK_B61 (1631.0 / 55296.0)
#define CK_B62 (175.0 / 512.0)
#define CK_B63 (575.0 / 13824.0)
#define CK_B64 (44275.0 / 110592.0)
#define CK_B65 (253.0 / 4096.0)
#define CK_C1 (37.0 / 378.0)
#define CK_C3 (250.0 / 621.0)
#define CK_C4 (125.0 / 594.0)
#define CK_C6 (512.0 / 1771.0)
#define CK_D1 (37.0 / 378.0 - 2825.0 / 27648.0)
#define CK_D3 (250.0 / 621.0 - 18575.0 / 48384.0)
#define CK_D4 (125.0 / 594.0 - 13525.0 / 55296.0)
#define CK_D5 (0.0 - 277.0 / 14336.0)
#define CK_D6 (512.0 / 1771.0 - 1.0 / 4.0)

struct RkckState {
    double t, h, P10, invP10;
    int cell, phase, last;
    Counts c;
    Agg agg;
};
static_assert(sizeof(RkckState) <= STATE_BYTES, "RKCK state exceeds its LDS slot");

template <int G, int NSL, int RUC, bool PD>
__global__ __launch_bounds__((Occ<RUC, NSL>::threads), (Occ<RUC, NSL>::waves)) void rkck_kernel(Params p) {
    RKC_KERNEL_PROLOGUE
    RkckState &S = *reinterpret_cast<RkckState *>(lp.states + (size_t)gib * STATE_BYTES);

    double y[NSL], k1[NSL], k2[NSL], k3[NSL], k4[NSL], k5[NSL], z[NSL], fz[NSL];
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
        y[i] = k1[i] = k2[i] = k3[i] = k4[i] = k5[i] = fz[i] = 0.0;
        z[i] = (i == 0 && g == 0) ? 1000.0 : 0.0;
    }
    S.P10 = 1e6;
    S.agg = Agg{0, 0, 0, 0, 0, 0, 0, 0};
    S.invP10 = 1e-6;

    auto acquire = [&](int first) {
        int cell = first;
        while (cell < p.n_cells) {
            double P10;
            if (load_state<G, NSL>(p, cell, g, y, P10)) {
                S.cell = cell;
                S.P10 = P10;
                S.invP10 = 1.0 / P10;
                S.c = Counts{0, 0, 0, 0, 0, 0, 0};
                S.t = 0.0;
                // first trial step is the whole interval; the last step lands on dt
                S.h = t_end;
                S.last = 1;
#pragma unroll
                for (int i = 0; i < NSL; ++i) z[i] = y[i];
                S.phase = CK_K1;
                return;
            }
            Counts zc{0, 0, 0, 0, 0, 0, 0};
            store_counts(p, cell, g, zc, ST_BADINPUT);
            agg_cell(S.agg, zc, ST_BADINPUT);
            cell = next_cell<G>(p, g);
        }
        S.cell = -1;
    };

    acquire(blockIdx.x * groups + gib);

    unsigned iters = 0;
    for (;;) {
        if (!__any(S.cell >= 0)) break;   // a wave whose groups hold no cell issues nothing
        ++iters;
        rhs_eval<G, NSL, RUC, PD>(z, S.P10, S.invP10, fz, L, ur, g, N, p.RU, p.NSEG, p.SEGL,
                                  p.L2P, p.L2N, p.RUp, p.NMS, p.RU2, p.invTmax);
        if (S.cell >= 0) {
            Counts c = S.c;
            c.n_rhs += 1;
            const double h = S.h;
            int fin = -1;
            switch (S.phase) {
            case CK_K1:
#pragma unroll
                for (int i = 0; i < NSL; ++i) { k1[i] = h * fz[i]; z[i] = y[i] + CK_B21 * k1[i]; }
                S.phase = CK_K2;
                break;
            case CK_K2:
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    k2[i] = h * fz[i];
                    z[i] = y[i] + CK_B31 * k1[i] + CK_B32 * k2[i];
                }
                S.phase = CK_K3;
                break;
            case CK_K3:
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    k3[i] = h * fz[i];
                    z[i] = y[i] + CK_B41 * k1[i] + CK_B42 * k2[i] + CK_B43 * k3[i];
                }
                S.phase = CK_K4;
                break;
            case CK_K4:
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    k4[i] = h * fz[i];
                    z[i] = y[i] + CK_B51 * k1[i] + CK_B52 * k2[i] + CK_B53 * k3[i] + CK_B54 * k4[i];
                }
                S.phase = CK_K5;
                break;
            case CK_K5:
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    k5[i] = h * fz[i];
                    z[i] = y[i] + CK_B61 * k1[i] + CK_B62 * k2[i] + CK_B63 * k3[i]
                         + CK_B64 * k4[i] + CK_B65 * k5[i];
                }
                S.phase = CK_K6;
                break;
            default: {   // CK_K6: embedded error estimate and step control (E:hnew)
                double y5[NSL];
                double emax = 0.0;
                int bad = 0;
#pragma unroll
                for (int i = 0; i < NSL; ++i) {
                    const double k6 = h * fz[i];
                    y5[i] = y[i] + CK_C1 * k1[i] + CK_C3 * k3[i] + CK_C4 * k4[i] + CK_C6 * k6;
                    const double del = CK_D1 * k1[i] + 0.0 * k2[i] + CK_D3 * k3[i] + CK_D4 * k4[i]
                                     + CK_D5 * k5[i] + CK_D6 * k6;
                    if (i * G + g < N) {
                        const double d0 = p.rtol * (fabs(y[i]) + fabs(k1[i]) + 1e-30);
                        const double r = fabs(del / d0);
                        if (!isfinite(r)) bad = 1;
                        else emax = fmax(emax, r);
                    }
                }
                emax = gmax<G>(emax);
                bad = gor<G>(bad);
                const double errmax = bad ? __builtin_inf() : emax;
                double hn = h;
                if (errmax <= 1.0) {
                    c.n_steps += 1;
#pragma unroll
                    for (int i = 0; i < NSL; ++i) y[i] = y5[i];
                    if (S.last) {
                        fin = ST_OK;
                    } else {
                        S.t = S.t + h;
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
                if (fin < 0) {
                    if (hn < h_min) fin = ST_UNDERFLOW;
                    else if (c.n_steps + c.n_reject >= p.max_steps) fin = ST_MAXSTEPS;
                    else {
                        const double t = S.t;
                        const int last = (hn >= t_end - t);
                        if (last) hn = t_end - t;
                        S.last = last;
                        S.h = hn;
#pragma unroll
                        for (int i = 0; i < NSL; ++i) z[i] = y[i];
                        S.phase = CK_K1;
                    }
                }
            }
            }
            S.c = c;
            if (fin >= 0) {
                store_state<G, NSL>(p, S.cell, g, y);
                store_counts(p, S.cell, g, c, fin);
                agg_cell(S.agg, c, fin);
                acquire(next_cell<G>(p, g));
            }
        }
    }
    flush_agg(p, S.agg, g == 0, (unsigned long long)iters * (64 / G));
}

}  // namespace rkcdev
