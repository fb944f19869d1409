// Host runtime of the C ABI declared in include/rkc.h: mechanism packing and
// upload, variant selection, launch configuration and host<->device staging.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "rkc.h"
#include "rkc_internal.h"
#include "rkc_lane.h"

using rkcdev::NFIELD;
using rkcdev::UNIT_DOUBLES;

namespace {

constexpr double R_J = 8.31446261815324;   // J/(mol K)
using rkchost::AGG_N;
constexpr double L2A_ZERO = -1e4;          // log2 A of a reaction whose rate is identically 0
constexpr double TROE_BOUND = 1e10;        // largest log2(e)/T***, log2(e)/T* and T** log2(e)
                                           // passed to the kernels
constexpr long double LOG2E_L = 1.442695040888963407359924681001892137L;

// Device tables that depend on the lane-group shape: the species table is
// laid out with stride NK, the gather is balanced over G lanes.
struct NkTables {
    int G = 0, NK = 0, RU = 0, NSEG = 0, SEGL = 0, L2P = 0, L2N = 0;
    int RUp = 0, NPR = 0, NMS = 0;   // pressure-dependent rounds and efficiency sets
    int RU2 = 0;                     // rounds [0, RU2) of units with two slots a side
    double *spec = nullptr;
    uint32_t *gather = nullptr;
    uint32_t *gather2 = nullptr;
    double *units_il = nullptr;      // [RU + 1][4][G] double2, for the RUC = -1 kernels
    double *pdep = nullptr;          // [NPR * G][12], lane-interleaved
    double *eff = nullptr;           // [NMS][NK]
};

}  // namespace

struct rkc_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long *agg_d = nullptr;
    int *queue_d = nullptr;
};

struct rkc_mech {
    int device = 0;
    int nS = 0, nR = 0, N = 0, nU = 0, nU_pad = 0, nnz = 0, max_row = 0;
    std::vector<double> units_h;                       // [nU_pad][8]
    int n_plain = 0, n_pdep = 0;                       // units [0, n_plain) plain, then pdep
    int n_two = 0;   // units [0, n_two) plain with at most two reactant slots per side
    double invTmax = 0.0;   // bound on 1/T in the Arrhenius factors (see rkc_mech_create)
    std::vector<double> pdep_h;                        // [n_pdep][PDEP_DOUBLES]
    std::vector<std::vector<double>> effsets;          // distinct efficiency vectors [nS]
    double *pdep_d = nullptr;
    std::vector<double> W, lo, hi, Tmid;               // species data
    std::vector<std::vector<std::pair<int, int>>> rows;  // species -> (unit, dnu)
    double *units_d = nullptr;
    std::vector<NkTables> nk;
    unsigned long long *agg_d = nullptr;               // [AGG_N]
    double *coef_d = nullptr;                          // RKC stage coefficient table
    int *queue_d = nullptr;
    void *stage_d = nullptr;
    size_t stage_bytes = 0;
    int num_cus = 0;
    size_t max_lds = 0;
    // tables of the one-lane-per-cell kernels (built on first use)
    double *l_spec_d = nullptr;        // [nS][LS_FIELDS]
    double *l_units_d = nullptr;       // [nU][LU_DOUBLES]
    double *l_eff_d = nullptr;         // [NMS][nS]
    // rkc_autotune results by (method, requested lanes and placement, layout,
    // log2 of the cell count)
    struct Tuned {
        int method, lanes, placement, layout, log2n;
        rkc_opts opts;
        float ms;
    };
    std::vector<Tuned> tuned;
};

namespace {

int count_in(const int32_t *slots, int sp) {
    int c = 0;
    for (int s = 0; s < 3; ++s) c += (slots[s] == sp);
    return c;
}

bool same_multiset(const int32_t *a, const int32_t *b) {
    int x[3], y[3];
    for (int s = 0; s < 3; ++s) { x[s] = a[s]; y[s] = b[s]; }
    std::sort(x, x + 3);
    std::sort(y, y + 3);
    return x[0] == y[0] && x[1] == y[1] && x[2] == y[2];
}

// Three reactant slots as 16-bit byte offsets into the concentration array;
// an empty slot points at index n_species (which holds 1.0).
uint64_t pack_slots(const int32_t *slots, int nS) {
    uint64_t v = 0;
    for (int s = 0; s < 3; ++s) {
        const uint64_t id = slots[s] >= 0 ? (uint64_t)slots[s] : (uint64_t)nS;
        v |= (id * 8u) << (16 * s);
    }
    return v;
}

// The kernels evaluate rate constants in base 2 (2^(log2 A + beta log2 T -
// theta'/T)): log2 A and theta' = (Ea/R) log2(e), each rounded once.
double l2_a(double A) { return A > 0.0 ? (double)std::log2((long double)A) : L2A_ZERO; }
double theta2(double Ea) { return (double)((long double)Ea / (long double)R_J * LOG2E_L); }

// Stage counts whose RKC coefficients are tabulated (larger ones are computed
// by the kernels' recurrences).
constexpr int COEF_SMAX = 128;

// The coefficient table described at rkcdev::coef_offset, for s = 2..COEF_SMAX
// (Sec. 2.4: Chebyshev values at w0 = 1 + kappa/s^2 by their recurrences,
// b_j = T''_j / T'_j^2 for j >= 2, b_1 = 1/w0, b_0 = b_2, a_j = 1 - b_j T_j).
std::vector<double> coef_table() {
    std::vector<double> t(4 * (size_t)rkcdev::coef_offset(COEF_SMAX + 1), 0.0);
    for (int s = 2; s <= COEF_SMAX; ++s) {
        const double w0 = 1.0 + rkcdev::KAPPA / ((double)s * (double)s);
        std::vector<double> T(s + 1), Tp(s + 1), Tpp(s + 1), b(s + 1);
        T[0] = 1.0; T[1] = w0; Tp[0] = 0.0; Tp[1] = 1.0; Tpp[0] = 0.0; Tpp[1] = 0.0;
        for (int j = 2; j <= s; ++j) {
            T[j] = 2.0 * w0 * T[j - 1] - T[j - 2];
            Tp[j] = 2.0 * w0 * Tp[j - 1] - Tp[j - 2] + 2.0 * T[j - 1];
            Tpp[j] = 2.0 * w0 * Tpp[j - 1] - Tpp[j - 2] + 4.0 * Tp[j - 1];
        }
        const double w1 = Tp[s] / Tpp[s];
        for (int j = 2; j <= s; ++j) b[j] = Tpp[j] / (Tp[j] * Tp[j]);
        b[1] = 1.0 / w0;
        b[0] = b[2];
        double *e = &t[4 * (size_t)rkcdev::coef_offset(s)];
        e[0] = b[1] * w1;
        for (int j = 2; j <= s; ++j) {
            double *q = e + 4 * (j - 1);
            q[0] = 2.0 * b[j] * w0 / b[j - 1];
            q[1] = -b[j] / b[j - 2];
            q[2] = 2.0 * b[j] * w1 / b[j - 1];
            q[3] = -(1.0 - b[j - 1] * T[j - 1]) * q[2];
        }
    }
    return t;
}

// A failed HIP call returns RKC_EDEVICE; with RKC_DEBUG set in the
// environment it is also reported on stderr. The runtime's per-thread last
// error is cleared, so that a failure reported here is not reported a second
// time by the caller's own next error check.
bool hip_failed(hipError_t e, const char *what, int line) {
    if (e == hipSuccess) return false;
    (void)hipGetLastError();
    if (std::getenv("RKC_DEBUG"))
        std::fprintf(stderr, "rkc: %s failed at rkc_host.hip:%d: %s\n", what, line,
                     hipGetErrorString(e));
    return true;
}

#define HIP_OK(expr)                                                    \
    do {                                                                \
        if (hip_failed((expr), #expr, __LINE__)) return RKC_EDEVICE;    \
    } while (0)

// Makes a device current for the length of one call and gives the caller's
// current device back when the call returns, whatever the return path.
struct DeviceScope {
    int prev = 0;
    bool switched = false;
    hipError_t enter(int dev) {
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess || prev == dev) return e;
        e = hipSetDevice(dev);
        switched = e == hipSuccess;
        return e;
    }
    ~DeviceScope() {
        if (switched) (void)hipSetDevice(prev);
    }
};

// Balanced gather for the net production sum (E:spec-rate), in two levels.
// Level 1: each species' terms (byte offsets of the units' net rates q,
// repeated |nu'' - nu'| times), split into positive and negative coefficients,
// are cut into chunks of at most SEGL terms; chunk c (species-major, positive
// before negative) runs in lane c % G, segment c / G, and its sum is piece c.
// Level 2: the lane that owns state index k adds the pieces of species k,
// L2P positive slots and L2N negative ones (byte offsets into the piece array,
// padded with its zero slot), and takes the difference.  Both levels have the
// same shape in every lane.  SEGL is chosen to minimise the vector
// instructions of both levels, about NSEG (2 SEGL + 1) + NSL (2 (L2P + L2N) + 1),
// among the lengths the kernels unroll (SEGL <= 12; piece counts above 8 take
// a loop and are charged three times as much).
struct GatherPlan {
    int NSEG = 1, SEGL = 2, L2P = 2, L2N = 2;
    std::vector<uint32_t> words;    // [NSEG * SEGL / 2][G]
    std::vector<uint32_t> words2;   // [NSL * (L2P + L2N) / 2][G]
};

// Order the terms inside each chunk so that at every position the lanes of a
// 16-lane LDS pass read distinct banks where they can: a double at byte offset
// o uses the bank pair (o / 8) mod 32, and lanes reading the same address are
// served together.  Greedy per pass: each lane takes, among its remaining
// terms, one whose bank pair is free or already holds that very address, else
// the least loaded one.  Only the order of a chunk's sum changes (rounding).
void order_for_banks(std::vector<uint32_t> *cellp, int NSEG, int G, int L) {
    std::vector<uint32_t> &cell = *cellp;
    const int PASS = std::min(16, G);
    for (int sg = 0; sg < NSEG; ++sg) {
        std::vector<std::vector<uint32_t>> left(G);
        for (int g = 0; g < G; ++g)
            left[g].assign(cell.begin() + ((size_t)sg * G + g) * L,
                           cell.begin() + ((size_t)sg * G + g + 1) * L);
        for (int e = 0; e < L; ++e) {
            for (int p0 = 0; p0 < G; p0 += PASS) {
                std::vector<std::vector<uint32_t>> bank(32);
                for (int g = p0; g < p0 + PASS; ++g) {
                    size_t best = 0, best_cost = (size_t)-1;
                    for (size_t k = 0; k < left[g].size(); ++k) {
                        const uint32_t a = left[g][k];
                        const std::vector<uint32_t> &u = bank[(a / 8) % 32];
                        const bool same = std::find(u.begin(), u.end(), a) != u.end();
                        const size_t cost = (u.empty() || same) ? 0 : u.size();
                        if (cost < best_cost) { best_cost = cost; best = k; }
                    }
                    const uint32_t a = left[g][best];
                    left[g].erase(left[g].begin() + (long)best);
                    std::vector<uint32_t> &u = bank[(a / 8) % 32];
                    if (std::find(u.begin(), u.end(), a) == u.end()) u.push_back(a);
                    cell[((size_t)sg * G + g) * L + e] = a;
                }
            }
        }
    }
}

int plan_gather(const rkc_mech *m, int G, int NK, int RU, GatherPlan *gp) {
    const int RUG = RU * G;
    if ((size_t)(RUG + 1) * 8 > rkcdev::TERM_MAX_BYTES) return RKC_ENOTSUP;
    const uint32_t zero_term = (uint32_t)(RUG * 8);
    const int NSL = NK / G;
    // lists[2 i] positive terms of species i, lists[2 i + 1] negative terms
    std::vector<std::vector<uint32_t>> lists(2 * (size_t)m->nS);
    int max_row = 0;
    for (int i = 0; i < m->nS; ++i) {
        for (const auto &pr : m->rows[i]) {
            const uint32_t off = (uint32_t)(pr.first * 8);
            std::vector<uint32_t> &dst = lists[2 * i + (pr.second < 0 ? 1 : 0)];
            for (int r = 0; r < std::abs(pr.second); ++r) dst.push_back(off);
        }
        max_row = std::max(max_row, (int)std::max(lists[2 * i].size(), lists[2 * i + 1].size()));
    }
    auto even = [](long v) { return std::max(2L, v + (v & 1)); };
    long best = -1;
    for (int L = 2; L <= std::min(12, std::max(2, max_row + (max_row & 1))); L += 2) {
        long chunks = 0, pp = 0, pn = 0;
        for (int i = 0; i < m->nS; ++i) {
            const long a = ((long)lists[2 * i].size() + L - 1) / L;
            const long b = ((long)lists[2 * i + 1].size() + L - 1) / L;
            chunks += a + b;
            pp = std::max(pp, a);
            pn = std::max(pn, b);
        }
        const long nseg = std::max(1L, (chunks + G - 1) / G);
        if ((nseg * G + 1) * 8 > (long)rkcdev::TERM_MAX_BYTES) continue;
        const long l2 = even(pp) + even(pn);
        const long cost =
            nseg * (2L * L + 1) + (long)NSL * (2 * l2 + 1) * (even(pp) > 8 || even(pn) > 8 ? 3 : 1);
        if (best < 0 || cost < best) {
            best = cost;
            gp->SEGL = L;
            gp->NSEG = (int)nseg;
            gp->L2P = (int)even(pp);
            gp->L2N = (int)even(pn);
        }
    }
    if (best < 0) return RKC_ENOTSUP;
    const int L = gp->SEGL;
    const int half = L / 2;
    const uint32_t zero_piece = (uint32_t)(gp->NSEG * G * 8);
    const int H2 = (gp->L2P + gp->L2N) / 2;
    // level-2 slots of state index k: [0, L2P) positive pieces, then negative
    std::vector<uint32_t> slot((size_t)NK * 2 * H2, zero_piece);
    // terms of chunk (segment sg, lane g) at cell[(sg G + g) L + e], zero-padded
    std::vector<uint32_t> cell((size_t)gp->NSEG * G * L, zero_term);
    int c = 0;
    for (int k = 1; k <= m->nS; ++k) {
        for (int sign = 0; sign < 2; ++sign) {
            const std::vector<uint32_t> &t = lists[2 * (k - 1) + sign];
            int n = 0;
            for (size_t b = 0; b < t.size(); b += L, ++c, ++n) {
                const int g = c % G, sg = c / G;
                for (int e = 0; e < L && b + e < t.size(); ++e)
                    cell[((size_t)sg * G + g) * L + e] = t[b + e];
                slot[(size_t)k * 2 * H2 + (sign ? gp->L2P : 0) + n] = (uint32_t)(c * 8);
            }
        }
    }
    if (c > gp->NSEG * G) return RKC_ENOTSUP;   // cannot happen by construction
    order_for_banks(&cell, gp->NSEG, G, L);
    gp->words.assign((size_t)gp->NSEG * half * G, 0u);
    for (int sg = 0; sg < gp->NSEG; ++sg)
        for (int g = 0; g < G; ++g)
            for (int e = 0; e < L; ++e) {
                const uint32_t term = cell[((size_t)sg * G + g) * L + e];
                uint32_t &w = gp->words[(size_t)(sg * half + e / 2) * G + g];
                w = (e % 2) ? ((w & 0xffffu) | (term << 16)) : ((w & 0xffff0000u) | term);
            }
    gp->words2.assign((size_t)NSL * H2 * G, 0u);
    for (int k = 0; k < NK; ++k) {
        const int s = k / G, g = k % G;
        for (int e = 0; e < 2 * H2; e += 2)
            gp->words2[(size_t)(s * H2 + e / 2) * G + g] =
                slot[(size_t)k * 2 * H2 + e] | (slot[(size_t)k * 2 * H2 + e + 1] << 16);
    }
    return RKC_OK;
}

int ensure_tables(rkc_mech *m, int G, int NK, int RU, NkTables **out, bool may_build = true) {
    for (auto &t : m->nk)
        if (t.NK == NK && t.G == G) { *out = &t; return RKC_OK; }
    if (!may_build) return RKC_ENOTSUP;
    const int nS = m->nS;
    std::vector<double> spec((size_t)NFIELD * NK, 0.0);
    for (int i = 0; i < nS; ++i) {
        const int k = i + 1;
        auto put = [&](int f, double v) { spec[(size_t)f * NK + k] = v; };
        put(rkcdev::F_W, m->W[i]);
        put(rkcdev::F_INVW, 1.0 / m->W[i]);
        put(rkcdev::F_TMID, m->Tmid[i]);
        const double *a[2] = {&m->lo[7 * i], &m->hi[7 * i]};
        const int cpo[2] = {rkcdev::F_CPLO, rkcdev::F_CPHI};
        const int ho[2] = {rkcdev::F_HLO, rkcdev::F_HHI};
        for (int r = 0; r < 2; ++r) {
            for (int q = 0; q < 5; ++q) put(cpo[r] + q, a[r][q]);
            put(ho[r] + 0, a[r][0]);
            put(ho[r] + 1, a[r][1] / 2.0);
            put(ho[r] + 2, a[r][2] / 3.0);
            put(ho[r] + 3, a[r][3] / 4.0);
            put(ho[r] + 4, a[r][4] / 5.0);
            put(ho[r] + 5, a[r][5]);
        }
    }
    GatherPlan gp;
    int rc = plan_gather(m, G, NK, RU, &gp);
    if (rc) return rc;
    NkTables t;
    t.G = G;
    t.NK = NK;
    t.RU = RU;
    t.NSEG = gp.NSEG;
    t.SEGL = gp.SEGL;
    t.L2P = gp.L2P;
    t.L2N = gp.L2N;
    // rounds from RUp on hold the pressure-dependent units (plain ones first)
    t.NMS = (int)m->effsets.size();
    t.RUp = m->n_pdep > 0 ? m->n_plain / G : RU;
    t.NPR = RU - t.RUp;
    t.RU2 = std::min(m->n_two / G, t.RUp);
    std::vector<double> pd((size_t)t.NPR * G * rkcdev::PDEP_DOUBLES, 0.0);
    for (int l = 0; l < t.NPR * G; ++l) {
        const int unit = t.RUp * G + l;
        if (unit < m->n_plain || unit >= m->nU) continue;
        const double *src = &m->pdep_h[(size_t)(unit - m->n_plain) * rkcdev::PDEP_DOUBLES];
        const int r = l / G, g = l % G;
        for (int q = 0; q < rkcdev::PDEP_DOUBLES / 2; ++q) {
            const size_t at = ((size_t)(r * (rkcdev::PDEP_DOUBLES / 2) + q) * G + g) * 2;
            pd[at] = src[2 * q];
            pd[at + 1] = src[2 * q + 1];
        }
    }
    std::vector<double> ef((size_t)t.NMS * NK, 0.0);
    for (int q = 0; q < t.NMS; ++q)
        for (int i = 0; i < nS; ++i) ef[(size_t)q * NK + i + 1] = m->effsets[q][i];
    if (!pd.empty() && hipMalloc(&t.pdep, pd.size() * 8) != hipSuccess) return RKC_ENOMEM;
    if (!ef.empty() && hipMalloc(&t.eff, ef.size() * 8) != hipSuccess) return RKC_ENOMEM;
    if (!pd.empty()) HIP_OK(hipMemcpy(t.pdep, pd.data(), pd.size() * 8, hipMemcpyHostToDevice));
    if (!ef.empty()) HIP_OK(hipMemcpy(t.eff, ef.data(), ef.size() * 8, hipMemcpyHostToDevice));
    if (hipMalloc(&t.spec, spec.size() * 8) != hipSuccess) return RKC_ENOMEM;
    if (hipMalloc(&t.gather, gp.words.size() * 4) != hipSuccess ||
        hipMalloc(&t.gather2, gp.words2.size() * 4) != hipSuccess) {
        (void)hipFree(t.spec); (void)hipFree(t.gather);
        return RKC_ENOMEM;
    }
    HIP_OK(hipMemcpy(t.spec, spec.data(), spec.size() * 8, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(t.gather, gp.words.data(), gp.words.size() * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(t.gather2, gp.words2.data(), gp.words2.size() * 4, hipMemcpyHostToDevice));
    {
        // unit records lane-interleaved in 16-byte pieces (piece q of unit
        // rG + g at double2 (4r + q)G + g), plus one zero round that the
        // kernels' one-round-ahead read of the reactant slots may touch
        std::vector<double> il((size_t)(RU + 1) * G * UNIT_DOUBLES, 0.0);
        for (int u = 0; u < RU * G && u < m->nU_pad; ++u) {
            const int r = u / G, g = u % G;
            for (int q = 0; q < UNIT_DOUBLES / 2; ++q) {
                const size_t at = ((size_t)(4 * r + q) * G + g) * 2;
                il[at] = m->units_h[(size_t)u * UNIT_DOUBLES + 2 * q];
                il[at + 1] = m->units_h[(size_t)u * UNIT_DOUBLES + 2 * q + 1];
            }
        }
        if (hipMalloc(&t.units_il, il.size() * 8) != hipSuccess) return RKC_ENOMEM;
        HIP_OK(hipMemcpy(t.units_il, il.data(), il.size() * 8, hipMemcpyHostToDevice));
    }
    m->nk.push_back(t);
    *out = &m->nk.back();
    return RKC_OK;
}

// Tables of the one-lane-per-cell kernels (rkc_lane.h): species records of
// LS_FIELDS doubles (W, 1/W, T_mid, the Horner coefficients of Cp/R and H/(RT)
// per range), and unit records of LU_DOUBLES doubles: the lane-group record
// followed by the unit's net-production terms (LDS rows of the species'
// production rates in 16-bit fields, unused slots naming the discard row,
// then nu'' - nu' of each as a double, 0 for unused slots), in species order.
int ensure_lane_tables(rkc_mech *m, bool may_build = true) {
    if (m->l_spec_d) return RKC_OK;
    if (!may_build) return RKC_ENOTSUP;
    const int nS = m->nS, nU = m->nU;
    std::vector<double> spec((size_t)nS * rkcdev::LS_FIELDS, 0.0);
    for (int i = 0; i < nS; ++i) {
        double *r = &spec[(size_t)i * rkcdev::LS_FIELDS];
        r[rkcdev::LS_W] = m->W[i];
        r[rkcdev::LS_INVW] = 1.0 / m->W[i];
        r[rkcdev::LS_TMID] = m->Tmid[i];
        const double *a[2] = {&m->lo[7 * i], &m->hi[7 * i]};
        const int cpo[2] = {rkcdev::LS_CPLO, rkcdev::LS_CPHI};
        const int ho[2] = {rkcdev::LS_HLO, rkcdev::LS_HHI};
        for (int q = 0; q < 2; ++q) {
            for (int c = 0; c < 5; ++c) r[cpo[q] + c] = a[q][c];
            r[ho[q] + 0] = a[q][0];
            r[ho[q] + 1] = a[q][1] / 2.0;
            r[ho[q] + 2] = a[q][2] / 3.0;
            r[ho[q] + 3] = a[q][3] / 4.0;
            r[ho[q] + 4] = a[q][4] / 5.0;
            r[ho[q] + 5] = a[q][5];
        }
    }
    // terms of each unit, in species order
    std::vector<std::vector<std::pair<int, int>>> terms(nU);
    for (int i = 0; i < nS; ++i)
        for (const auto &pr : m->rows[i]) terms[pr.first].push_back({i, pr.second});
    std::vector<double> units((size_t)std::max(1, nU) * rkcdev::LU_DOUBLES, 0.0);
    for (int u = 0; u < nU; ++u) {
        if ((int)terms[u].size() > rkcdev::LU_TERMS) return RKC_ENOTSUP;   // cannot happen: <= 6 species
        double *r = &units[(size_t)u * rkcdev::LU_DOUBLES];
        std::memcpy(r, &m->units_h[(size_t)u * UNIT_DOUBLES], UNIT_DOUBLES * sizeof(double));
        uint64_t w[2] = {0, 0};
        for (int t = 0; t < rkcdev::LU_TERMS; ++t) {
            const bool used = t < (int)terms[u].size();
            const uint64_t row = used ? (uint64_t)(rkcdev::lane_row_omega(nS) + terms[u][t].first)
                                      : (uint64_t)rkcdev::lane_row_discard(nS);
            w[t / 4] |= row << (16 * (t % 4));
            r[10 + t] = used ? (double)terms[u][t].second : 0.0;
        }
        std::memcpy(&r[8], &w[0], 8);
        std::memcpy(&r[9], &w[1], 8);
    }
    const int NMS = (int)m->effsets.size();
    std::vector<double> eff((size_t)std::max(1, NMS) * nS, 0.0);
    for (int q = 0; q < NMS; ++q)
        for (int i = 0; i < nS; ++i) eff[(size_t)q * nS + i] = m->effsets[q][i];
    double *sp = nullptr, *ef = nullptr, *un = nullptr;
    if (hipMalloc(&sp, spec.size() * 8) != hipSuccess || hipMalloc(&ef, eff.size() * 8) != hipSuccess ||
        hipMalloc(&un, units.size() * 8) != hipSuccess) {
        (void)hipFree(sp); (void)hipFree(ef); (void)hipFree(un);
        return RKC_ENOMEM;
    }
    if (hipMemcpy(sp, spec.data(), spec.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ef, eff.data(), eff.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(un, units.data(), units.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(sp); (void)hipFree(ef); (void)hipFree(un);
        return RKC_EDEVICE;
    }
    m->l_spec_d = sp;
    m->l_eff_d = ef;
    m->l_units_d = un;
    return RKC_OK;
}

// LDS rows of 64 doubles one wave of a one-lane-per-cell kernel needs:
// concentrations, net production rates, third-body concentrations.
int lane_rows(const rkc_mech *m) {
    return rkcdev::lane_row_mset(m->nS) + (m->n_pdep > 0 ? (int)m->effsets.size() : 0);
}

struct Choice {
    rkchost::VariantDesc v;
    int RU;
};

const rkchost::VariantDesc *find_variant(int G, int NSL, int RUC) {
    int n = 0;
    const rkchost::VariantDesc *tab = nullptr;
    switch (G) {
    case 64: tab = rkchost::variants_g64(&n); break;
    case 32: tab = rkchost::variants_g32(&n); break;
    case 16: tab = rkchost::variants_g16(&n); break;
    case 8: tab = rkchost::variants_g8(&n); break;
    default: return nullptr;
    }
    for (int i = 0; i < n; ++i)
        if (tab[i].NSL == NSL && tab[i].RUC == RUC) return &tab[i];
    return nullptr;
}

// Automatic group size: 16 lanes up to 16 state elements, 32 up to 39, 64
// above.  A set with pressure-dependent units and at most 64 state elements
// keeps 32 lanes (two slots per lane, two cells per wave): the work that every
// lane repeats per cell (group reductions, third-body sums, step control) is
// then shared by two cells, which outweighs the lower occupancy of the
// two-slot kernels (53-species falloff set: 3.23 M against 2.79 M cell-ODEs/s
// at 64 lanes; without pressure-dependent units the two are level).
int choose_variant(const rkc_mech *m, int lanes, int placement, Choice *out) {
    if (lanes == 1) {
        // one lane per cell: the smallest state capacity that holds N
        int n = 0;
        const rkchost::VariantDesc *tab = rkchost::variants_lane(&n);
        const rkchost::VariantDesc *pick = nullptr;
        for (int i = 0; i < n; ++i)
            if (tab[i].NSL >= m->N && (!pick || tab[i].NSL < pick->NSL)) pick = &tab[i];
        if (!pick) return RKC_ENOTSUP;
        out->v = *pick;
        out->RU = m->nU;
        return RKC_OK;
    }
    int G = lanes;
    if (G == 0) {
        G = (m->N >= 40) ? 64 : (m->N > 16 ? 32 : 16);
        if (G == 64 && m->n_pdep > 0 && m->N <= 64) G = 32;
    }
    int n = 0;
    const rkchost::VariantDesc *tab = nullptr;
    switch (G) {
    case 64: tab = rkchost::variants_g64(&n); break;
    case 32: tab = rkchost::variants_g32(&n); break;
    case 16: tab = rkchost::variants_g16(&n); break;
    case 8: tab = rkchost::variants_g8(&n); break;
    default: return RKC_EINVAL;
    }
    const int nsl_need = (m->N + G - 1) / G;
    const int ru = std::max(1, (m->nU + G - 1) / G);
    int best_nsl = 1 << 30;
    for (int i = 0; i < n; ++i)
        if (tab[i].NSL >= nsl_need) best_nsl = std::min(best_nsl, tab[i].NSL);
    if (best_nsl == (1 << 30)) return RKC_ENOTSUP;
    const rkchost::VariantDesc *pick = nullptr;
    // register-resident parameters cover plain units only
    if (placement == RKC_PARAMS_REGISTERS && m->n_pdep == 0)
        for (int i = 0; i < n; ++i)
            if (tab[i].NSL == best_nsl && tab[i].RUC == ru) pick = &tab[i];
    if (!pick)
        for (int i = 0; i < n; ++i)
            if (tab[i].NSL == best_nsl && tab[i].RUC == 0) pick = &tab[i];
    if (!pick) return RKC_ENOTSUP;
    out->v = *pick;
    out->RU = ru;
    return RKC_OK;
}

rkcdev::Shape shape_for(const Choice &ch, const NkTables *nk) {
    return rkcdev::Shape{nk->NK, ch.RU, ch.v.G, nk->NSEG, nk->SEGL, nk->L2P + nk->L2N,
                         nk->NPR, nk->NMS, ch.v.RUC == 0, ch.v.RUC >= 0};
}

// choose_variant, the device tables of its shape, and the placement of the
// reaction parameters: automatic placement keeps them in LDS unless LDS then
// limits the workgroup below the variant's occupancy target and a variant
// reading them from global memory exists for the same shape.
int select_variant(rkc_mech *m, const rkc_opts &o, Choice *ch, NkTables **nk,
                   bool may_build = true) {
    int rc = choose_variant(m, o.lanes_per_cell, o.param_placement, ch);
    if (rc) return rc;
    if (ch->v.G == 1) {
        *nk = nullptr;
        return ensure_lane_tables(m, may_build);
    }
    rc = ensure_tables(m, ch->v.G, ch->v.NSL * ch->v.G, ch->RU, nk, may_build);
    if (rc) return rc;
    if (ch->v.RUC != 0 || o.param_placement == RKC_PARAMS_LDS) return RKC_OK;
    const rkchost::VariantDesc *glob = find_variant(ch->v.G, ch->v.NSL, -1);
    if (!glob) return o.param_placement == RKC_PARAMS_GLOBAL ? RKC_ENOTSUP : RKC_OK;
    bool use = o.param_placement == RKC_PARAMS_GLOBAL;
    if (!use) {
        const int want = std::max(1, ch->v.max_threads / ch->v.G);
        const rkcdev::Shape sh = shape_for(*ch, *nk);
        use = rkcdev::lds_bytes(sh, want) > m->max_lds;
    }
    if (use) ch->v = *glob;
    return RKC_OK;
}

int ensure_stage(rkc_mech *m, size_t bytes) {
    if (m->stage_bytes >= bytes) return RKC_OK;
    if (m->stage_d) (void)hipFree(m->stage_d);
    m->stage_d = nullptr;
    m->stage_bytes = 0;
    if (hipMalloc(&m->stage_d, bytes) != hipSuccess) return RKC_ENOMEM;
    m->stage_bytes = bytes;
    return RKC_OK;
}

__global__ void reset_scratch_kernel(unsigned long long *agg, int *queue) {
    if (threadIdx.x < AGG_N) agg[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) *queue = 0;
}

struct Launch {
    int threads, blocks, groups_per_block;
    size_t lds;
    bool persistent;
};

int plan_launch(const rkc_mech *m, const Choice &ch, const void *kernel, size_t n_cells,
                const rkc_opts &o, bool allow_persistent, NkTables *nk, Launch *L);

// One lane per cell: workgroups of up to 256 lanes (o.block_groups lanes,
// rounded up to whole waves), fewer waves when their LDS rows do not fit.
int plan_lane_launch(const rkc_mech *m, const Choice &ch, const void *kernel, size_t n_cells,
                     const rkc_opts &o, bool allow_persistent, Launch *L) {
    const size_t wave_bytes = (size_t)lane_rows(m) * rkcdev::LROW;
    int waves = o.block_groups > 0 ? (o.block_groups + 63) / 64 : 4;
    waves = std::min(waves, ch.v.max_threads / 64);
    while (waves > 1 && wave_bytes * (size_t)waves > m->max_lds) --waves;
    if (waves < 1 || wave_bytes * (size_t)waves > m->max_lds) return RKC_ENOTSUP;
    L->groups_per_block = waves * 64;
    L->threads = waves * 64;
    L->lds = wave_bytes * (size_t)waves;
    hipFuncAttributes fa{};
    HIP_OK(hipFuncGetAttributes(&fa, kernel));
    if (L->threads > fa.maxThreadsPerBlock) return RKC_ENOTSUP;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L->lds) !=
        hipSuccess)
        return RKC_EDEVICE;
    const size_t blocks_all = (n_cells + L->threads - 1) / L->threads;
    L->persistent = false;
    size_t blocks = blocks_all;
    if (allow_persistent && o.schedule != RKC_SCHED_PLAIN) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, L->threads, L->lds) !=
            hipSuccess)
            return RKC_EDEVICE;
        per_cu = std::max(1, per_cu);
        size_t resident = (size_t)per_cu * (size_t)m->num_cus;
        if (o.grid_blocks > 0) resident = (size_t)o.grid_blocks;
        if (o.schedule == RKC_SCHED_PERSISTENT || resident < blocks_all) {
            L->persistent = true;
            blocks = std::min(blocks_all, resident);
        }
    }
    if (blocks > 0x7fffffff) return RKC_ENOTSUP;
    L->blocks = (int)std::max<size_t>(1, blocks);
    return RKC_OK;
}

int plan_launch(const rkc_mech *m, const Choice &ch, const void *kernel, size_t n_cells,
                const rkc_opts &o, bool allow_persistent, NkTables *nk, Launch *L) {
    if (ch.v.G == 1) return plan_lane_launch(m, ch, kernel, n_cells, o, allow_persistent, L);
    const int G = ch.v.G;
    const int NK = nk->NK;
    const int max_threads = ch.v.max_threads;
    int gpb = o.block_groups > 0 ? o.block_groups : std::max(1, max_threads / G);
    if (gpb * G > max_threads) gpb = max_threads / G;
    const rkcdev::Shape sh = shape_for(ch, nk);
    auto need = [&](int groups) { return rkcdev::lds_bytes(sh, groups); };
    while (gpb > 1 && need(gpb) > m->max_lds) --gpb;
    if (need(gpb) > m->max_lds) return RKC_ENOTSUP;
    L->groups_per_block = gpb;
    L->threads = gpb * G;
    L->lds = need(gpb);
    // The workgroup must fit the kernel's own launch bound.
    hipFuncAttributes fa{};
    HIP_OK(hipFuncGetAttributes(&fa, kernel));
    if (L->threads > fa.maxThreadsPerBlock) return RKC_ENOTSUP;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L->lds) !=
        hipSuccess)
        return RKC_EDEVICE;
    const size_t blocks_all = (n_cells + gpb - 1) / gpb;
    L->persistent = false;
    size_t blocks = blocks_all;
    const int sched = o.schedule;
    if (allow_persistent && sched != RKC_SCHED_PLAIN) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, L->threads, L->lds) !=
            hipSuccess)
            return RKC_EDEVICE;
        per_cu = std::max(1, per_cu);
        size_t resident = (size_t)per_cu * (size_t)m->num_cus;
        if (o.grid_blocks > 0) resident = (size_t)o.grid_blocks;
        if (sched == RKC_SCHED_PERSISTENT || resident < blocks_all) {
            L->persistent = true;
            blocks = std::min(blocks_all, resident);
        }
    }
    if (blocks > 0x7fffffff) return RKC_ENOTSUP;
    L->blocks = (int)std::max<size_t>(1, blocks);
    return RKC_OK;
}

void fill_params(const rkc_mech *m, const Choice &ch, const NkTables *nk, rkcdev::Params *p) {
    std::memset(p, 0, sizeof(*p));
    p->nS = m->nS;
    p->N = m->N;
    p->ycs = m->nS;
    p->yss = 1;
    p->fcs = m->N;
    p->fss = 1;
    if (ch.v.G == 1) {
        p->nU = m->nU;
        p->RU = m->nU;
        p->NMS = (int)m->effsets.size();
        p->n_plain = m->n_plain;
        p->tab.units = m->units_d;
        p->l_spec = m->l_spec_d;
        p->l_units = m->l_units_d;
        p->l_pdep = m->pdep_d;
        p->l_eff = m->l_eff_d;
        p->lane_rows = lane_rows(m);
        p->invTmax = m->invTmax;
        p->agg = m->agg_d;
        p->queue = m->queue_d;
        p->coef = m->coef_d;
        p->coef_smax = m->coef_d ? COEF_SMAX : 0;
        p->invN = 1.0 / (double)m->N;
        return;
    }
    p->NK = nk->NK;
    p->nU = m->nU;
    p->RU = ch.RU;
    p->NSEG = nk->NSEG;
    p->SEGL = nk->SEGL;
    p->L2P = nk->L2P;
    p->L2N = nk->L2N;
    p->tab.units = m->units_d;
    p->tab.spec = nk->spec;
    p->tab.gather = nk->gather;
    p->tab.gather2 = nk->gather2;
    p->tab.units_il = nk->units_il;
    p->tab.pdep = nk->pdep;
    p->tab.eff = nk->eff;
    p->RUp = nk->RUp;
    p->RU2 = nk->RU2;
    p->invTmax = m->invTmax;
    p->NPR = nk->NPR;
    p->NMS = nk->NMS;
    p->agg = m->agg_d;
    p->queue = m->queue_d;
    p->coef = m->coef_d;
    p->coef_smax = m->coef_d ? COEF_SMAX : 0;
    p->invN = 1.0 / (double)m->N;
}

// Divergence measure of a run of consecutive cells (Sec. 3.1): the work of the
// run over `width` times its largest member's work.
__global__ void divergence_kernel(const int32_t *w, int stride, long long n, int width,
                                  double *D) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long first = r * (long long)width;
    if (first >= n) return;
    const long long last = first + width < n ? first + width : n;
    long long sum = 0;
    int mx = 0;
    for (long long i = first; i < last; ++i) {
        const int d = w[i * stride];
        sum += d;
        mx = d > mx ? d : mx;
    }
    D[r] = mx > 0 ? (double)sum / ((double)(last - first) * (double)mx) : 1.0;
}

}  // namespace

namespace rkchost {

int check_integrate_args(double dt, double rtol, double atol, const rkc_opts &o) {
    if (!(dt > 0.0) || !std::isfinite(dt) || !(rtol > 0.0) || !std::isfinite(rtol) ||
        !(atol >= 0.0) || !std::isfinite(atol))
        return RKC_EINVAL;
    if (o.method != RKC_METHOD_RKC && o.method != RKC_METHOD_RKCK) return RKC_EINVAL;
    if (o.s_max < 2 || o.max_steps < 1) return RKC_EINVAL;
    if (o.schedule < 0 || o.schedule > 2 || o.block_groups < 0 || o.grid_blocks < 0 ||
        o.param_placement < 0 || o.param_placement > 3 ||
        (o.stage_coefs != RKC_COEFS_TABLE && o.stage_coefs != RKC_COEFS_RECURRENCE) ||
        (o.layout != RKC_LAYOUT_CELL_MAJOR && o.layout != RKC_LAYOUT_SPECIES_MAJOR))
        return RKC_EINVAL;
    return RKC_OK;
}

int enqueue_integrate(rkc_mech *m, size_t n, double *Td, const double *Pd, double *Yd, double dt,
                      double rtol, double atol, const rkc_opts &o, int32_t *sd, int32_t *cd,
                      unsigned long long *agg_d, int *queue_d, hipStream_t st, LaunchInfo *li,
                      bool may_build) {
    Choice ch;
    NkTables *nk = nullptr;
    int rc = select_variant(m, o, &ch, &nk, may_build);
    if (rc) return rc;
    const bool pd = m->n_pdep > 0;
    const void *kernel = o.method == RKC_METHOD_RKC ? (pd ? ch.v.k_rkc_pd : ch.v.k_rkc)
                                                    : (pd ? ch.v.k_rkck_pd : ch.v.k_rkck);
    if (!kernel) return RKC_ENOTSUP;
    Launch L;
    rc = plan_launch(m, ch, kernel, n, o, true, nk, &L);
    if (rc) return rc;
    // launch errors are taken from the launch call itself: the thread's last
    // error can hold an unrelated earlier status (e.g. a not-ready query made
    // by other code in the process)
    {
        void *rargs[] = {&agg_d, &queue_d};
        HIP_OK(hipLaunchKernel(reinterpret_cast<const void *>(&reset_scratch_kernel), dim3(1),
                               dim3(64), rargs, 0, st));
    }
    rkcdev::Params p;
    fill_params(m, ch, nk, &p);
    p.agg = agg_d;
    p.queue = queue_d;
    p.n_cells = (int)n;
    p.T = Td;
    p.P = Pd;
    p.Y = Yd;
    p.dt = dt;
    p.rtol = rtol;
    p.atol = atol;
    p.s_max = o.s_max;
    p.max_steps = o.max_steps;
    p.cell_status = sd;
    p.cell_counters = cd;
    p.persistent = L.persistent ? 1 : 0;
    p.groups_total = L.blocks * L.groups_per_block;
    if (o.stage_coefs == RKC_COEFS_RECURRENCE) p.coef_smax = 0;
    if (o.layout == RKC_LAYOUT_SPECIES_MAJOR) {
        p.ycs = 1;
        p.yss = (long long)n;
    }
    void *args[] = {&p};
    HIP_OK(hipLaunchKernel(kernel, dim3(L.blocks), dim3(L.threads), args, L.lds, st));
    li->G = ch.v.G;
    li->RUC = ch.v.RUC;
    li->persistent = L.persistent;
    li->blocks = L.blocks;
    li->threads = L.threads;
    li->lds = L.lds;
    return RKC_OK;
}

int prepare(rkc_mech *m, const rkc_opts &o, size_t n_cells) {
    Choice ch;
    NkTables *nk = nullptr;
    int rc = select_variant(m, o, &ch, &nk);
    if (rc || n_cells == 0) return rc;
    // sets the kernels' dynamic-LDS limit now rather than inside a capture
    Launch L;
    const bool pd = m->n_pdep > 0;
    for (const void *k : {pd ? ch.v.k_rkc_pd : ch.v.k_rkc, pd ? ch.v.k_rkck_pd : ch.v.k_rkck}) {
        if (!k) return RKC_ENOTSUP;
        rc = plan_launch(m, ch, k, n_cells, o, true, nk, &L);
        if (rc) return rc;
    }
    return RKC_OK;
}

int mech_species(const rkc_mech *m) { return m->nS; }
int mech_device(const rkc_mech *m) { return m->device; }

void fill_stats(const unsigned long long *agg, const LaunchInfo &li, rkc_stats *stats) {
    stats->n_rhs = (int64_t)agg[0];
    stats->n_steps = (int64_t)agg[1];
    stats->n_reject = (int64_t)agg[2];
    stats->n_sigma = (int64_t)agg[3];
    stats->n_power_iter = (int64_t)agg[4];
    stats->s_max_used = (int32_t)agg[5];
    stats->n_failed = (int32_t)agg[6];
    stats->worst_status = (int32_t)agg[7];
    stats->lanes_per_cell = li.G;
    stats->schedule = li.persistent ? RKC_SCHED_PERSISTENT : RKC_SCHED_PLAIN;
    stats->grid_blocks = li.blocks;
    stats->block_threads = li.threads;
    stats->lds_bytes = (int32_t)li.lds;
    stats->n_rhs_slots = (int64_t)agg[8];
    stats->param_placement = li.RUC > 0 ? RKC_PARAMS_REGISTERS
                                        : (li.RUC == 0 ? RKC_PARAMS_LDS : RKC_PARAMS_GLOBAL);
}

}  // namespace rkchost

extern "C" {

int rkc_opts_default(rkc_opts *o) {
    if (!o) return RKC_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->method = RKC_METHOD_RKC;
    o->s_max = 1000;
    o->max_steps = 1000000;
    o->schedule = RKC_SCHED_AUTO;
    return RKC_OK;
}

const char *rkc_strerror(int code) {
    switch (code) {
    case RKC_OK: return "ok";
    case RKC_EINVAL: return "invalid argument";
    case RKC_ENOMEM: return "out of memory";
    case RKC_EDEVICE: return "HIP runtime error";
    case RKC_ECELLS: return "some cells failed";
    case RKC_ENOTSUP: return "mechanism or option not supported by the compiled variants";
    default: return "unknown error";
    }
}

int rkc_mech_destroy(rkc_mech *m) {
    if (!m) return RKC_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(m->device);
    if (m->units_d) (void)hipFree(m->units_d);
    for (auto &t : m->nk) {
        (void)hipFree(t.spec);
        (void)hipFree(t.gather);
        (void)hipFree(t.gather2);
        if (t.units_il) (void)hipFree(t.units_il);
        if (t.pdep) (void)hipFree(t.pdep);
        if (t.eff) (void)hipFree(t.eff);
    }
    if (m->agg_d) (void)hipFree(m->agg_d);
    if (m->queue_d) (void)hipFree(m->queue_d);
    if (m->coef_d) (void)hipFree(m->coef_d);
    if (m->pdep_d) (void)hipFree(m->pdep_d);
    if (m->stage_d) (void)hipFree(m->stage_d);
    if (m->l_spec_d) (void)hipFree(m->l_spec_d);
    if (m->l_units_d) (void)hipFree(m->l_units_d);
    if (m->l_eff_d) (void)hipFree(m->l_eff_d);
    (void)hipSetDevice(dev);
    delete m;
    return RKC_OK;
}

int rkc_mech_create(const rkc_mech_desc *d, rkc_mech **out) {
    if (!d || !out) return RKC_EINVAL;
    *out = nullptr;
    const int nS = d->n_species, nR = d->n_reactions;
    if (nS < 1 || nR < 0) return RKC_EINVAL;
    if (nS > 1021) return RKC_ENOTSUP;
    if (!d->W || !d->nasa_low || !d->nasa_high || !d->T_mid) return RKC_EINVAL;
    if (nR > 0 && (!d->reac || !d->prod || !d->A || !d->beta || !d->Ea)) return RKC_EINVAL;
    for (int i = 0; i < nS; ++i) {
        if (!(d->W[i] > 0.0) || !std::isfinite(d->W[i]) || !std::isfinite(d->T_mid[i]))
            return RKC_EINVAL;
        for (int q = 0; q < 7; ++q)
            if (!std::isfinite(d->nasa_low[7 * i + q]) || !std::isfinite(d->nasa_high[7 * i + q]))
                return RKC_EINVAL;
    }
    for (int j = 0; j < nR && d->pdep; ++j) {
        const int kind = d->pdep[j];
        if (kind < RKC_PDEP_PLAIN || kind > RKC_PDEP_TROE) return RKC_EINVAL;
        if (kind != RKC_PDEP_PLAIN && d->eff)
            for (int i = 0; i < nS; ++i)
                if (!(d->eff[(size_t)j * nS + i] >= 0.0) || !std::isfinite(d->eff[(size_t)j * nS + i]))
                    return RKC_EINVAL;
        if (kind >= RKC_PDEP_LINDEMANN) {
            if (!d->A0 || !d->beta0 || !d->Ea0) return RKC_EINVAL;
            if (!(d->A0[j] >= 0.0) || !std::isfinite(d->A0[j]) ||
                !(std::fabs(d->beta0[j]) <= 1e5) || !std::isfinite(d->Ea0[j]))
                return RKC_EINVAL;
        }
        if (kind == RKC_PDEP_TROE) {
            if (!d->troe) return RKC_EINVAL;
            const double *t = d->troe + 4 * (size_t)j;
            if (!std::isfinite(t[0]) || !(t[1] > 0.0) || !(t[2] > 0.0) || !std::isfinite(t[3]))
                return RKC_EINVAL;
        }
    }
    for (int j = 0; j < nR; ++j) {
        if (!(d->A[j] >= 0.0) || !std::isfinite(d->A[j]) || !(std::fabs(d->beta[j]) <= 1e5) ||
            !std::isfinite(d->Ea[j]))
            return RKC_EINVAL;
        for (int s = 0; s < 3; ++s) {
            const int a = d->reac[3 * j + s], b = d->prod[3 * j + s];
            if (a < -1 || a >= nS || b < -1 || b >= nS) return RKC_EINVAL;
        }
    }
    rkc_mech *m = new (std::nothrow) rkc_mech();
    if (!m) return RKC_ENOMEM;
    m->nS = nS;
    m->nR = nR;
    m->N = nS + 1;
    m->W.assign(d->W, d->W + nS);
    m->lo.assign(d->nasa_low, d->nasa_low + 7 * nS);
    m->hi.assign(d->nasa_high, d->nasa_high + 7 * nS);
    m->Tmid.assign(d->T_mid, d->T_mid + nS);
    m->rows.assign(nS, {});

    // Reaction units: a reaction immediately followed by its exact reverse
    // (with the same pressure dependence) is one unit with net rate of
    // progress; any other reaction is a unit alone.  Plain units come first,
    // then the pressure-dependent ones by kind, so that the kernels' unit
    // rounds are uniform except for a few.
    struct UnitSrc {
        double rec[UNIT_DOUBLES];
        double pd[rkcdev::PDEP_DOUBLES];
        int kind;
        int three;                              // a side with three reactant slots
        std::vector<std::pair<int, int>> dnu;   // (species, nu'' - nu')
    };
    auto kind_of = [&](int j) { return d->pdep ? d->pdep[j] : RKC_PDEP_PLAIN; };
    auto eff_row = [&](int j) {
        std::vector<double> e(nS, 1.0);
        if (d->eff) e.assign(d->eff + (size_t)j * nS, d->eff + (size_t)(j + 1) * nS);
        return e;
    };
    std::vector<UnitSrc> srcs;
    for (int j = 0; j < nR;) {
        const int32_t *rf = d->reac + 3 * j, *pf = d->prod + 3 * j;
        const int kind = kind_of(j);
        bool pair = (j + 1 < nR) && same_multiset(d->reac + 3 * (j + 1), pf) &&
                    same_multiset(d->prod + 3 * (j + 1), rf) && kind_of(j + 1) == kind;
        if (pair && kind != RKC_PDEP_PLAIN) pair = eff_row(j) == eff_row(j + 1);
        if (pair && kind == RKC_PDEP_TROE)
            pair = std::equal(d->troe + 4 * (size_t)j, d->troe + 4 * (size_t)j + 4,
                              d->troe + 4 * (size_t)(j + 1));
        UnitSrc u;
        std::memset(u.rec, 0, sizeof(u.rec));
        std::memset(u.pd, 0, sizeof(u.pd));
        u.kind = kind;
        u.rec[0] = l2_a(d->A[j]);
        u.rec[1] = d->beta[j];
        u.rec[2] = theta2(d->Ea[j]);
        uint64_t idr = 0;
        const int32_t none[3] = {-1, -1, -1};
        if (pair) {
            u.rec[3] = l2_a(d->A[j + 1]);
            u.rec[4] = d->beta[j + 1];
            u.rec[5] = theta2(d->Ea[j + 1]);
            idr = pack_slots(d->reac + 3 * (j + 1), nS);
        } else {
            u.rec[3] = L2A_ZERO;
            idr = pack_slots(none, nS);
        }
        auto n_slots = [](const int32_t *x) { return (x[0] >= 0) + (x[1] >= 0) + (x[2] >= 0); };
        u.three = n_slots(rf) == 3 || (pair && n_slots(d->reac + 3 * (j + 1)) == 3);
        const uint64_t idf = pack_slots(rf, nS);
        std::memcpy(&u.rec[6], &idf, 8);
        std::memcpy(&u.rec[7], &idr, 8);
        if (kind != RKC_PDEP_PLAIN) {
            // efficiency set index
            const std::vector<double> e = eff_row(j);
            size_t q = 0;
            while (q < m->effsets.size() && m->effsets[q] != e) ++q;
            if (q == m->effsets.size()) m->effsets.push_back(e);
            const uint64_t tag = (uint64_t)kind | ((uint64_t)q << 8);
            std::memcpy(&u.pd[0], &tag, 8);
            if (kind >= RKC_PDEP_LINDEMANN) {
                u.pd[1] = l2_a(d->A0[j]);
                u.pd[2] = d->beta0[j];
                u.pd[3] = theta2(d->Ea0[j]);
                u.pd[4] = pair ? l2_a(d->A0[j + 1]) : L2A_ZERO;
                u.pd[5] = pair ? d->beta0[j + 1] : 0.0;
                u.pd[6] = pair ? theta2(d->Ea0[j + 1]) : 0.0;
            }
            if (kind == RKC_PDEP_TROE) {
                const double *t = d->troe + 4 * (size_t)j;
                // The kernels evaluate exp(-T / T***), exp(-T / T*) and
                // exp(-T** / T) as powers of 2 with a saturating exponential
                // exact for arguments of magnitude below 2^51.  Sentinels
                // such as T*** = 1e-30 or T** = 1e30 ("term off") are bounded
                // to TROE_BOUND, which leaves every value unchanged between
                // 1e-5 K and 1e5 K: the term is exactly 0 there either way.
                u.pd[8] = t[0];
                u.pd[9] = std::min((double)(LOG2E_L / t[1]), TROE_BOUND);
                u.pd[10] = std::min((double)(LOG2E_L / t[2]), TROE_BOUND);
                u.pd[11] = std::min((double)(t[3] * LOG2E_L), TROE_BOUND);
            }
        }
        for (int i = 0; i < nS; ++i) {
            const int dnu = count_in(pf, i) - count_in(rf, i);
            if (dnu != 0) u.dnu.push_back({i, dnu});
        }
        srcs.push_back(u);
        j += pair ? 2 : 1;
    }
    // Bound on the 1/T of the Arrhenius factors that keeps every base-2
    // exponent |log2 A + beta log2 T - theta' / T| below 2^30 (|log2 T| <= 1075
    // for a positive double), as the kernels' exponential needs; with
    // |beta| <= 1e5 the numerator stays above 2^29.
    {
        double amax = 0.0, bmax = 0.0, tmax = 0.0;
        auto arr = [&](const double *x) {
            amax = std::max(amax, std::fabs(x[0]));
            bmax = std::max(bmax, std::fabs(x[1]));
            tmax = std::max(tmax, std::fabs(x[2]));
        };
        for (const UnitSrc &u : srcs) {
            arr(u.rec);
            arr(u.rec + 3);
            if (u.kind >= RKC_PDEP_LINDEMANN) {
                arr(u.pd + 1);
                arr(u.pd + 4);
            }
        }
        const double num = 1073741824.0 - amax - 1075.0 * bmax;
        m->invTmax = tmax > 0.0 ? num / tmax : DBL_MAX;
    }
    // plain units with at most two reactant slots on each side first: whole
    // rounds of them skip the third concentration factor (always the 1.0 slot)
    std::stable_sort(srcs.begin(), srcs.end(), [](const UnitSrc &x, const UnitSrc &y) {
        return x.kind != y.kind ? x.kind < y.kind : x.three < y.three;
    });
    if (m->effsets.size() > (size_t)rkcdev::MAX_EFFSETS) { delete m; return RKC_ENOTSUP; }
    std::vector<double> units;
    int p = 0;
    for (const UnitSrc &u : srcs) {
        units.insert(units.end(), u.rec, u.rec + UNIT_DOUBLES);
        if (u.kind != RKC_PDEP_PLAIN) m->pdep_h.insert(m->pdep_h.end(), u.pd, u.pd + rkcdev::PDEP_DOUBLES);
        else ++m->n_plain;
        if (u.kind == RKC_PDEP_PLAIN && !u.three) ++m->n_two;
        for (const auto &e : u.dnu) m->rows[e.first].push_back({p, e.second});
        ++p;
    }
    m->n_pdep = p - m->n_plain;
    m->nU = p;
    m->nU_pad = std::max(64, (p + 63) / 64 * 64);
    if (m->nU_pad >= (1 << 23)) { delete m; return RKC_ENOTSUP; }
    // padding units: zero parameters and empty slots -> net rate 1 - 1 = 0, never gathered
    double pad[UNIT_DOUBLES] = {0};
    {
        const int32_t none[3] = {-1, -1, -1};
        const uint64_t bits = pack_slots(none, nS);
        std::memcpy(&pad[6], &bits, 8);
        std::memcpy(&pad[7], &bits, 8);
    }
    for (int q = p; q < m->nU_pad; ++q) units.insert(units.end(), pad, pad + UNIT_DOUBLES);
    m->units_h = units;
    for (int i = 0; i < nS; ++i) {
        m->nnz += (int)m->rows[i].size();
        m->max_row = std::max(m->max_row, (int)m->rows[i].size());
    }

    int rc = RKC_OK;
    hipDeviceProp_t prop;
    if (hipGetDevice(&m->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, m->device) != hipSuccess) {
        rc = RKC_EDEVICE;
    } else {
        m->num_cus = prop.multiProcessorCount;
        m->max_lds = prop.sharedMemPerBlock;
        if (hipMalloc(&m->units_d, m->units_h.size() * 8) != hipSuccess ||
            hipMalloc(&m->agg_d, AGG_N * sizeof(unsigned long long)) != hipSuccess ||
            hipMalloc(&m->queue_d, sizeof(int)) != hipSuccess)
            rc = RKC_ENOMEM;
        else if (hipMemcpy(m->units_d, m->units_h.data(), m->units_h.size() * 8,
                           hipMemcpyHostToDevice) != hipSuccess)
            rc = RKC_EDEVICE;
        if (rc == RKC_OK && m->n_pdep > 0) {
            if (hipMalloc(&m->pdep_d, m->pdep_h.size() * 8) != hipSuccess)
                rc = RKC_ENOMEM;
            else if (hipMemcpy(m->pdep_d, m->pdep_h.data(), m->pdep_h.size() * 8,
                               hipMemcpyHostToDevice) != hipSuccess)
                rc = RKC_EDEVICE;
        }
        if (rc == RKC_OK) {
            const std::vector<double> ct = coef_table();
            if (hipMalloc(&m->coef_d, ct.size() * 8) != hipSuccess)
                rc = RKC_ENOMEM;
            else if (hipMemcpy(m->coef_d, ct.data(), ct.size() * 8, hipMemcpyHostToDevice) !=
                     hipSuccess)
                rc = RKC_EDEVICE;
        }
    }
    if (rc != RKC_OK) {
        rkc_mech_destroy(m);
        return rc;
    }
    *out = m;
    return RKC_OK;
}

int rkc_mech_info(const rkc_mech *m, int32_t *n_species, int32_t *n_reactions, int32_t *n_units,
                  int32_t *nnz) {
    if (!m) return RKC_EINVAL;
    if (n_species) *n_species = m->nS;
    if (n_reactions) *n_reactions = m->nR;
    if (n_units) *n_units = m->nU;
    if (nnz) *nnz = m->nnz;
    return RKC_OK;
}

int rkc_rhs(const rkc_mech *mc, size_t n, const double *T, const double *P, const double *Y,
            double *f, const rkc_opts *opts) {
    if (!mc) return RKC_EINVAL;
    rkc_mech *m = const_cast<rkc_mech *>(mc);
    rkc_opts o;
    if (opts) o = *opts; else rkc_opts_default(&o);
    if (n == 0) return RKC_OK;
    if (!T || !P || !Y || !f) return RKC_EINVAL;
    if (n > RKC_MAX_CELLS) return RKC_ENOTSUP;
    DeviceScope dev;
    HIP_OK(dev.enter(m->device));
    Choice ch;
    NkTables *nk = nullptr;
    int rc = select_variant(m, o, &ch, &nk);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)o.stream;
    const double *Td = T, *Pd = P, *Yd = Y;
    double *fd = f;
    const size_t N = (size_t)m->N, nS = (size_t)m->nS;
    if (!o.device_ptrs) {
        const size_t bytes = 8 * n * (2 + nS + N);
        rc = ensure_stage(m, bytes);
        if (rc) return rc;
        double *b = (double *)m->stage_d;
        double *Tb = b, *Pb = b + n, *Yb = b + 2 * n;
        fd = b + 2 * n + n * nS;
        HIP_OK(hipMemcpyAsync(Tb, T, 8 * n, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(Pb, P, 8 * n, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(Yb, Y, 8 * n * nS, hipMemcpyHostToDevice, st));
        Td = Tb; Pd = Pb; Yd = Yb;
    }
    rkc_opts lo = o;
    lo.schedule = RKC_SCHED_PLAIN;
    Launch L;
    const void *krhs = m->n_pdep > 0 ? ch.v.k_rhs_pd : ch.v.k_rhs;
    if (!krhs) return RKC_ENOTSUP;
    rc = plan_launch(m, ch, krhs, n, lo, false, nk, &L);
    if (rc) return rc;
    rkcdev::Params p;
    fill_params(m, ch, nk, &p);
    p.n_cells = (int)n;
    p.T = const_cast<double *>(Td);
    p.P = Pd;
    p.Y = const_cast<double *>(Yd);
    p.F = fd;
    if (o.layout == RKC_LAYOUT_SPECIES_MAJOR) {
        p.ycs = 1;
        p.yss = (long long)n;
        p.fcs = 1;
        p.fss = (long long)n;
    } else if (o.layout != RKC_LAYOUT_CELL_MAJOR) {
        return RKC_EINVAL;
    }
    void *args[] = {&p};
    HIP_OK(hipLaunchKernel(krhs, dim3(L.blocks), dim3(L.threads), args, L.lds, st));
    if (!o.device_ptrs) {
        HIP_OK(hipMemcpyAsync(f, fd, 8 * n * N, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    return RKC_OK;
}

int rkc_integrate(const rkc_mech *mc, size_t n, double *T, const double *P, double *Y,
                  double dt, double rtol, double atol, const rkc_opts *opts,
                  int32_t *cell_status, rkc_stats *stats) {
    if (!mc) return RKC_EINVAL;
    rkc_mech *m = const_cast<rkc_mech *>(mc);
    rkc_opts o;
    if (opts) o = *opts; else rkc_opts_default(&o);
    int rc = rkchost::check_integrate_args(dt, rtol, atol, o);
    if (rc) return rc;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0) return RKC_OK;
    if (!T || !P || !Y) return RKC_EINVAL;
    if (n > RKC_MAX_CELLS) return RKC_ENOTSUP;
    DeviceScope dev;
    HIP_OK(dev.enter(m->device));

    hipStream_t st = (hipStream_t)o.stream;
    const size_t nS = (size_t)m->nS;
    double *Td = T, *Yd = Y;
    const double *Pd = P;
    int32_t *sd = cell_status, *cd = o.cell_counters;
    if (!o.device_ptrs) {
        const size_t bytes = 8 * n * (2 + nS) + 4 * n + (o.cell_counters ? 32 * n : 0);
        rc = ensure_stage(m, bytes);
        if (rc) return rc;
        double *b = (double *)m->stage_d;
        Td = b;
        double *Pb = b + n;
        Yd = b + 2 * n;
        sd = (int32_t *)(b + 2 * n + n * nS);
        cd = o.cell_counters ? sd + n : nullptr;
        HIP_OK(hipMemcpyAsync(Td, T, 8 * n, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(Pb, P, 8 * n, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(Yd, Y, 8 * n * nS, hipMemcpyHostToDevice, st));
        Pd = Pb;
    }
    rkchost::LaunchInfo li;
    rc = rkchost::enqueue_integrate(m, n, Td, Pd, Yd, dt, rtol, atol, o, sd, cd, m->agg_d,
                                    m->queue_d, st, &li);
    if (rc) return rc;
    unsigned long long agg[AGG_N] = {0};
    const bool sync = !o.device_ptrs || stats;
    if (!o.device_ptrs) {
        HIP_OK(hipMemcpyAsync(T, Td, 8 * n, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(Y, Yd, 8 * n * nS, hipMemcpyDeviceToHost, st));
        if (cell_status) HIP_OK(hipMemcpyAsync(cell_status, sd, 4 * n, hipMemcpyDeviceToHost, st));
        if (o.cell_counters)
            HIP_OK(hipMemcpyAsync(o.cell_counters, cd, 32 * n, hipMemcpyDeviceToHost, st));
    }
    if (sync) {
        HIP_OK(hipMemcpyAsync(agg, m->agg_d, sizeof(agg), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    if (stats) rkchost::fill_stats(agg, li, stats);
    if (sync && agg[6] > 0) return RKC_ECELLS;
    return RKC_OK;
}

int rkc_divergence(size_t n, const int32_t *work, int32_t stride, int32_t width, double *D,
                   const rkc_opts *opts) {
    rkc_opts o;
    if (opts) o = *opts; else rkc_opts_default(&o);
    if (stride < 1 || width < 1) return RKC_EINVAL;
    if (n == 0) return RKC_OK;
    if (!work || !D) return RKC_EINVAL;
    if (n > 0x7fffffff || (size_t)stride * n > ((size_t)1 << 40)) return RKC_ENOTSUP;
    const size_t runs = (n + (size_t)width - 1) / (size_t)width;
    hipStream_t st = (hipStream_t)o.stream;
    const int32_t *wd = work;
    double *Dd = D;
    void *tmp = nullptr;
    const size_t wbytes = 4 * ((n - 1) * (size_t)stride + 1);
    if (!o.device_ptrs) {
        if (hipMalloc(&tmp, (wbytes + 7) / 8 * 8 + 8 * runs) != hipSuccess) return RKC_ENOMEM;
        wd = (const int32_t *)tmp;
        Dd = (double *)((char *)tmp + ((wbytes + 7) / 8) * 8);
        if (hip_failed(hipMemcpyAsync((void *)wd, work, wbytes, hipMemcpyHostToDevice, st),
                       "hipMemcpyAsync(work)", __LINE__)) {
            (void)hipFree(tmp);
            return RKC_EDEVICE;
        }
    }
    const int threads = 256;
    const size_t blocks = (runs + threads - 1) / threads;
    int stride_a = stride, width_a = width;
    long long n_a = (long long)n;
    void *args[] = {&wd, &stride_a, &n_a, &width_a, &Dd};
    int rc = RKC_OK;
    if (hip_failed(hipLaunchKernel(reinterpret_cast<const void *>(&divergence_kernel),
                                   dim3((unsigned)blocks), dim3(threads), args, 0, st),
                   "hipLaunchKernel(divergence_kernel)", __LINE__))
        rc = RKC_EDEVICE;
    if (!o.device_ptrs) {
        if (rc == RKC_OK &&
            (hip_failed(hipMemcpyAsync(D, Dd, 8 * runs, hipMemcpyDeviceToHost, st),
                        "hipMemcpyAsync(D)", __LINE__) ||
             hip_failed(hipStreamSynchronize(st), "hipStreamSynchronize", __LINE__)))
            rc = RKC_EDEVICE;
        (void)hipFree(tmp);
    }
    return rc;
}

int rkc_graph_destroy(rkc_graph *g) {
    if (!g) return RKC_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(g->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->agg_d) (void)hipFree(g->agg_d);
    if (g->queue_d) (void)hipFree(g->queue_d);
    (void)hipSetDevice(dev);
    delete g;
    return RKC_OK;
}

int rkc_graph_create(const rkc_mech *mc, size_t n, double *T, const double *P, double *Y,
                     double dt, double rtol, double atol, const rkc_opts *opts,
                     int32_t *cell_status, rkc_graph **out) {
    if (!mc || !out || !opts) return RKC_EINVAL;
    *out = nullptr;
    rkc_mech *m = const_cast<rkc_mech *>(mc);
    rkc_opts o = *opts;
    if (!o.device_ptrs) return RKC_EINVAL;
    int rc = rkchost::check_integrate_args(dt, rtol, atol, o);
    if (rc) return rc;
    if (n == 0 || !T || !P || !Y) return RKC_EINVAL;
    if (n > RKC_MAX_CELLS) return RKC_ENOTSUP;
    DeviceScope dev;
    HIP_OK(dev.enter(m->device));
    rkc_graph *g = new (std::nothrow) rkc_graph();
    if (!g) return RKC_ENOMEM;
    g->device = m->device;
    hipStream_t cap = nullptr;
    rkchost::LaunchInfo li;
    if (hipMalloc(&g->agg_d, AGG_N * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&g->queue_d, sizeof(int)) != hipSuccess)
        rc = RKC_ENOMEM;
    if (rc == RKC_OK) rc = rkchost::prepare(m, o, n);
    if (rc == RKC_OK &&
        hip_failed(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate",
                   __LINE__))
        rc = RKC_EDEVICE;
    if (rc == RKC_OK &&
        hip_failed(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed), "BeginCapture",
                   __LINE__))
        rc = RKC_EDEVICE;
    if (rc == RKC_OK) {
        const int erc = rkchost::enqueue_integrate(m, n, T, P, Y, dt, rtol, atol, o, cell_status,
                                                   o.cell_counters, g->agg_d, g->queue_d, cap,
                                                   &li);
        const bool end_bad = hip_failed(hipStreamEndCapture(cap, &g->graph), "EndCapture",
                                        __LINE__);
        rc = erc ? erc : (end_bad ? RKC_EDEVICE : RKC_OK);
    }
    if (rc == RKC_OK &&
        hip_failed(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0),
                   "hipGraphInstantiate", __LINE__))
        rc = RKC_EDEVICE;
    if (cap) (void)hipStreamDestroy(cap);
    if (rc) {
        rkc_graph_destroy(g);
        return rc;
    }
    *out = g;
    return RKC_OK;
}

int rkc_graph_launch(rkc_graph *g, void *stream) {
    if (!g) return RKC_EINVAL;
    HIP_OK(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return RKC_OK;
}

int rkc_autotune(const rkc_mech *mc, size_t n, const double *T, const double *P,
                 const double *Y, double dt, double rtol, double atol, const rkc_opts *opts,
                 rkc_opts *tuned, float *best_ms) {
    if (!mc || !tuned) return RKC_EINVAL;
    rkc_mech *m = const_cast<rkc_mech *>(mc);
    rkc_opts o;
    if (opts) o = *opts; else rkc_opts_default(&o);
    int rc = rkchost::check_integrate_args(dt, rtol, atol, o);
    if (rc) return rc;
    if (n == 0 || !T || !P || !Y) return RKC_EINVAL;
    if (n > RKC_MAX_CELLS) return RKC_ENOTSUP;
    int log2n = 0;
    while (((size_t)1 << (log2n + 1)) <= n) ++log2n;
    for (const auto &e : m->tuned)
        if (e.method == o.method && e.lanes == o.lanes_per_cell &&
            e.placement == o.param_placement && e.layout == o.layout && e.log2n == log2n) {
            *tuned = o;
            tuned->lanes_per_cell = e.opts.lanes_per_cell;
            tuned->param_placement = e.opts.param_placement;
            tuned->schedule = e.opts.schedule;
            tuned->block_groups = e.opts.block_groups;
            tuned->grid_blocks = 0;
            if (best_ms) *best_ms = e.ms;
            return RKC_OK;
        }
    DeviceScope dev;
    HIP_OK(dev.enter(m->device));
    hipStream_t st = (hipStream_t)o.stream;
    const size_t nS = (size_t)m->nS;
    // working copies: [T0 | P | Y0 | T | Y | status]
    const size_t bytes = 8 * n * (3 + 2 * nS) + 4 * n;
    double *buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) return RKC_ENOMEM;
    double *T0 = buf, *Pd = buf + n, *Y0 = buf + 2 * n, *Tw = Y0 + n * nS, *Yw = Tw + n;
    int32_t *sd = (int32_t *)(Yw + n * nS);
    const hipMemcpyKind kind = o.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = RKC_OK;
    if (hip_failed(hipMemcpyAsync(T0, T, 8 * n, kind, st), "copy T", __LINE__) ||
        hip_failed(hipMemcpyAsync(Pd, P, 8 * n, kind, st), "copy P", __LINE__) ||
        hip_failed(hipMemcpyAsync(Y0, Y, 8 * n * nS, kind, st), "copy Y", __LINE__) ||
        hip_failed(hipEventCreate(&e0), "event", __LINE__) ||
        hip_failed(hipEventCreate(&e1), "event", __LINE__))
        rc = RKC_EDEVICE;

    // Time one candidate: `reps` runs from the same copied state (the first
    // use of a variant, which builds its tables, is not timed); the minimum.
    auto time_it = [&](const rkc_opts &c, int reps, float *ms_out) -> int {
        float best = -1.0f;
        for (int r = -1; r < reps; ++r) {
            rkchost::LaunchInfo li;
            if (hip_failed(hipMemcpyAsync(Tw, T0, 8 * n, hipMemcpyDeviceToDevice, st), "copy",
                           __LINE__) ||
                hip_failed(hipMemcpyAsync(Yw, Y0, 8 * n * nS, hipMemcpyDeviceToDevice, st), "copy",
                           __LINE__) ||
                hip_failed(hipEventRecord(e0, st), "record", __LINE__))
                return RKC_EDEVICE;
            const int erc = rkchost::enqueue_integrate(m, n, Tw, Pd, Yw, dt, rtol, atol, c, sd,
                                                       nullptr, m->agg_d, m->queue_d, st, &li);
            if (erc) return erc;
            float ms = 0.0f;
            if (hip_failed(hipEventRecord(e1, st), "record", __LINE__) ||
                hip_failed(hipEventSynchronize(e1), "sync", __LINE__) ||
                hip_failed(hipEventElapsedTime(&ms, e0, e1), "elapsed", __LINE__))
                return RKC_EDEVICE;
            if (r >= 0 && (best < 0.0f || ms < best)) best = ms;
        }
        *ms_out = best;
        return RKC_OK;
    };

    // Stage 1: every lane-group size and parameter placement the mechanism can
    // run (or the requested ones), default schedule and grain.
    std::vector<int> lanes_c, place_c;
    if (o.lanes_per_cell != 0) lanes_c = {o.lanes_per_cell};
    else lanes_c = {64, 32, 16, 8, 1};
    if (o.param_placement != RKC_PARAMS_AUTO) place_c = {o.param_placement};
    else place_c = {RKC_PARAMS_LDS, RKC_PARAMS_GLOBAL, RKC_PARAMS_REGISTERS};
    struct Cand {
        rkc_opts c;
        float ms;
    };
    std::vector<Cand> stage1;
    for (int G : lanes_c)
        for (int pl : place_c) {
            if (rc) break;
            Choice ch;
            if (choose_variant(m, G, pl, &ch) != RKC_OK) continue;
            if (pl == RKC_PARAMS_REGISTERS && ch.v.RUC <= 0) continue;   // fell back to LDS
            if (pl == RKC_PARAMS_GLOBAL && (G == 1 || !find_variant(ch.v.G, ch.v.NSL, -1)))
                continue;
            if (G == 1 && pl != RKC_PARAMS_LDS) continue;   // one placement for one lane per cell
            rkc_opts c = o;
            c.device_ptrs = 1;
            c.cell_counters = nullptr;
            c.lanes_per_cell = G;
            c.param_placement = pl;
            c.schedule = RKC_SCHED_PERSISTENT;
            c.block_groups = 0;
            c.grid_blocks = 0;
            float ms = 0.0f;
            const int trc = time_it(c, 2, &ms);
            if (trc == RKC_ENOTSUP) continue;   // does not fit (LDS, variant)
            if (trc) { rc = trc; break; }
            stage1.push_back({c, ms});
        }
    if (rc == RKC_OK && stage1.empty()) rc = RKC_ENOTSUP;
    // Stage 2: for the two fastest, both schedules and workgroups of the
    // largest, half and a quarter of the lane groups (or lanes) they allow.
    Cand best{o, -1.0f};
    if (rc == RKC_OK) {
        std::sort(stage1.begin(), stage1.end(),
                  [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
        best = stage1[0];
        for (size_t k = 0; k < std::min<size_t>(2, stage1.size()) && rc == RKC_OK; ++k) {
            Choice ch;
            (void)choose_variant(m, stage1[k].c.lanes_per_cell, stage1[k].c.param_placement, &ch);
            const int gmax = ch.v.G == 1 ? ch.v.max_threads : std::max(1, ch.v.max_threads / ch.v.G);
            for (int sched : {RKC_SCHED_PERSISTENT, RKC_SCHED_PLAIN})
                for (int div : {1, 2, 4}) {
                    if (sched == RKC_SCHED_PERSISTENT && div == 1) continue;   // stage 1 ran it
                    const int bg = ch.v.G == 1 ? std::max(64, gmax / div) : std::max(1, gmax / div);
                    rkc_opts c = stage1[k].c;
                    c.schedule = sched;
                    c.block_groups = bg;
                    float ms = 0.0f;
                    const int trc = time_it(c, 2, &ms);
                    if (trc == RKC_ENOTSUP) continue;
                    if (trc) { rc = trc; break; }
                    if (ms < best.ms) best = {c, ms};
                }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (rc) return rc;
    *tuned = o;
    tuned->lanes_per_cell = best.c.lanes_per_cell;
    tuned->param_placement = best.c.param_placement;
    tuned->schedule = best.c.schedule;
    tuned->block_groups = best.c.block_groups;
    tuned->grid_blocks = 0;
    m->tuned.push_back({o.method, o.lanes_per_cell, o.param_placement, o.layout, log2n, *tuned,
                        best.ms});
    if (best_ms) *best_ms = best.ms;
    return RKC_OK;
}

}  // extern "C"
