// Device code of the batched chemical-kinetics integrator (gfx950, FP64).
//
// One cell (an independent kinetics ODE, Sec. 2.2) is owned by a group of G
// lanes of a 64-wide wavefront (G = 8, 16, 32 or 64).  Inside a group:
//   - state element k of y = {T, Y_1..Y_nS} lives on lane k % G, slot k / G;
//   - reaction unit p (a forward/reverse pair, or one unpaired reaction) is
//     evaluated by lane p % G, round p / G;
//   - the net production sum (E:spec-rate) is a gather over a species-major
//     table of (unit, nu'' - nu') entries, one species row per lane slot;
//   - norms and mixture sums are XOR-butterfly reductions over the G lanes,
//     so every lane of a group holds bitwise identical scalars and takes the
//     same decisions.
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
//   [0..2] ln A, beta, theta = Ea/R of the forward reaction
//   [3..5] the same for the reverse reaction (ln A = -1e300 for an unpaired
//          reaction, so its reverse rate is exactly zero)
//   [6]    bit pattern: low 32 bits forward reactant slots, high 32 bits
//          reverse reactant slots; three 10-bit species indices each, the
//          value n_species meaning an empty slot (LDS C[n_species] == 1.0)
//   [7]    0
constexpr int UNIT_DOUBLES = 8;

struct Tables {
    const double *units;     // [RU * G][8]
    const double *spec;      // [NFIELD][NK]
    const int32_t *ent;      // [nnz] species-major: (unit << 8) | (dnu + 128)
    const int32_t *row_ptr;  // [NK + 1] start of each state index's entries
};

struct Params {
    int nS, N, NK, nU, RU, nnz;
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
    unsigned long long *agg;         // [8] aggregate counters
    int *queue;                      // persistent work-queue head
    int persistent;
    int groups_total;                // groups in the launched grid
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ double gsum(double x) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) x += __shfl_xor(x, m, G);
    return x;
}

template <int G>
__device__ __forceinline__ void gsum2(double &a, double &b) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        double ta = __shfl_xor(a, m, G);
        double tb = __shfl_xor(b, m, G);
        a += ta;
        b += tb;
    }
}

template <int G>
__device__ __forceinline__ double gmax(double x) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) x = fmax(x, __shfl_xor(x, m, G));
    return x;
}

template <int G>
__device__ __forceinline__ int gor(int x) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) x |= __shfl_xor(x, m, G);
    return x;
}

// Registers holding the reaction parameters of a lane's units (RUC > 0).
template <int RUC>
struct UnitRegs {
    double lnAf[RUC], bf[RUC], tf[RUC], lnAr[RUC], br[RUC], tr[RUC];
    uint32_t idf[RUC], idr[RUC];
};
template <>
struct UnitRegs<0> {};

struct GroupLds {
    const double *spec;
    const int32_t *ent;
    const int32_t *rowptr;
    const double *units;   // LDS copy (RUC == 0 only)
    double *C;             // [NK] concentrations, C[nS] == 1.0
    double *Q;             // [RU * G] net rates of progress
};

__device__ __forceinline__ double unpack_c(const double *C, uint32_t id, int s) {
    return C[(id >> (10 * s)) & 1023u];
}

// Source term of E:mass and E:energy for the group's cell at state z.
// z/fz hold this lane's NSL elements (index k = s * G + g).
template <int G, int NSL, int RUC>
__device__ __forceinline__ void rhs_eval(const double (&z)[NSL], double P10, double (&fz)[NSL],
                                         const GroupLds &L, const UnitRegs<RUC> &ur,
                                         int g, int NK, int N, int RU) {
    const double T = __shfl(z[0], 0, G);
    const double invT = 1.0 / T;
    const double lnT = log(T);

    double sYW = 0.0, sYcp = 0.0;
    double hRT[NSL], invW[NSL];
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        const double Y = (k == 0) ? 0.0 : z[s];
        invW[s] = L.spec[F_INVW * NK + k];
        const bool hi = T >= L.spec[F_TMID * NK + k];
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
    const double rho = P10 / (R_ERG * T * sYW);

    wave_sync();   // previous evaluation's readers of C are done
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        if (k >= 1 && k < N) L.C[k - 1] = rho * z[s] * invW[s];
    }
    wave_sync();

    // Rates of progress (E:rxn-rate) with Arrhenius coefficients (E:rxn-const),
    // net of each forward/reverse pair.
    if constexpr (RUC > 0) {
#pragma unroll
        for (int r = 0; r < RUC; ++r) {
            const double kf = exp(ur.lnAf[r] + ur.bf[r] * lnT - ur.tf[r] * invT);
            const double kr = exp(ur.lnAr[r] + ur.br[r] * lnT - ur.tr[r] * invT);
            const uint32_t a = ur.idf[r], b = ur.idr[r];
            const double of = kf * unpack_c(L.C, a, 0) * unpack_c(L.C, a, 1) * unpack_c(L.C, a, 2);
            const double orv = kr * unpack_c(L.C, b, 0) * unpack_c(L.C, b, 1) * unpack_c(L.C, b, 2);
            L.Q[r * G + g] = of - orv;
        }
    } else {
        for (int r = 0; r < RU; ++r) {
            const int p = r * G + g;
            const double2 *u = reinterpret_cast<const double2 *>(L.units + (size_t)p * UNIT_DOUBLES);
            const double2 u0 = u[0], u1 = u[1], u2 = u[2], u3 = u[3];
            const uint64_t bits = __double_as_longlong(u3.x);
            const uint32_t a = (uint32_t)bits, b = (uint32_t)(bits >> 32);
            const double kf = exp(u0.x + u0.y * lnT - u1.x * invT);
            const double kr = exp(u1.y + u2.x * lnT - u2.y * invT);
            const double of = kf * unpack_c(L.C, a, 0) * unpack_c(L.C, a, 1) * unpack_c(L.C, a, 2);
            const double orv = kr * unpack_c(L.C, b, 0) * unpack_c(L.C, b, 1) * unpack_c(L.C, b, 2);
            L.Q[p] = of - orv;
        }
    }
    wave_sync();

    // Net production (E:spec-rate), species equations (E:mass) and the
    // enthalpy sum of the energy equation (E:energy).
    double hs = 0.0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const int k = s * G + g;
        const int e0 = L.rowptr[k], e1 = L.rowptr[k + 1];
        double w = 0.0;
        for (int e = e0; e < e1; ++e) {
            const int en = L.ent[e];
            w += (double)((en & 0xff) - 128) * L.Q[en >> 8];
        }
        fz[s] = L.spec[F_W * NK + k] * w / rho;
        hs += hRT[s] * w;
    }
    hs = gsum<G>(hs);
    // dT/dt = -sum_i H_i omega_i / (rho cp); R cancels between H and cp.
    const double fT = -T * hs / (rho * sYcp);
    if (g == 0) fz[0] = fT;
}

// ---------------------------------------------------------------- staging

__device__ __forceinline__ void stage_tables(const Params &p, double *spec_l, int32_t *ent_l,
                                             int32_t *rowptr_l, double *units_l, int n_units_l) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < NFIELD * p.NK; i += nt) spec_l[i] = p.tab.spec[i];
    for (int i = tid; i < p.nnz; i += nt) ent_l[i] = p.tab.ent[i];
    for (int i = tid; i <= p.NK; i += nt) rowptr_l[i] = p.tab.row_ptr[i];
    for (int i = tid; i < n_units_l * UNIT_DOUBLES; i += nt) units_l[i] = p.tab.units[i];
}

template <int RUC>
__device__ __forceinline__ void load_unit_regs(const Params &p, UnitRegs<RUC> &ur, int g, int G) {
    if constexpr (RUC > 0) {
#pragma unroll
        for (int r = 0; r < RUC; ++r) {
            const double *u = p.tab.units + (size_t)(r * G + g) * UNIT_DOUBLES;
            ur.lnAf[r] = u[0]; ur.bf[r] = u[1]; ur.tf[r] = u[2];
            ur.lnAr[r] = u[3]; ur.br[r] = u[4]; ur.tr[r] = u[5];
            const uint64_t bits = __double_as_longlong(u[6]);
            ur.idf[r] = (uint32_t)bits;
            ur.idr[r] = (uint32_t)(bits >> 32);
        }
    }
}

// Bytes of per-group control state kept in LDS by the integrator kernels.
constexpr int STATE_BYTES = 256;

// Bytes of dynamic LDS for a workgroup of `groups` groups.
__host__ __device__ inline size_t lds_bytes(int NK, int RU, int G, int nnz, int groups,
                                            bool units_in_lds) {
    size_t b = (size_t)NFIELD * NK * 8;
    if (units_in_lds) b += (size_t)RU * G * UNIT_DOUBLES * 8;
    b += (size_t)groups * ((size_t)NK + (size_t)RU * G) * 8;
    b += (size_t)groups * STATE_BYTES;
    b += (size_t)nnz * 4 + ((size_t)NK + 1) * 4;
    return b;
}

struct LdsPtrs {
    double *spec, *units;
    int32_t *ent, *rowptr;
    double *groups;
    unsigned char *states;
};

__device__ __forceinline__ LdsPtrs carve(unsigned char *base, int NK, int RU, int G, int nnz,
                                         int groups, bool units_in_lds) {
    LdsPtrs l;
    size_t off = 0;
    l.spec = reinterpret_cast<double *>(base + off); off += (size_t)NFIELD * NK * 8;
    l.units = reinterpret_cast<double *>(base + off);
    if (units_in_lds) off += (size_t)RU * G * UNIT_DOUBLES * 8;
    l.groups = reinterpret_cast<double *>(base + off);
    off += (size_t)groups * ((size_t)NK + (size_t)RU * G) * 8;
    l.states = base + off;
    off += (size_t)groups * STATE_BYTES;
    l.ent = reinterpret_cast<int32_t *>(base + off); off += (size_t)nnz * 4;
    l.rowptr = reinterpret_cast<int32_t *>(base + off);
    return l;
}

// ------------------------------------------------------- source-term kernel

template <int G, int NSL, int RUC>
__global__ __launch_bounds__(512) void rhs_kernel(Params p) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int groups = blockDim.x / G;
    const int gib = threadIdx.x / G;
    const int g = threadIdx.x % G;
    LdsPtrs lp = carve(lds_raw, p.NK, p.RU, G, p.nnz, groups, RUC == 0);
    stage_tables(p, lp.spec, lp.ent, lp.rowptr, lp.units, RUC == 0 ? p.RU * G : 0);
    GroupLds L;
    L.spec = lp.spec; L.ent = lp.ent; L.rowptr = lp.rowptr; L.units = lp.units;
    L.C = lp.groups + (size_t)gib * (p.NK + p.RU * G);
    L.Q = L.C + p.NK;
    for (int k = g; k < p.NK; k += G) L.C[k] = (k == p.nS) ? 1.0 : 0.0;
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
            else if (k < p.N) v = p.Y[(size_t)cell * p.nS + (k - 1)];
        }
        z[s] = v;
    }
    if (!active) z[0] = (g == 0) ? 1000.0 : z[0];
    const double P10 = active ? p.P[cell] * 10.0 : 1e6;
    rhs_eval<G, NSL, RUC>(z, P10, fz, L, ur, g, p.NK, p.N, p.RU);
    if (active) {
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
            const int k = s * G + g;
            if (k < p.N) p.F[(size_t)cell * p.N + k] = fz[s];
        }
    }
}

}  // namespace rkcdev
