/*
 * rkc.h - C ABI of the MI355X (gfx950) batched chemical-kinetics integrator.
 *
 * Each grid cell of an operator-split reactive-flow simulation carries an
 * independent constant-pressure adiabatic kinetics ODE for y = {T, Y_1..Y_nS}
 * (Niemeyer & Sung, Sec. 2.2, Eqs. E:mass, E:spec-rate, E:rxn-rate,
 * E:rxn-const, E:energy).  rkc_integrate advances every cell over one global
 * chemistry step [0, dt] with internal sub-stepping (Sec. 3: the integrator
 * takes initial conditions and a global time step and restarts every call)
 * using either
 *   - RKC: the second-order Runge-Kutta-Chebyshev method with adaptive step
 *     size, stage count from a nonlinear power-method spectral radius
 *     (Sec. 2.4), or
 *   - RKCK: the fifth-order Runge-Kutta-Cash-Karp method with embedded error
 *     estimate (Sec. 2.3, Table 1).
 * All arithmetic is IEEE double precision in HIP kernels on the GPU.
 *
 * Conventions for every function:
 *   - return value: RKC_OK (0) or a negative RKC_E* code; nothing is thrown
 *     across the ABI; rkc_strerror() names a code.
 *   - arrays are caller-owned.  By default they are host pointers, copied to
 *     and from the device inside the call (which then returns after the work
 *     completed).  With opts->device_ptrs != 0 every array argument (T, P, Y,
 *     f, cell_status, opts->cell_counters) is a device pointer on the
 *     mechanism's device; the work is enqueued on opts->stream and the call
 *     returns without waiting unless a rkc_stats pointer is passed (then it
 *     synchronises the stream to fill it).
 *   - units: T in K, P in Pa, Y mass fractions, dt in s; mechanism units are
 *     listed at rkc_mech_desc.
 *   - calls that share one rkc_mech handle must not overlap in time (they share
 *     the handle's device scratch: work-queue counter and statistics).
 */
#ifndef RKC_H
#define RKC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define RKC_OK        0
#define RKC_EINVAL   (-1)   /* bad argument (NULL array, dt <= 0, rtol <= 0, size mismatch) */
#define RKC_ENOMEM   (-2)   /* device or host allocation failed */
#define RKC_EDEVICE  (-3)   /* a HIP runtime call failed */
#define RKC_ECELLS   (-4)   /* call completed but at least one cell failed */
#define RKC_ENOTSUP  (-5)   /* mechanism or option outside the compiled variants */

/* ---- per-cell status (cell_status[i], counters column 6) --------------- */
#define RKC_CELL_OK         0
#define RKC_CELL_UNDERFLOW  1   /* proposed step fell below 10 u dt */
#define RKC_CELL_MAXSTEPS   2   /* accepted + rejected steps reached max_steps */
#define RKC_CELL_NONFINITE  3   /* f(y0), the spectral radius or the initial error was not finite */
#define RKC_CELL_BADINPUT   4   /* T <= 0, P <= 0 or a non-finite input; cell left unchanged */

/* ---- integration method ------------------------------------------------- */
#define RKC_METHOD_RKC   0      /* Sec. 2.4 */
#define RKC_METHOD_RKCK  1      /* Sec. 2.3, Table 1 */

/* ---- launch schedule (never changes results: see rkc_integrate) --------- */
#define RKC_SCHED_AUTO        0
#define RKC_SCHED_PLAIN       1  /* one lane group per cell, grid covers all cells */
#define RKC_SCHED_PERSISTENT  2  /* resident grid; groups pull cells from a device queue
                                    in index order (cells ordered by decreasing expected
                                    cost, e.g. temperature, shorten the final tail) */

/* ---- placement of reaction parameters (never changes results) --------- */
#define RKC_PARAMS_AUTO       0  /* LDS (the measured faster placement), or global
                                    memory when the tables in LDS would hold the
                                    workgroup below its occupancy target (large
                                    mechanisms) and such a variant is compiled */
#define RKC_PARAMS_REGISTERS  1  /* registers, when a variant for the mechanism's size
                                    is compiled (else LDS) */
#define RKC_PARAMS_LDS        2
#define RKC_PARAMS_GLOBAL     3  /* reaction parameters and species table read from
                                    global memory through the caches (the range
                                    switch temperatures staged in LDS); RKC_ENOTSUP
                                    when no such variant is compiled for the shape */

/* Largest n_cells of one call (2^31 - 2^20): cell indices and work-queue
 * claims stay within int32 with room for every lane group of the grid;
 * larger calls return RKC_ENOTSUP. */
#define RKC_MAX_CELLS 2146435072

/* Number of int32 per cell in opts->cell_counters. */
#define RKC_NCOUNTERS 8
/* Column order of opts->cell_counters rows. */
enum { RKC_CNT_RHS = 0, RKC_CNT_STEPS = 1, RKC_CNT_REJECT = 2, RKC_CNT_SIGMA = 3,
       RKC_CNT_SMAX = 4, RKC_CNT_SHASH = 5, RKC_CNT_STATUS = 6, RKC_CNT_POWER_ITER = 7 };

typedef struct rkc_mech rkc_mech;   /* opaque, owned by the library */
typedef struct rkc_graph rkc_graph; /* opaque, owned by the library */

/* Mechanism description: irreversible reactions with Arrhenius rates
 * (E:rxn-const), mass-action rates of progress (E:rxn-rate) and two-range
 * NASA 7-coefficient thermodynamics (E:energy).  All arrays are host memory,
 * read during rkc_mech_create only.
 *   W          [n_species]            molar mass, g/mol (> 0)
 *   nasa_low   [n_species][7]         Cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4,
 *   nasa_high  [n_species][7]         H/(R T) = a1 + a2 T/2 + ... + a5 T^4/5 + a6/T
 *   T_mid      [n_species]            K; the high range is used iff T >= T_mid
 *   reac, prod [n_reactions][3]       species indices with repetition (a species
 *                                     listed twice has coefficient 2); -1 = empty;
 *                                     at most 3 molecules per side
 *   A          [n_reactions]          (cm^3/mol)^(m-1)/s, m = reactant molecules
 *   beta       [n_reactions]          temperature exponent
 *   Ea         [n_reactions]          J/mol
 * A reaction immediately followed by its exact reverse is evaluated as one
 * forward/reverse pair (net rate of progress), which is how mechanisms
 * converted by the paper's Appendix A procedure are laid out. */
typedef struct {
    int32_t n_species, n_reactions;
    const double *W;
    const double *nasa_low;
    const double *nasa_high;
    const double *T_mid;
    const int32_t *reac;
    const int32_t *prod;
    const double *A, *beta, *Ea;
    /* Optional pressure dependence (the third-body and falloff reactions of
     * Sec. 2.2, Chemkin formulation); pdep = NULL means every reaction plain.
     *   pdep   [n_reactions]              RKC_PDEP_* kind of each reaction
     *   eff    [n_reactions][n_species]   third-body efficiencies alpha, used by
     *                                     kinds 1-3 ([M] = sum alpha_i C_i); NULL = 1
     *   A0, beta0, Ea0 [n_reactions]      low-pressure limit k_0 of falloff
     *                                     reactions (units of A times cm^3/mol)
     *   troe   [n_reactions][4]           Troe a, T3, T1, T2 (K; T2 <= 0: the
     *                                     exp(-T2/T) term is absent)
     * Third body: rate k [M] prod C.  Falloff: k = k_inf Pr/(1 + Pr) F with
     * Pr = k_0 [M] / k_inf, F = 1 (Lindemann) or the Troe form; k = 0 when
     * k_inf or k_0 [M] is 0. */
    const int32_t *pdep;
    const double *eff;
    const double *A0, *beta0, *Ea0;
    const double *troe;
} rkc_mech_desc;

/* Kinds of rkc_mech_desc.pdep. */
#define RKC_PDEP_PLAIN      0
#define RKC_PDEP_THIRD_BODY 1
#define RKC_PDEP_LINDEMANN  2
#define RKC_PDEP_TROE       3

/* Options; rkc_opts_default() fills the defaults shown. */
typedef struct {
    int32_t method;          /* RKC_METHOD_RKC */
    int32_t s_max;           /* 1000: largest RKC stage count (>= 2) */
    int32_t max_steps;       /* 1000000: accepted + rejected steps per cell */
    int32_t lanes_per_cell;  /* 0 = automatic; else 1, 8, 16, 32 or 64.  Automatic:
                                N = n_species + 1 state elements, 16 lanes for
                                N <= 16, 32 for N <= 39 (or N <= 64 with
                                pressure-dependent reactions), else 64.
                                1 = one lane per cell (N <= 32): each lane of a
                                wavefront integrates its own cell, the mechanism
                                tables are read as wave-uniform scalars, and a
                                wave's per-cell rows of concentrations and net
                                production rates ((2 n_species + 2 + efficiency
                                sets) x 512 bytes) must fit in LDS, else
                                RKC_ENOTSUP */
    int32_t schedule;        /* RKC_SCHED_AUTO */
    int32_t block_groups;    /* lane groups per workgroup, 0 = automatic */
    int32_t grid_blocks;     /* persistent grid size in workgroups, 0 = automatic */
    int32_t device_ptrs;     /* 0: host arrays; 1: device arrays (see top) */
    void   *stream;          /* hipStream_t; NULL = the null stream */
    int32_t *cell_counters;  /* optional [n_cells][RKC_NCOUNTERS] per-cell counters */
    int32_t param_placement; /* RKC_PARAMS_AUTO */
    int32_t stage_coefs;     /* RKC_COEFS_TABLE: how RKC kernels obtain the stage
                                coefficients of Sec. 2.4 (rounding-level differences) */
    int32_t layout;          /* RKC_LAYOUT_CELL_MAJOR: memory order of Y (and of f
                                in rkc_rhs) */
} rkc_opts;

/* Values of rkc_opts.layout (the same for host and device arrays; T and P are
 * always [n_cells]):
 *   CELL_MAJOR     Y[cell][species] (element i of cell c at Y[c * n_species + i]),
 *                  f[cell][k] (at f[c * (n_species + 1) + k])
 *   SPECIES_MAJOR  Y[species][cell] (at Y[i * n_cells + c]), f[k][cell] (at
 *                  f[k * n_cells + c]): cell-fastest, so the lanes of a wave
 *                  that each hold one cell (lanes_per_cell = 1) read and write
 *                  consecutive doubles */
#define RKC_LAYOUT_CELL_MAJOR     0
#define RKC_LAYOUT_SPECIES_MAJOR  1

/* Values of rkc_opts.stage_coefs.  The coefficients mu~_1 and, per stage j,
 * mu_j, nu_j, mu~_j, gamma~_j of Sec. 2.4 depend only on (s, j). */
#define RKC_COEFS_TABLE       0  /* a table computed once on the host for s <= 128;
                                    larger stage counts advance the Chebyshev
                                    recurrences inside the kernel, one stage at a time */
#define RKC_COEFS_RECURRENCE  1  /* the in-kernel recurrences for every stage count */

/* Aggregate statistics of one call. */
typedef struct {
    int64_t n_rhs, n_steps, n_reject, n_sigma, n_power_iter;
    int32_t s_max_used;      /* largest RKC stage count any cell used */
    int32_t n_failed;        /* cells whose status is not RKC_CELL_OK */
    int32_t worst_status;    /* largest per-cell status code */
    int32_t lanes_per_cell;  /* variant that ran */
    int32_t schedule;        /* schedule that ran */
    int32_t grid_blocks;     /* workgroups launched */
    int32_t block_threads;   /* threads per workgroup */
    int32_t lds_bytes;       /* dynamic LDS per workgroup */
    int64_t n_rhs_slots;     /* source-term evaluations the lane groups issued: every
                                iteration of the integrator loop issues one per group,
                                whether or not the group still holds a cell, so
                                n_rhs / n_rhs_slots is the fraction of issued work that
                                advanced a cell (1 = no idle groups) */
    int32_t param_placement; /* placement that ran: RKC_PARAMS_REGISTERS, _LDS or _GLOBAL */
} rkc_stats;

/* Fill *opts with the defaults.  Returns RKC_EINVAL for NULL. */
int rkc_opts_default(rkc_opts *opts);

/* Validate a mechanism, pack its tables and upload them to the current HIP
 * device.  On success *out owns device memory until rkc_mech_destroy.
 * Errors: RKC_EINVAL (sizes < 1, index out of range, > 3 molecules per side,
 * W <= 0, non-finite parameter, A < 0, |beta| or |beta0| > 1e5, a pdep kind
 * outside 0..3, a falloff reaction without A0/beta0/Ea0, a Troe reaction
 * without troe or with T3 <= 0 or T1 <= 0, a negative efficiency),
 * RKC_ENOTSUP (n_species > 1021), RKC_ENOMEM, RKC_EDEVICE.
 * The kernels evaluate every Arrhenius factor with 1/T bounded by
 * (2^30 - max|log2 A| - 1075 max|beta|) / max|Ea/R log2(e)| over the
 * mechanism's reactions and low-pressure limits (for activation energies up
 * to 1e6 J/mol a bound above 5e3 1/K, i.e. temperatures below 2e-4 K are
 * treated as that temperature in these factors only); this keeps every
 * base-2 exponent below 2^30 in magnitude. */
int rkc_mech_create(const rkc_mech_desc *desc, rkc_mech **out);

/* Release a mechanism; NULL is accepted. */
int rkc_mech_destroy(rkc_mech *mech);

/* Sizes of a created mechanism: species, reactions, reaction units (pairs
 * plus unpaired reactions) and nonzero stoichiometric entries of the net
 * production sum (E:spec-rate).  Any pointer may be NULL. */
int rkc_mech_info(const rkc_mech *mech, int32_t *n_species, int32_t *n_reactions,
                  int32_t *n_units, int32_t *nnz);

/* Source term f(y) of E:mass and E:energy for n cells:
 *   T [n], P [n], Y [n][n_species]  ->  f [n][n_species + 1]
 * with f[i][0] = dT/dt and f[i][1 + k] = dY_k/dt.  Same lane-group variants
 * as rkc_integrate (opts->lanes_per_cell).  n = 0 is a no-op. */
int rkc_rhs(const rkc_mech *mech, size_t n, const double *T, const double *P,
            const double *Y, double *f, const rkc_opts *opts);

/* Integrate every cell from 0 to dt at constant pressure.
 *   T [n_cells]               in: initial temperature; out: temperature at dt
 *   P [n_cells]               pressure, unchanged
 *   Y [n_cells][n_species]    in: initial mass fractions; out: at dt
 *   dt > 0, rtol > 0, atol >= 0   (RKCK uses rtol as its tolerance and ignores atol)
 *   cell_status [n_cells]     optional per-cell RKC_CELL_* codes
 *   stats                     optional aggregate statistics (synchronises)
 * A failed cell keeps its last accepted state (its input for BADINPUT) and
 * never affects other cells.  Results of a cell do not depend on the
 * schedule, the workgroup size, the grid size or the other cells in the call;
 * they depend on lanes_per_cell only through summation order (rounding).
 * Returns RKC_OK, RKC_ECELLS (some cell failed; only known when the call
 * synchronises, i.e. host arrays or stats != NULL), RKC_EINVAL, RKC_ENOTSUP,
 * RKC_ENOMEM or RKC_EDEVICE.  n_cells = 0 is a no-op. */
int rkc_integrate(const rkc_mech *mech, size_t n_cells, double *T, const double *P,
                  double *Y, double dt, double rtol, double atol, const rkc_opts *opts,
                  int32_t *cell_status, rkc_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * rkc_integrate with device arrays (opts->device_ptrs must be 1, opts must not
 * be NULL) that calls no hipMalloc, hipFree or other allocating routine.  The
 * launch's scratch -- the aggregate counters and the work-queue head of the
 * kernels, 256 bytes -- is a file-scope device array of the library, one per
 * GPU, cleared by a kernel at the start of every call; the call's size limit is
 * that of rkc_integrate (RKC_MAX_CELLS cells, RKC_ENOTSUP above).  Results are
 * those of rkc_integrate with the same options.  The mechanism's tables for the
 * kernel variant these options select are built by the first ordinary call
 * (rkc_integrate, rkc_rhs or rkc_graph_create with the same lanes_per_cell and
 * param_placement); before that this call returns RKC_ENOTSUP and does
 * nothing.  The work is enqueued on opts->stream and the call returns without
 * waiting; statistics are not available (use rkc_integrate for them).  Calls
 * on one GPU share its scratch: calls that overlap in time on one GPU race
 * (the same rule as calls sharing a mechanism handle).  Errors: RKC_EINVAL
 * (host arrays, NULL, bad scalars), RKC_ENOTSUP, RKC_EDEVICE. */
int rkc_integrate_device_noalloc(const rkc_mech *mech, size_t n_cells, double *T,
                                 const double *P, double *Y, double dt, double rtol,
                                 double atol, const rkc_opts *opts, int32_t *cell_status);

/* Choose the kernel form and launch grain for a workload by timing it: runs
 * rkc_integrate over the given cells (left unchanged: the runs use internal
 * copies), each candidate twice after an untimed first run, keeping the
 * minimum.  Stage 1 times every lanes_per_cell the mechanism can run (1, 8, 16,
 * 32, 64; or the one requested in *opts) with every parameter placement that
 * has a compiled variant (or the one requested), persistent schedule; stage 2
 * times the two fastest with both schedules and workgroups of the largest, half
 * and a quarter of their lane groups (lanes for one lane per cell).  The fastest
 * setting is written into *tuned (lanes_per_cell, param_placement, schedule,
 * block_groups; every other field copied from *opts) and *best_ms (may be NULL)
 * receives its time.  Schedule, grain and placement never change results;
 * lanes_per_cell changes them by rounding only (summation order).  The choice
 * is cached in the mechanism handle by (method, requested lanes_per_cell and
 * param_placement, layout, floor(log2 n_cells)): a later call with the same key
 * returns it without timing.  A sample of the real cells is the intended input.
 * Arrays are host or device pointers per opts->device_ptrs; opts may be NULL
 * (defaults).  Errors: RKC_EINVAL, RKC_ENOTSUP, RKC_ENOMEM, RKC_EDEVICE. */
int rkc_autotune(const rkc_mech *mech, size_t n_cells, const double *T, const double *P,
                 const double *Y, double dt, double rtol, double atol, const rkc_opts *opts,
                 rkc_opts *tuned, float *best_ms);

/* Record the device work of one rkc_integrate call with device arrays as a
 * HIP graph, for repeated launches with the same arrays and sizes (one
 * replay = one global step, as in the paper's repeated global steps of
 * Sec. 3).  opts->device_ptrs must be 1 and every array (T, P, Y,
 * cell_status, opts->cell_counters) stays bound to the graph, which owns its
 * own scratch: replays never share state with other calls on the handle.
 * Mechanism tables and launch attributes are prepared before recording, so
 * nothing is allocated while recording; the graph holds no memset nodes.
 * Errors: RKC_EINVAL (host arrays, NULL, n_cells = 0, bad scalars),
 * RKC_ENOTSUP, RKC_ENOMEM, RKC_EDEVICE. */
int rkc_graph_create(const rkc_mech *mech, size_t n_cells, double *T, const double *P,
                     double *Y, double dt, double rtol, double atol, const rkc_opts *opts,
                     int32_t *cell_status, rkc_graph **out);

/* Enqueue one replay on stream (hipStream_t, NULL = null stream). */
int rkc_graph_launch(rkc_graph *graph, void *stream);

/* Release a graph; NULL is accepted. */
int rkc_graph_destroy(rkc_graph *graph);

/* Divergence measure D of Sec. 3.1 (results section, divergence of GPU
 * threads), for runs of `width` consecutive cells:
 *   D_r = (sum_{i in run r} d_i) / (c_r * max_{i in run r} d_i),
 * d_i = work[i * stride] >= 0 the work of cell i (the paper uses its number of
 * source-term evaluations, e.g. the RKC_CNT_RHS column of cell_counters with
 * stride RKC_NCOUNTERS, or a per-cell sum over several global steps with
 * stride 1), c_r = width except for a shorter last run, and D_r = 1 when every
 * d_i of the run is 0.  width 32 is the paper's warp; 64 a wavefront of
 * cells.  D = 1 means equal work, D -> 1/c_r one cell doing all of it.
 *   D [ceil(n_cells / width)] output.
 * Arrays are host pointers unless opts->device_ptrs (then device pointers,
 * enqueued on opts->stream); opts may be NULL.  Runs on the current device.
 * Returns RKC_OK, RKC_EINVAL (stride or width < 1, NULL array), RKC_ENOMEM,
 * RKC_ENOTSUP (n_cells above RKC_MAX_CELLS) or RKC_EDEVICE; n_cells = 0 is a no-op. */
int rkc_divergence(size_t n_cells, const int32_t *work, int32_t stride, int32_t width,
                   double *D, const rkc_opts *opts);

/* Static string for a return code. */
const char *rkc_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RKC_H */
