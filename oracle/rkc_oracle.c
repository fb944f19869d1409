/*
 * Serial FP64 CPU oracle for the batched chemical-kinetics integrator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the HIP library.
 *
 * Method: Niemeyer & Sung, "Accelerating moderately stiff chemical kinetics in
 * reactive-flow simulations using GPUs".
 *   - Source terms: Sec. 2.2, Eqs. (E:mass), (E:spec-rate), (E:rxn-rate),
 *     (E:rxn-const), (E:energy); state y = {T, Y_1..Y_nS}, N = nS + 1.
 *   - RKCK: Sec. 2.3, Table 1 coefficients, error scale Delta_0 and step
 *     formula (E:hnew) with S = 0.9, growth <= 5x, shrink >= 0.1x.
 *   - RKC: Sec. 2.4, stage recurrence (E:rkc0)-(E:rkcs), coefficient formulas,
 *     error estimate and weighted RMS norm (E:rmsE), step-size controller,
 *     initial step, stage count, nonlinear power method for the spectral radius.
 *
 * Readings where the paper is silent or garbled:
 *   b_1 = 1/omega_0 as printed; a_j = 1 - b_j T_j(omega_0); stage count is
 *   1 + floor(sqrt(1 + 1.54 h sigma)), capped at s_max; predictive controller
 *   0.8 (h_n/h_{n-1}) err_n^{1/3} / err_{n+1}^{2/3}, non-predictive 0.8/err^{1/3}
 *   on the first step and after a rejection; initial tentative step capped at
 *   dt; power method with delta = sqrt(u)|y|, 1% stopping test, at most 50
 *   iterations, safety factor 1.2, re-estimated every 25 accepted steps and
 *   after every rejection, warm-started from the saved direction; scalar atol
 *   for every component; the last step lands exactly on dt; RKCK uses the
 *   largest |Delta_i / Delta_0,i| (the standard reading of Press et al.); a
 *   trial step whose error estimate is not finite is rejected with the
 *   largest shrink factor 0.1; status NONFINITE is reserved for a non-finite
 *   f(y0) or spectral radius.
 *
 * Units: P in Pa (x10 -> dyn/cm^2), W g/mol, rho g/cm^3, C mol/cm^3,
 * A (cm^3/mol)^(m-1)/s, Ea J/mol, enthalpy and heat capacity in J.
 *
 * Parity pins live in tests/test_oracle_*.py.  Build: gcc -O2 -ffp-contract=off
 * -fno-fast-math -shared -fPIC (see oracle/build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define R_J   8.31446261815324      /* J/(mol K) */
#define R_ERG 8.31446261815324e7    /* erg/(mol K) */

enum { ORC_OK = 0, ORC_UNDERFLOW = 1, ORC_MAXSTEPS = 2, ORC_NONFINITE = 3, ORC_BADINPUT = 4 };
enum { ORC_RKC = 0, ORC_RKCK = 1 };

typedef struct {
    int n_species, n_reactions;
    const double *W;          /* [nS] g/mol */
    const double *nasa_low;   /* [nS][7] */
    const double *nasa_high;  /* [nS][7] */
    const double *T_mid;      /* [nS] K */
    const int32_t *reac;      /* [nR][3] species index with repetition, -1 empty */
    const int32_t *prod;      /* [nR][3] */
    const double *A, *beta, *Ea;  /* [nR] */
    /* Pressure dependence (Sec. 2.2 after E:rxn-rate: third-body and falloff
     * reactions in the Chemkin formulation the paper refers to).  Any pointer
     * may be NULL: no reaction of that kind.
     *   pdep [nR]      0 plain, 1 third body, 2 Lindemann falloff, 3 Troe falloff
     *   eff  [nR][nS]  third-body efficiencies alpha (NULL: all 1)
     *   A0, beta0, Ea0 [nR]  low-pressure limit k_0 of falloff reactions
     *   troe [nR][4]   a, T3, T1, T2 (the Troe temperatures; T2 <= 0: its term
     *                  absent) */
    const int32_t *pdep;
    const double *eff;
    const double *A0, *beta0, *Ea0;
    const double *troe;
} orc_mech;

/* Per-species list of (reaction, nu'' - nu') with nonzero coefficient, in
 * increasing reaction index: the nonzero terms of the sum in (E:spec-rate). */
typedef struct {
    orc_mech m;
    int *row;      /* [nS+1] */
    int *rxn;      /* [nnz] */
    int *dnu;      /* [nnz] */
} orc_model;

typedef struct {
    int32_t n_rhs, n_steps, n_reject, n_sigma, s_max_used, s_hash, status, n_power_iter;
} orc_counters;

/* One attempted step, for the pins of the step-size control (test use):
 * t and h of the attempt, the stage count s (RKC; 0 for RKCK), the error
 * measure (RKC: weighted RMS norm of E:rmsE; RKCK: the largest
 * |Delta_i / Delta_0,i|), the spectral radius estimate in use (RKC), whether
 * the estimate was recomputed just before this attempt, whether the attempt
 * was accepted, and the first three state components after it (the accepted
 * state; on rejection the state the attempt started from). */
typedef struct {
    double t, h, err, sigma;
    double y[3];
    int32_t s, new_sigma, accepted, pad;
} orc_step;

typedef struct {
    orc_step *buf;
    int cap, n;
} orc_trace;

static void trace_put(orc_trace *tr, double t, double h, double err, double sigma, int s,
                      int new_sigma, int accepted, const double *y, int N) {
    if (!tr || tr->n >= tr->cap) { if (tr) tr->n += 1; return; }
    orc_step *e = &tr->buf[tr->n++];
    e->t = t; e->h = h; e->err = err; e->sigma = sigma;
    for (int i = 0; i < 3; ++i) e->y[i] = (i < N) ? y[i] : 0.0;
    e->s = s; e->new_sigma = new_sigma; e->accepted = accepted; e->pad = 0;
}

static int count_in(const int32_t *slots, int sp) {
    int c = 0;
    for (int s = 0; s < 3; ++s) c += (slots[s] == sp);
    return c;
}

orc_model *orc_model_create(const orc_mech *m) {
    orc_model *md = (orc_model *)calloc(1, sizeof(orc_model));
    md->m = *m;
    int nS = m->n_species, nR = m->n_reactions;
    md->row = (int *)calloc((size_t)nS + 1, sizeof(int));
    int nnz = 0;
    for (int i = 0; i < nS; ++i)
        for (int j = 0; j < nR; ++j)
            if (count_in(m->prod + 3 * j, i) - count_in(m->reac + 3 * j, i) != 0) ++nnz;
    md->rxn = (int *)malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    md->dnu = (int *)malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    int e = 0;
    for (int i = 0; i < nS; ++i) {
        md->row[i] = e;
        for (int j = 0; j < nR; ++j) {
            int d = count_in(m->prod + 3 * j, i) - count_in(m->reac + 3 * j, i);
            if (d != 0) { md->rxn[e] = j; md->dnu[e] = d; ++e; }
        }
    }
    md->row[nS] = e;
    return md;
}

void orc_model_destroy(orc_model *md) {
    if (!md) return;
    free(md->row); free(md->rxn); free(md->dnu); free(md);
}

/* ---------------------------------------------------------------- RHS ---- */

/* Scratch for one RHS evaluation. */
typedef struct { double *C, *omega, *Omega; } rhs_ws;

/* Troe broadening factor F(T, Pr) (Chemkin form), with the three Troe
 * temperatures written T3 (T-triple-star), T1 (T-star) and T2 (T-double-star):
 *   F_cent = (1 - a) exp(-T / T3) + a exp(-T / T1) + exp(-T2 / T)
 *   c = -0.4 - 0.67 log10 F_cent, n = 0.75 - 1.27 log10 F_cent, d = 0.14
 *   log10 F = log10 F_cent / (1 + ((log10 Pr + c) / (n - d (log10 Pr + c)))^2) */
static double troe_F(double T, double Pr, const double *t) {
    const double a = t[0], T3 = t[1], T1 = t[2], T2 = t[3];
    double Fc = (1.0 - a) * exp(-T / T3) + a * exp(-T / T1);
    if (T2 > 0.0) Fc += exp(-T2 / T);
    const double lFc = log10(Fc);
    const double c = -0.4 - 0.67 * lFc;
    const double n = 0.75 - 1.27 * lFc;
    const double x = log10(Pr) + c;
    const double f1 = x / (n - 0.14 * x);
    return pow(10.0, lFc / (1.0 + f1 * f1));
}

/* f(y) for the constant-pressure adiabatic kinetics system, Sec. 2.2. */
static void rhs_eval(const orc_model *md, double P, const double *y, double *f, rhs_ws *ws) {
    const orc_mech *m = &md->m;
    const int nS = m->n_species, nR = m->n_reactions;
    const double T = y[0];
    const double *Y = y + 1;

    /* mixture density from the ideal gas law: rho = P Wbar / (R T) */
    double sumYW = 0.0;
    for (int i = 0; i < nS; ++i) sumYW += Y[i] / m->W[i];
    const double P_cgs = P * 10.0;
    const double rho = P_cgs / (R_ERG * T * sumYW);
    for (int i = 0; i < nS; ++i) ws->C[i] = rho * Y[i] / m->W[i];

    /* (E:rxn-const) and (E:rxn-rate) */
    for (int j = 0; j < nR; ++j) {
        double k = m->A[j] * pow(T, m->beta[j]) * exp(-m->Ea[j] / (R_J * T));
        const int kind = m->pdep ? m->pdep[j] : 0;
        if (kind != 0) {
            /* third-body concentration [M] = sum_i alpha_ji C_i */
            double M = 0.0;
            for (int i = 0; i < nS; ++i) M += (m->eff ? m->eff[(size_t)j * nS + i] : 1.0) * ws->C[i];
            if (kind == 1) {
                k = k * M;
            } else {
                /* falloff: k = k_inf Pr / (1 + Pr) F, Pr = k_0 [M] / k_inf */
                const double k0 = m->A0[j] * pow(T, m->beta0[j]) * exp(-m->Ea0[j] / (R_J * T));
                if (k == 0.0 || k0 * M == 0.0) {
                    k = 0.0;
                } else {
                    const double Pr = k0 * M / k;
                    const double F = (kind == 3) ? troe_F(T, Pr, m->troe + 4 * (size_t)j) : 1.0;
                    k = k * (Pr / (1.0 + Pr)) * F;
                }
            }
        }
        double Om = k;
        for (int s = 0; s < 3; ++s) {
            int sp = m->reac[3 * j + s];
            if (sp >= 0) Om = Om * ws->C[sp];
        }
        ws->Omega[j] = Om;
    }
    /* (E:spec-rate): omega_i = sum_j (nu''_ij - nu'_ij) Omega_j, j ascending */
    for (int i = 0; i < nS; ++i) {
        double w = 0.0;
        for (int e = md->row[i]; e < md->row[i + 1]; ++e)
            w += (double)md->dnu[e] * ws->Omega[md->rxn[e]];
        ws->omega[i] = w;
    }
    /* (E:mass) */
    for (int i = 0; i < nS; ++i) f[1 + i] = m->W[i] * ws->omega[i] / rho;

    /* (E:energy) with NASA-7 polynomials; high range iff T >= T_mid */
    double cp = 0.0, sum_h = 0.0;
    for (int i = 0; i < nS; ++i) {
        const double *a = (T >= m->T_mid[i]) ? m->nasa_high + 7 * i : m->nasa_low + 7 * i;
        double cp_R = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        double h_RT = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
                    + a[4] * T * T * T * T / 5.0 + a[5] / T;
        double Cp_molar = R_J * cp_R;          /* J/(mol K) */
        double H_molar = R_J * T * h_RT;       /* J/mol */
        double cp_i = Cp_molar / m->W[i];      /* J/(g K) */
        double h_i = H_molar / m->W[i];        /* J/g */
        cp += Y[i] * cp_i;
        sum_h += h_i * ws->omega[i] * m->W[i];
    }
    f[0] = -sum_h / (rho * cp);
}

static rhs_ws ws_alloc(const orc_mech *m) {
    rhs_ws w;
    w.C = (double *)malloc(sizeof(double) * (size_t)m->n_species);
    w.omega = (double *)malloc(sizeof(double) * (size_t)m->n_species);
    w.Omega = (double *)malloc(sizeof(double) * (size_t)(m->n_reactions > 0 ? m->n_reactions : 1));
    return w;
}
static void ws_free(rhs_ws *w) { free(w->C); free(w->omega); free(w->Omega); }

/* Public: f(y) for n cells; y and f are [n][N]. */
void orc_rhs(const orc_model *md, int n, const double *P, const double *y, double *f) {
    const int N = md->m.n_species + 1;
    rhs_ws ws = ws_alloc(&md->m);
    for (int c = 0; c < n; ++c) rhs_eval(md, P[c], y + (size_t)c * N, f + (size_t)c * N, &ws);
    ws_free(&ws);
}

/* ------------------------------------------------- RKC coefficients ---- */

/* Coefficients of the s-stage RKC method (Sec. 2.4), kappa = 2/13.
 * Fills mu_t[1..s], mu[2..s], nu[2..s], gam_t[2..s] (index 0 unused). */
void orc_rkc_coeffs(int s, double *mu_t, double *mu, double *nu, double *gam_t) {
    const double kappa = 2.0 / 13.0;
    double *Tc = (double *)malloc(sizeof(double) * (size_t)(s + 1));
    double *Tp = (double *)malloc(sizeof(double) * (size_t)(s + 1));
    double *Tpp = (double *)malloc(sizeof(double) * (size_t)(s + 1));
    double *b = (double *)malloc(sizeof(double) * (size_t)(s + 1));
    double *a = (double *)malloc(sizeof(double) * (size_t)(s + 1));
    const double w0 = 1.0 + kappa / ((double)s * (double)s);
    /* Chebyshev polynomials of the first kind and their derivatives at w0 */
    Tc[0] = 1.0; Tc[1] = w0;
    Tp[0] = 0.0; Tp[1] = 1.0;
    Tpp[0] = 0.0; Tpp[1] = 0.0;
    for (int j = 2; j <= s; ++j) {
        Tc[j] = 2.0 * w0 * Tc[j - 1] - Tc[j - 2];
        Tp[j] = 2.0 * w0 * Tp[j - 1] - Tp[j - 2] + 2.0 * Tc[j - 1];
        Tpp[j] = 2.0 * w0 * Tpp[j - 1] - Tpp[j - 2] + 4.0 * Tp[j - 1];
    }
    const double w1 = Tp[s] / Tpp[s];
    for (int j = 2; j <= s; ++j) b[j] = Tpp[j] / (Tp[j] * Tp[j]);
    b[1] = 1.0 / w0;
    b[0] = (s >= 2) ? b[2] : 0.0;
    for (int j = 0; j <= s; ++j) a[j] = 1.0 - b[j] * Tc[j];
    mu_t[1] = b[1] * w1;
    for (int j = 2; j <= s; ++j) {
        mu[j] = 2.0 * b[j] * w0 / b[j - 1];
        nu[j] = -b[j] / b[j - 2];
        mu_t[j] = 2.0 * b[j] * w1 / b[j - 1];
        gam_t[j] = -a[j - 1] * mu_t[j];
    }
    free(Tc); free(Tp); free(Tpp); free(b); free(a);
}

/* ---------------------------------------------------------- helpers ---- */

static double norm2(const double *v, int N) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += v[i] * v[i];
    return sqrt(s);
}

static int all_finite(const double *v, int N) {
    for (int i = 0; i < N; ++i) if (!isfinite(v[i])) return 0;
    return 1;
}

typedef struct {
    const orc_model *md; double P; rhs_ws ws; int N; orc_counters *cnt;
} ctx_t;

static void F(ctx_t *c, const double *y, double *f) {
    rhs_eval(c->md, c->P, y, f, &c->ws);
    c->cnt->n_rhs += 1;
}

/* Nonlinear power method for the spectral radius of the Jacobian at y, using
 * differences of f only.  v is the starting direction on entry and receives
 * the last difference direction on exit.  Returns 1.2 * sigma. */
static double power_sigma(ctx_t *c, const double *y, const double *fy, double *v,
                          double *z, double *fz, double *g) {
    const int N = c->N;
    const double u = ldexp(1.0, -53);
    const double sqrt_u = sqrt(u);
    double ny = norm2(y, N);
    double delta = (ny > 0.0) ? sqrt_u * ny : sqrt_u;
    double nv = norm2(v, N);
    if (!(nv > 0.0)) {
        for (int i = 0; i < N; ++i) v[i] = 1.0;
        nv = norm2(v, N);
    }
    for (int i = 0; i < N; ++i) z[i] = y[i] + (delta / nv) * v[i];
    double sigma = 0.0, sigma_prev = 0.0;
    for (int k = 1; k <= 50; ++k) {
        F(c, z, fz);
        c->cnt->n_power_iter += 1;
        for (int i = 0; i < N; ++i) g[i] = fz[i] - fy[i];
        double ng = norm2(g, N);
        double dz = 0.0;
        for (int i = 0; i < N; ++i) { double d = z[i] - y[i]; dz += d * d; }
        dz = sqrt(dz);
        sigma = ng / dz;
        if (k >= 2 && fabs(sigma - sigma_prev) <= 0.01 * sigma) break;
        if (ng == 0.0) { sigma = 0.0; break; }
        if (k == 50) break;
        for (int i = 0; i < N; ++i) z[i] = y[i] + (delta / ng) * g[i];
        sigma_prev = sigma;
    }
    for (int i = 0; i < N; ++i) v[i] = z[i] - y[i];
    c->cnt->n_sigma += 1;
    return 1.2 * sigma;
}

static double rms_err(const double *d, const double *y0, const double *y1, double rtol,
                      double atol, int N) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        double m = fabs(y0[i]);
        double m1 = fabs(y1[i]);
        if (m1 > m) m = m1;
        double w = atol + rtol * m;
        double q = d[i] / w;
        s += q * q;
    }
    return sqrt(s / (double)N);
}

static int bad_input(const double *y, double P, int N) {
    if (!isfinite(P) || !(P > 0.0)) return 1;
    if (!isfinite(y[0]) || !(y[0] > 0.0)) return 1;
    return !all_finite(y, N);
}

static void hash_s(orc_counters *cnt, int s) {
    cnt->s_hash = (int32_t)((uint32_t)cnt->s_hash * 31u + (uint32_t)s);
    if (s > cnt->s_max_used) cnt->s_max_used = s;
}

/* ---------------------------------------------------------------- RKC ---- */

/* Integrate one cell over [0, dt] with RKC; y (length N) is overwritten.
 * tr (may be NULL) receives every attempted step. */
static int rkc_cell(const orc_model *md, double P, double *y, double dt, double rtol,
                    double atol, int s_max, int max_steps, orc_counters *cnt, orc_trace *tr) {
    const int N = md->m.n_species + 1;
    memset(cnt, 0, sizeof(*cnt));
    if (bad_input(y, P, N)) { cnt->status = ORC_BADINPUT; return ORC_BADINPUT; }
    ctx_t c; c.md = md; c.P = P; c.ws = ws_alloc(&md->m); c.N = N; c.cnt = cnt;
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 10);
    double *f0 = buf, *f1 = buf + N, *v = buf + 2 * N, *z = buf + 3 * N, *fz = buf + 4 * N;
    double *g = buf + 5 * N, *wm1 = buf + 6 * N, *wm2 = buf + 7 * N, *wj = buf + 8 * N;
    double *del = buf + 9 * N;
    double *cm = (double *)malloc(sizeof(double) * 4 * (size_t)(s_max + 1));
    double *mu_t = cm, *mu = cm + (s_max + 1), *nu = cm + 2 * (s_max + 1),
           *gam_t = cm + 3 * (s_max + 1);
    const double u = ldexp(1.0, -53);
    const double t_end = dt;
    const double h_min = 10.0 * u * t_end;
    int status = ORC_OK;

    F(&c, y, f0);
    if (!all_finite(f0, N)) { status = ORC_NONFINITE; goto done; }
    for (int i = 0; i < N; ++i) v[i] = f0[i];
    double sigma = power_sigma(&c, y, f0, v, z, fz, g);
    if (!isfinite(sigma)) { status = ORC_NONFINITE; goto done; }

    /* initial step: tentative 1/sigma, capped at dt */
    double ht = (sigma > 0.0) ? 1.0 / sigma : t_end;
    if (ht > t_end) ht = t_end;
    for (int i = 0; i < N; ++i) z[i] = y[i] + ht * f0[i];
    F(&c, z, fz);
    for (int i = 0; i < N; ++i) del[i] = ht * (fz[i] - f0[i]);
    double e0 = rms_err(del, y, y, rtol, atol, N);
    if (!isfinite(e0)) { status = ORC_NONFINITE; goto done; }
    double h = (e0 > 0.0) ? 0.1 * ht / sqrt(e0) : ht;
    if (h < h_min) h = h_min;
    if (h > t_end) h = t_end;

    double t = 0.0, h_prev = 0.0, err_prev = 0.0;
    int need_sigma = 0, since_sigma = 0, predictive = 0, fresh_sigma = 1;
    for (;;) {
        if (cnt->n_steps + cnt->n_reject >= max_steps) { status = ORC_MAXSTEPS; break; }
        if (need_sigma) {
            sigma = power_sigma(&c, y, f0, v, z, fz, g);
            if (!isfinite(sigma)) { status = ORC_NONFINITE; break; }
            need_sigma = 0;
            since_sigma = 0;
            fresh_sigma = 1;
        }
        const double t_attempt = t;
        int last = (h >= t_end - t);
        if (last) h = t_end - t;
        int s = 1 + (int)floor(sqrt(1.0 + 1.54 * h * sigma));
        if (s > s_max) {
            s = s_max;
            h = ((double)(s_max - 1) * (double)(s_max - 1) - 1.0) / (1.54 * sigma);
            last = 0;
        }
        hash_s(cnt, s);
        orc_rkc_coeffs(s, mu_t, mu, nu, gam_t);
        /* (E:rkc0), (E:rkc1) */
        for (int i = 0; i < N; ++i) {
            wm2[i] = y[i];
            wm1[i] = y[i] + mu_t[1] * h * f0[i];
        }
        /* (E:rkcj) */
        for (int j = 2; j <= s; ++j) {
            F(&c, wm1, fz);
            for (int i = 0; i < N; ++i)
                wj[i] = (1.0 - mu[j] - nu[j]) * y[i] + mu[j] * wm1[i] + nu[j] * wm2[i]
                      + mu_t[j] * h * fz[i] + gam_t[j] * h * f0[i];
            for (int i = 0; i < N; ++i) { wm2[i] = wm1[i]; wm1[i] = wj[i]; }
        }
        /* (E:rkcs): y_{n+1} = w_s, now in wm1 */
        F(&c, wm1, f1);
        for (int i = 0; i < N; ++i) del[i] = 0.8 * (y[i] - wm1[i]) + 0.4 * h * (f0[i] + f1[i]);
        double err = rms_err(del, y, wm1, rtol, atol, N);
        /* a trial step whose error is not finite is rejected with the largest shrink */
        const int accept = (err <= 1.0);
        trace_put(tr, t_attempt, h, err, sigma, s, fresh_sigma, accept, accept ? wm1 : y, N);
        fresh_sigma = 0;
        if (accept) {
            cnt->n_steps += 1;
            for (int i = 0; i < N; ++i) { y[i] = wm1[i]; f0[i] = f1[i]; }
            if (last) { t = t_end; break; }
            t = t + h;
            since_sigma += 1;
            need_sigma = (since_sigma >= 25);
            double fac;
            if (err == 0.0) fac = 10.0;
            else if (!predictive) fac = 0.8 * pow(err, -1.0 / 3.0);
            else fac = 0.8 * (h / h_prev) * pow(err_prev, 1.0 / 3.0) * pow(err, -2.0 / 3.0);
            if (fac > 10.0) fac = 10.0;
            if (fac < 0.1) fac = 0.1;
            h_prev = h;
            err_prev = err;
            predictive = 1;
            h = h * fac;
        } else {
            cnt->n_reject += 1;
            double fac = isfinite(err) ? 0.8 * pow(err, -1.0 / 3.0) : 0.1;
            if (fac < 0.1) fac = 0.1;
            h = h * fac;
            need_sigma = 1;
            predictive = 0;
        }
        if (h < h_min) { status = ORC_UNDERFLOW; break; }
    }
done:
    cnt->status = status;
    free(cm); free(buf); ws_free(&c.ws);
    return status;
}

int orc_rkc_cell(const orc_model *md, double P, double *y, double dt, double rtol,
                 double atol, int s_max, int max_steps, orc_counters *cnt) {
    return rkc_cell(md, P, y, dt, rtol, atol, s_max, max_steps, cnt, NULL);
}

/* RKC or RKCK on one cell with every attempted step recorded in trace[0..cap)
 * (*n_trace receives the number of attempts, which may exceed cap). */
int orc_cell_trace(const orc_model *md, int method, double P, double *y, double dt, double rtol,
                   double atol, int s_max, int max_steps, orc_counters *cnt, orc_step *trace,
                   int cap, int *n_trace);

/* --------------------------------------------------------------- RKCK ---- */

/* Table 1 of the paper, Cash & Karp 5(4). */
static const double ck_b21 = 1.0 / 5.0;
static const double ck_b31 = 3.0 / 40.0, ck_b32 = 9.0 / 40.0;
static const double ck_b41 = 3.0 / 10.0, ck_b42 = -9.0 / 10.0, ck_b43 = 6.0 / 5.0;
static const double ck_b51 = -11.0 / 54.0, ck_b52 = 5.0 / 2.0, ck_b53 = -70.0 / 27.0,
                    ck_b54 = 35.0 / 27.0;
static const double ck_b61 = 1631.0 / 55296.0, ck_b62 = 175.0 / 512.0,
                    ck_b63 = 575.0 / 13824.0, ck_b64 = 44275.0 / 110592.0,
                    ck_b65 = 253.0 / 4096.0;
static const double ck_c1 = 37.0 / 378.0, ck_c3 = 250.0 / 621.0, ck_c4 = 125.0 / 594.0,
                    ck_c6 = 512.0 / 1771.0;
static const double ck_cs1 = 2825.0 / 27648.0, ck_cs3 = 18575.0 / 48384.0,
                    ck_cs4 = 13525.0 / 55296.0, ck_cs5 = 277.0 / 14336.0, ck_cs6 = 1.0 / 4.0;

/* One RKCK step of size h from y with f(y) already known as k1/h; returns the
 * fifth-order solution in y5 and Delta = sum (c_i - c*_i) k_i in del. */
static void rkck_step(ctx_t *c, const double *y, double h, double *k, double *z,
                      double *y5, double *del) {
    const int N = c->N;
    double *k1 = k, *k2 = k + N, *k3 = k + 2 * N, *k4 = k + 3 * N, *k5 = k + 4 * N,
           *k6 = k + 5 * N;
    F(c, y, k1);
    for (int i = 0; i < N; ++i) k1[i] = h * k1[i];
    for (int i = 0; i < N; ++i) z[i] = y[i] + ck_b21 * k1[i];
    F(c, z, k2);
    for (int i = 0; i < N; ++i) k2[i] = h * k2[i];
    for (int i = 0; i < N; ++i) z[i] = y[i] + ck_b31 * k1[i] + ck_b32 * k2[i];
    F(c, z, k3);
    for (int i = 0; i < N; ++i) k3[i] = h * k3[i];
    for (int i = 0; i < N; ++i) z[i] = y[i] + ck_b41 * k1[i] + ck_b42 * k2[i] + ck_b43 * k3[i];
    F(c, z, k4);
    for (int i = 0; i < N; ++i) k4[i] = h * k4[i];
    for (int i = 0; i < N; ++i)
        z[i] = y[i] + ck_b51 * k1[i] + ck_b52 * k2[i] + ck_b53 * k3[i] + ck_b54 * k4[i];
    F(c, z, k5);
    for (int i = 0; i < N; ++i) k5[i] = h * k5[i];
    for (int i = 0; i < N; ++i)
        z[i] = y[i] + ck_b61 * k1[i] + ck_b62 * k2[i] + ck_b63 * k3[i] + ck_b64 * k4[i]
             + ck_b65 * k5[i];
    F(c, z, k6);
    for (int i = 0; i < N; ++i) k6[i] = h * k6[i];
    for (int i = 0; i < N; ++i) {
        y5[i] = y[i] + ck_c1 * k1[i] + ck_c3 * k3[i] + ck_c4 * k4[i] + ck_c6 * k6[i];
        del[i] = (ck_c1 - ck_cs1) * k1[i] + (0.0 - 0.0) * k2[i] + (ck_c3 - ck_cs3) * k3[i]
               + (ck_c4 - ck_cs4) * k4[i] + (0.0 - ck_cs5) * k5[i] + (ck_c6 - ck_cs6) * k6[i];
    }
}

static int rkck_cell(const orc_model *md, double P, double *y, double dt, double rtol,
                     int max_steps, orc_counters *cnt, orc_trace *tr) {
    const int N = md->m.n_species + 1;
    memset(cnt, 0, sizeof(*cnt));
    if (bad_input(y, P, N)) { cnt->status = ORC_BADINPUT; return ORC_BADINPUT; }
    ctx_t c; c.md = md; c.P = P; c.ws = ws_alloc(&md->m); c.N = N; c.cnt = cnt;
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 9);
    double *k = buf, *z = buf + 6 * N, *y5 = buf + 7 * N, *del = buf + 8 * N;
    const double u = ldexp(1.0, -53);
    const double t_end = dt;
    const double h_min = 10.0 * u * t_end;
    double t = 0.0, h = dt;
    int status = ORC_OK;
    for (;;) {
        if (cnt->n_steps + cnt->n_reject >= max_steps) { status = ORC_MAXSTEPS; break; }
        int last = (h >= t_end - t);
        if (last) h = t_end - t;
        rkck_step(&c, y, h, k, z, y5, del);
        /* largest |Delta_i / Delta_0,i|; any non-finite ratio makes the whole
         * estimate non-finite (the step is then rejected) */
        double errmax = 0.0;
        int nonfinite = 0;
        for (int i = 0; i < N; ++i) {
            double d0 = rtol * (fabs(y[i]) + fabs(k[i]) + 1e-30);
            double r = fabs(del[i] / d0);
            if (!isfinite(r)) nonfinite = 1;
            else if (r > errmax) errmax = r;
        }
        if (nonfinite) errmax = INFINITY;
        /* a trial step whose error is not finite is rejected with the largest shrink */
        trace_put(tr, t, h, errmax, 0.0, 0, 0, errmax <= 1.0, errmax <= 1.0 ? y5 : y, N);
        if (errmax <= 1.0) {
            cnt->n_steps += 1;
            for (int i = 0; i < N; ++i) y[i] = y5[i];
            if (last) { t = t_end; break; }
            t = t + h;
            double fac = (errmax == 0.0) ? 5.0 : 0.9 * pow(errmax, -0.2);
            if (fac > 5.0) fac = 5.0;
            h = h * fac;
        } else {
            cnt->n_reject += 1;
            double fac = isfinite(errmax) ? 0.9 * pow(errmax, -0.25) : 0.1;
            if (fac < 0.1) fac = 0.1;
            h = h * fac;
        }
        if (h < h_min) { status = ORC_UNDERFLOW; break; }
    }
    cnt->status = status;
    free(buf); ws_free(&c.ws);
    return status;
}

int orc_rkck_cell(const orc_model *md, double P, double *y, double dt, double rtol,
                  int max_steps, orc_counters *cnt) {
    return rkck_cell(md, P, y, dt, rtol, max_steps, cnt, NULL);
}

int orc_cell_trace(const orc_model *md, int method, double P, double *y, double dt, double rtol,
                   double atol, int s_max, int max_steps, orc_counters *cnt, orc_step *trace,
                   int cap, int *n_trace) {
    orc_trace tr = {trace, cap, 0};
    int st = (method == ORC_RKCK) ? rkck_cell(md, P, y, dt, rtol, max_steps, cnt, &tr)
                                  : rkc_cell(md, P, y, dt, rtol, atol, s_max, max_steps, cnt, &tr);
    if (n_trace) *n_trace = tr.n;
    return st;
}

/* ----------------------------------------------- fixed-step primitives ---- */
/* For convergence-order pins: one RKC step of given (h, s) or one RKCK step of
 * given h, no error control.  y is overwritten with the new state. */
void orc_rkc_fixed_step(const orc_model *md, double P, double *y, double h, int s) {
    const int N = md->m.n_species + 1;
    orc_counters cnt; memset(&cnt, 0, sizeof cnt);
    ctx_t c; c.md = md; c.P = P; c.ws = ws_alloc(&md->m); c.N = N; c.cnt = &cnt;
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 5);
    double *f0 = buf, *fz = buf + N, *wm1 = buf + 2 * N, *wm2 = buf + 3 * N, *wj = buf + 4 * N;
    double *cm = (double *)malloc(sizeof(double) * 4 * (size_t)(s + 1));
    double *mu_t = cm, *mu = cm + (s + 1), *nu = cm + 2 * (s + 1), *gam_t = cm + 3 * (s + 1);
    orc_rkc_coeffs(s, mu_t, mu, nu, gam_t);
    F(&c, y, f0);
    for (int i = 0; i < N; ++i) { wm2[i] = y[i]; wm1[i] = y[i] + mu_t[1] * h * f0[i]; }
    for (int j = 2; j <= s; ++j) {
        F(&c, wm1, fz);
        for (int i = 0; i < N; ++i)
            wj[i] = (1.0 - mu[j] - nu[j]) * y[i] + mu[j] * wm1[i] + nu[j] * wm2[i]
                  + mu_t[j] * h * fz[i] + gam_t[j] * h * f0[i];
        for (int i = 0; i < N; ++i) { wm2[i] = wm1[i]; wm1[i] = wj[i]; }
    }
    for (int i = 0; i < N; ++i) y[i] = wm1[i];
    free(cm); free(buf); ws_free(&c.ws);
}

void orc_rkck_fixed_step(const orc_model *md, double P, double *y, double h, double *y4) {
    const int N = md->m.n_species + 1;
    orc_counters cnt; memset(&cnt, 0, sizeof cnt);
    ctx_t c; c.md = md; c.P = P; c.ws = ws_alloc(&md->m); c.N = N; c.cnt = &cnt;
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 9);
    double *k = buf, *z = buf + 6 * N, *y5 = buf + 7 * N, *del = buf + 8 * N;
    rkck_step(&c, y, h, k, z, y5, del);
    for (int i = 0; i < N; ++i) { y4[i] = y5[i] - del[i]; y[i] = y5[i]; }
    free(buf); ws_free(&c.ws);
}

/* Spectral radius estimate at y (for pins on linear systems). */
double orc_sigma(const orc_model *md, double P, const double *y, int *n_iter) {
    const int N = md->m.n_species + 1;
    orc_counters cnt; memset(&cnt, 0, sizeof cnt);
    ctx_t c; c.md = md; c.P = P; c.ws = ws_alloc(&md->m); c.N = N; c.cnt = &cnt;
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 5);
    double *f0 = buf, *v = buf + N, *z = buf + 2 * N, *fz = buf + 3 * N, *g = buf + 4 * N;
    F(&c, y, f0);
    for (int i = 0; i < N; ++i) v[i] = f0[i];
    double s = power_sigma(&c, y, f0, v, z, fz, g);
    if (n_iter) *n_iter = cnt.n_power_iter;
    free(buf); ws_free(&c.ws);
    return s;
}

/* ------------------------------------------------------ batch driver ---- */

typedef struct {
    const orc_model *md; int method; int n; const double *P; double *T; double *Y;
    double dt, rtol, atol; int s_max, max_steps; orc_counters *cnt;
    int tid, nthreads;
} job_t;

static void *run_job(void *arg) {
    job_t *jb = (job_t *)arg;
    const int nS = jb->md->m.n_species, N = nS + 1;
    double *y = (double *)malloc(sizeof(double) * (size_t)N);
    for (int c = jb->tid; c < jb->n; c += jb->nthreads) {
        y[0] = jb->T[c];
        memcpy(y + 1, jb->Y + (size_t)c * nS, sizeof(double) * (size_t)nS);
        orc_counters cn;
        if (jb->method == ORC_RKCK)
            orc_rkck_cell(jb->md, jb->P[c], y, jb->dt, jb->rtol, jb->max_steps, &cn);
        else
            orc_rkc_cell(jb->md, jb->P[c], y, jb->dt, jb->rtol, jb->atol, jb->s_max,
                         jb->max_steps, &cn);
        /* a failed cell keeps its last accepted state */
        jb->T[c] = y[0];
        memcpy(jb->Y + (size_t)c * nS, y + 1, sizeof(double) * (size_t)nS);
        if (jb->cnt) jb->cnt[c] = cn;
    }
    free(y);
    return NULL;
}

/* Integrate n cells over [0, dt]; T[n] and Y[n][nS] are overwritten with the
 * state at dt, or with the last accepted state of a cell that failed.  Cells are split
 * over n_threads POSIX threads; the per-cell code is serial. */
void orc_integrate(const orc_model *md, int method, int n, const double *P, double *T,
                   double *Y, double dt, double rtol, double atol, int s_max, int max_steps,
                   orc_counters *cnt, int n_threads) {
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n) n_threads = n > 0 ? n : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    job_t *jobs = (job_t *)malloc(sizeof(job_t) * (size_t)n_threads);
    for (int t = 0; t < n_threads; ++t) {
        job_t j = {md, method, n, P, T, Y, dt, rtol, atol, s_max, max_steps, cnt, t, n_threads};
        jobs[t] = j;
    }
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
    run_job(&jobs[0]);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th); free(jobs);
}
