"""Seeded synthetic workloads: mechanisms, cell states and the served request trace.

The paper's mechanisms (hydrogen, H2/CO, GRI-Mech 3.0, USC Mech II) and its
ignition-sampled initial conditions (Sec. 3, "Results and discussion") are not
available, so every workload here is synthetic, seeded and reproducible.  The
sizes match the paper's four mechanisms: 9/38, 13/54, 53/634 and 111/1566
species/irreversible reactions.  Like the paper's converted mechanisms, the
reactions come as forward/reverse pairs: a reversible reaction with a random
forward Arrhenius rate is split into two irreversible ones, the reverse rate
coefficient k_f / K_c(T) being fitted with Arrhenius parameters at three
temperatures by the closed form of the paper's Appendix A.  The pairs are
therefore (to the accuracy of that fit) consistent with the mixture's
thermodynamics, and a cell relaxes toward chemical equilibrium.

This module only draws inputs.  It evaluates no right-hand side and integrates
nothing.  Besides the Appendix A fit (and the equilibrium constants it needs),
the one rate-like quantity it computes is a log-space upper bound of a
reaction's pseudo-first-order rate, used to reject parameter draws that would
make the system stiffer than a stated stage budget allows.

Units carried by every mechanism dict:
  W           g/mol
  A           (cm^3/mol)^(m-1) / s, m = number of reactant molecules
  beta        dimensionless temperature exponent
  Ea          J/mol
  nasa_low/high  NASA 7-coefficient polynomials, Cp/R, H/(R T) and S/R forms
  T_mid       K, switch between the low and high fit ranges
  reac, prod  [n_R][3] species indices with repetition (a species listed twice
              has stoichiometric coefficient 2); -1 marks an empty slot
States: T in K, P in Pa, Y mass fractions (rows sum to 1).
"""
from __future__ import annotations

import functools
import math

import numpy as np

R_J = 8.31446261815324          # J/(mol K)
R_ERG = 8.31446261815324e7      # erg/(mol K)
ATM = 101325.0                  # Pa

ATOMIC_WEIGHTS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "Ar": 39.948}

# Reactant / product molecularity distribution (1, 2 or 3 molecules per side).
_SIDE_SIZE_P = np.array([0.25, 0.60, 0.15])


def _compositions(elements, limits, max_atoms):
    """All nonzero element-count vectors over `elements` (Ar excluded) within limits."""
    mol_elems = [e for e in elements if e != "Ar"]
    ranges = [range(limits[e] + 1) for e in mol_elems]
    out = []
    for counts in np.ndindex(*[len(r) for r in ranges]):
        tot = sum(counts)
        if 0 < tot <= max_atoms:
            vec = [0] * len(elements)
            for e, c in zip(mol_elems, counts):
                vec[elements.index(e)] = c
            out.append(tuple(vec))
    return out


def _nasa_species(rng, inert=False):
    """Random two-range NASA-7 polynomials.

    Molar Cp stays within 20-60 J/(mol K) on 300-3500 K.  The low range equals
    the high range plus c (T - T_mid)^2, so Cp and dCp/dT are continuous at
    T_mid; a6 of the high range is fitted so H is continuous there too.
    Returns (low[7], high[7], T_mid, dHf_J).
    """
    T_mid = 1000.0
    if inert:
        hi = np.array([2.5, 0, 0, 0, 0, 0.0, 0.0])
        lo = hi.copy()
        hf = 0.0
        # H(298.15) = 0 and S(298.15)/R = 18.6 for the inert monatomic species
        lo[5] = -2.5 * 298.15
        hi[5] = lo[5]
        lo[6] = 18.6 - 2.5 * math.log(298.15)
        hi[6] = lo[6]
        return lo, hi, T_mid, hf
    Tg = np.linspace(300.0, 3500.0, 161)
    while True:
        base = rng.uniform(2.5, 4.0)
        d = rng.uniform(0.5, 2.0)
        e5 = rng.uniform(-0.01, 0.01) * d
        hi = np.zeros(7)
        hi[0] = base
        hi[1] = 1.2 * d / 1e3
        hi[2] = -0.5 * d / 1e6
        hi[3] = 0.08 * d / 1e9
        hi[4] = e5 / 1e12
        c = rng.uniform(-1.0, 1.0) * 1e-7
        lo = hi.copy()
        lo[0] += c * T_mid * T_mid
        lo[1] += -2.0 * c * T_mid
        lo[2] += c
        cp_hi = np.polyval(hi[4::-1], Tg)
        cp_lo = np.polyval(lo[4::-1], Tg)
        cp = np.where(Tg >= T_mid, cp_hi, cp_lo) * R_J
        if cp.min() >= 20.0 and cp.max() <= 60.0:
            break
    hf = rng.uniform(-1.5e5, 1.5e5)

    def hint(a, T):  # integral of Cp/R dT without the constant
        return a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5

    lo[5] = hf / R_J - hint(lo, 298.15)
    hi[5] = lo[5] + hint(lo, T_mid) - hint(hi, T_mid)

    def sint(a, T):  # integral of Cp/(R T) dT without the constant
        return a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4

    s298 = rng.uniform(20.0, 35.0)      # standard entropy S(298.15)/R
    lo[6] = s298 - sint(lo, 298.15)
    hi[6] = lo[6] + sint(lo, T_mid) - sint(hi, T_mid)
    return lo, hi, T_mid, hf


def gibbs_RT(nasa_low, nasa_high, T_mid, T):
    """G/(R T) = H/(R T) - S/R of every species at temperature T (NASA-7)."""
    out = np.empty(len(T_mid))
    for i in range(len(T_mid)):
        a = nasa_high[i] if T >= T_mid[i] else nasa_low[i]
        h = a[0] + a[1] * T / 2 + a[2] * T**2 / 3 + a[3] * T**3 / 4 + a[4] * T**4 / 5 + a[5] / T
        s_ = a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4 + a[6]
        out[i] = h - s_
    return out


def ln_kc(dnu, g_rt, T):
    """ln K_c of a reaction with net coefficients dnu (products minus reactants)
    at T: K_p = exp(-sum dnu G/(RT)), K_c = K_p (P_atm/(R T))^(sum dnu), cgs."""
    return -float(dnu @ g_rt) + float(dnu.sum()) * math.log(ATM * 10.0 / (R_ERG * T))


def fit_three_point(T3, lnk3):
    """Arrhenius parameters (ln A, beta, T_a = E/R) through three (T, ln k) points:
    the closed form of the paper's Appendix A (Eqs. e:beta_r, e:Tar and ln A_r)."""
    T1, T2, T3_ = T3
    a1, a2, a3 = lnk3
    x1, x2, x3 = math.log(T1), math.log(T2), math.log(T3_)
    D = x1 * T1 * (T3_ - T2) + x2 * T2 * (T1 - T3_) + x3 * T3_ * (T2 - T1)
    beta = (a1 * T1 * (T3_ - T2) + a2 * T2 * (T1 - T3_) + a3 * T3_ * (T2 - T1)) / D
    Ta = T1 * T2 * T3_ * (a1 * (x2 - x3) + a2 * (x3 - x1) + a3 * (x1 - x2)) / D
    lnA = (a1 * T1 * (x2 * T2 - x3 * T3_) + a2 * T2 * (x3 * T3_ - x1 * T1)
           + a3 * T3_ * (x1 * T1 - x2 * T2)) / D
    return lnA, beta, Ta


def _ln_rate_bound(lnA, beta, Ea, m, T, P_pa):
    """ln of m * k(T) * C_tot(T)^(m-1), the pseudo-first-order rate bound."""
    ln_ctot = math.log(P_pa * 10.0) - math.log(R_ERG) - np.log(T)
    return math.log(m) + lnA + beta * np.log(T) - Ea / (R_J * T) + (m - 1) * ln_ctot


def make_mechanism(n_species, n_reactions, elements, seed, *, ea_max=2e5,
                   T_lo=800.0, T_hi=2200.0, P_max=ATM, dt=1e-6, s_target=30,
                   limits=None, max_atoms=6, name=None):
    """Seeded, element-balanced mechanism of forward/reverse reaction pairs.

    Arrhenius draws: log10 A ~ U(6, 14), beta ~ U(-2, 2), Ea ~ U(0, ea_max).
    A draw is rejected (and redrawn) while its rate bound on [T_lo, T_hi] at
    P_max exceeds lambda_cap = ((s_target-1)^2 - 1) / (1.54 dt), the spectral
    radius whose RKC stage count over one full step dt is s_target.
    """
    assert n_reactions % 2 == 0, "reactions come as forward/reverse pairs"
    rng = np.random.Generator(np.random.PCG64(seed))
    if limits is None:
        limits = {"C": 2, "H": 4, "O": 2, "N": 2}
    has_ar = "Ar" in elements
    comps = _compositions(elements, limits, max_atoms)
    n_mol = n_species - (1 if has_ar else 0)
    if len(comps) < n_mol:
        raise ValueError("not enough distinct compositions for %d species" % n_species)
    # prefer small molecules: weight 1/atoms^1.5
    w = np.array([1.0 / (sum(c) ** 1.5) for c in comps])
    w /= w.sum()
    mol_elems = [e for e in elements if e != "Ar"]
    for _ in range(1000):
        pick = rng.choice(len(comps), size=n_mol, replace=False, p=w)
        chosen = [comps[i] for i in pick]
        present = np.array(chosen).sum(axis=0)
        if all(present[elements.index(e)] > 0 for e in mol_elems):
            break
    else:
        raise RuntimeError("could not cover every element")
    if has_ar:
        ar = [0] * len(elements)
        ar[elements.index("Ar")] = 1
        chosen.append(tuple(ar))
    comp = np.array(chosen, dtype=np.int64)
    W = comp @ np.array([ATOMIC_WEIGHTS[e] for e in elements])

    nasa_low = np.zeros((n_species, 7))
    nasa_high = np.zeros((n_species, 7))
    T_mid = np.zeros(n_species)
    hf = np.zeros(n_species)
    for i in range(n_species):
        inert = has_ar and i == n_species - 1
        lo, hi, tm, h = _nasa_species(rng, inert=inert)
        nasa_low[i], nasa_high[i], T_mid[i], hf[i] = lo, hi, tm, h

    # index of multisets (sorted species tuples) of size 1..3 by composition
    index = {1: {}, 2: {}, 3: {}}
    for size in (1, 2, 3):
        for ms in _multisets(n_species, size):
            key = tuple(comp[list(ms)].sum(axis=0))
            index[size].setdefault(key, []).append(ms)

    n_pairs = n_reactions // 2
    lam_cap = ((s_target - 1) ** 2 - 1) / (1.54 * dt)
    ln_cap = math.log(lam_cap)
    Tg = np.linspace(T_lo, T_hi, 33)
    T_fit = (T_lo, math.sqrt(T_lo * T_hi), T_hi)
    g_fit = [gibbs_RT(nasa_low, nasa_high, T_mid, T) for T in T_fit]
    reac = np.full((n_reactions, 3), -1, dtype=np.int32)
    prod = np.full((n_reactions, 3), -1, dtype=np.int32)
    A = np.zeros(n_reactions)
    beta = np.zeros(n_reactions)
    Ea = np.zeros(n_reactions)

    def dnu_of(r_ms, p_ms):
        d = np.zeros(n_species)
        for sp in r_ms:
            d[sp] -= 1
        for sp in p_ms:
            d[sp] += 1
        return d

    def draw_params(r_ms, p_ms, tries):
        """Forward rate drawn from the configured distributions; the reverse
        rate k_f / K_c fitted at three temperatures (Appendix A closed form).
        Both must respect the stiffness cap.  None if no draw passes."""
        dnu = dnu_of(r_ms, p_ms)
        lnkc = [ln_kc(dnu, g_fit[q], T_fit[q]) for q in range(3)]
        for _ in range(tries):
            lA = rng.uniform(6.0, 14.0) * math.log(10.0)
            b = rng.uniform(-2.0, 2.0)
            e = rng.uniform(0.0, ea_max)
            if _ln_rate_bound(lA, b, e, len(r_ms), Tg, P_max).max() > ln_cap:
                continue
            lnkf = [lA + b * math.log(T) - e / (R_J * T) for T in T_fit]
            lAr, br, Tar = fit_three_point(T_fit, [lnkf[q] - lnkc[q] for q in range(3)])
            if not (-300.0 < lAr < 300.0):
                continue
            if _ln_rate_bound(lAr, br, Tar * R_J, len(p_ms), Tg, P_max).max() > ln_cap:
                continue
            return (math.exp(lA), b, e), (math.exp(lAr), br, Tar * R_J)
        return None

    pairs = set()
    guard = 0
    p = 0
    while p < n_pairs:
        guard += 1
        if guard > 200000:
            raise RuntimeError("could not draw enough distinct balanced reactions")
        m = 1 + rng.choice(3, p=_SIDE_SIZE_P)
        q = 1 + rng.choice(3, p=_SIDE_SIZE_P)
        r_ms = tuple(sorted(rng.choice(n_species, size=m, replace=True).tolist()))
        key = tuple(comp[list(r_ms)].sum(axis=0))
        cands = [c for c in index[q].get(key, []) if c != r_ms]
        if not cands:
            continue
        p_ms = cands[rng.integers(len(cands))]
        pk = (min(r_ms, p_ms), max(r_ms, p_ms))
        if pk in pairs:
            continue
        # write the thermodynamically favoured direction (K_c >= 1 at the
        # middle fit temperature) first
        if ln_kc(dnu_of(r_ms, p_ms), g_fit[1], T_fit[1]) < 0.0:
            r_ms, p_ms = p_ms, r_ms
        got = draw_params(r_ms, p_ms, 2000)
        if got is None:
            continue
        pairs.add(pk)
        reac[2 * p, :len(r_ms)] = r_ms
        prod[2 * p, :len(p_ms)] = p_ms
        reac[2 * p + 1, :len(p_ms)] = p_ms
        prod[2 * p + 1, :len(r_ms)] = r_ms
        (A[2 * p], beta[2 * p], Ea[2 * p]), (A[2 * p + 1], beta[2 * p + 1], Ea[2 * p + 1]) = got
        p += 1
    msize = (reac >= 0).sum(axis=1)

    # keep at least 10 % of reactions active (rate >= 1e-3/dt at T_hi)
    ln_act = math.log(1e-3 / dt)

    def active(j):
        return _ln_rate_bound(math.log(A[j]), beta[j], Ea[j], msize[j],
                              np.array([T_hi]), P_max)[0] >= ln_act

    act = np.array([active(j) for j in range(n_reactions)])
    tries = 0
    while act.mean() < 0.10 and tries < 100 * n_reactions:
        j = 2 * (int(rng.choice(np.flatnonzero(~act))) // 2)
        tries += 1
        got = draw_params(tuple(x for x in reac[j] if x >= 0), tuple(x for x in prod[j] if x >= 0),
                          2000)
        if got is not None:
            (A[j], beta[j], Ea[j]), (A[j + 1], beta[j + 1], Ea[j + 1]) = got
            act[j], act[j + 1] = active(j), active(j + 1)

    names = []
    for i in range(n_species):
        s = "".join("%s%s" % (el, "" if c == 1 else c)
                    for el, c in zip(elements, comp[i]) if c > 0)
        names.append(s)
    return {
        "name": name or "synth_%dsp_%drx_seed%d" % (n_species, n_reactions, seed),
        "seed": seed,
        "n_species": n_species,
        "n_reactions": n_reactions,
        "elements": list(elements),
        "species": names,
        "comp": comp,
        "W": W,
        "nasa_low": nasa_low,
        "nasa_high": nasa_high,
        "T_mid": T_mid,
        "dHf": hf,
        "reac": reac,
        "prod": prod,
        "A": A,
        "beta": beta,
        "Ea": Ea,
        "lambda_cap": lam_cap,
        "T_fit": T_fit,
        "active_fraction": float(act.mean()),
    }


def _multisets(n, size):
    if size == 1:
        for a in range(n):
            yield (a,)
    elif size == 2:
        for a in range(n):
            for b in range(a, n):
                yield (a, b)
    else:
        for a in range(n):
            for b in range(a, n):
                for c in range(b, n):
                    yield (a, b, c)


def make_states(mech, n_cells, seed, *, T_dist, P_dist, Y_dist, order="shuffled"):
    """Seeded cell states.

    T_dist: ("uniform", lo, hi) | ("bimodal", m1, m2, sd)
    P_dist: ("const", P_pa) | ("uniform", lo_pa, hi_pa)
    Y_dist: ("dirichlet",) | ("majors", n_major, m_lo, m_hi)
    order:  "shuffled" (cells in random order, the paper's worst case) or
            "sorted" (by temperature, the paper's similar-neighbour case)
    Returns dict T[n], P[n], Y[n][n_S] (float64, C-contiguous).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nS = mech["n_species"]
    if T_dist[0] == "uniform":
        T = rng.uniform(T_dist[1], T_dist[2], size=n_cells)
    elif T_dist[0] == "bimodal":
        hot = rng.random(n_cells) < 0.5
        T = np.where(hot, rng.normal(T_dist[2], T_dist[3], n_cells),
                     rng.normal(T_dist[1], T_dist[3], n_cells))
    else:
        raise ValueError(T_dist)
    if P_dist[0] == "const":
        P = np.full(n_cells, float(P_dist[1]))
    else:
        P = rng.uniform(P_dist[1], P_dist[2], size=n_cells)
    if Y_dist[0] == "dirichlet":
        Y = rng.dirichlet(np.ones(nS), size=n_cells)
    elif Y_dist[0] == "majors":
        nm = Y_dist[1]
        majors = np.asarray(mech.get("major_species", list(range(nm))))
        minors = np.setdiff1d(np.arange(nS), majors)
        m = rng.uniform(Y_dist[2], Y_dist[3], size=n_cells)
        Y = np.zeros((n_cells, nS))
        Y[:, majors] = m[:, None] * rng.dirichlet(np.ones(nm), size=n_cells)
        Y[:, minors] = (1.0 - m)[:, None] * rng.dirichlet(np.ones(len(minors)), size=n_cells)
    else:
        raise ValueError(Y_dist)
    Y = Y / Y.sum(axis=1, keepdims=True)
    if order == "sorted":
        perm = np.argsort(T, kind="stable")
        T, P, Y = T[perm], P[perm], Y[perm]
    return {"T": np.ascontiguousarray(T, dtype=np.float64),
            "P": np.ascontiguousarray(P, dtype=np.float64),
            "Y": np.ascontiguousarray(Y, dtype=np.float64)}


# Workload configurations (mechanism seed 1000+k, state seed 2000+k).
CONFIGS = {
    "c1": dict(n_species=9, n_reactions=38, elements=["H", "O", "N"], mech_seed=1001,
               state_seed=2001, n_cells=1024, T=("uniform", 1000.0, 1500.0),
               P=("const", ATM), Y=("dirichlet",), dt=1e-6, rtol=1e-6, atol=1e-10,
               ea_max=2e5, T_range=(950.0, 1600.0), P_max=ATM, s_target=30,
               label="9sp/38rx, 1024 cells, dt 1e-6"),
    "c2": dict(n_species=13, n_reactions=54, elements=["H", "O", "C", "N"], mech_seed=1002,
               state_seed=2002, n_cells=262144, T=("uniform", 900.0, 1800.0),
               P=("uniform", ATM, 10 * ATM), Y=("dirichlet",), dt=1e-6, rtol=1e-6,
               atol=1e-10, ea_max=2e5, T_range=(850.0, 1900.0), P_max=10 * ATM,
               s_target=30, label="13sp/54rx, 262144 cells, dt 1e-6"),
    "c3": dict(n_species=53, n_reactions=634, elements=["H", "O", "C", "N", "Ar"],
               mech_seed=1003, state_seed=2003, n_cells=131072,
               T=("uniform", 800.0, 2200.0), P=("const", ATM), Y=("majors", 5, 0.90, 0.99),
               dt=1e-6, rtol=1e-6, atol=1e-10, ea_max=2e5, T_range=(750.0, 2300.0),
               P_max=ATM, s_target=30, label="53sp/634rx, 131072 cells, dt 1e-6"),
    # the 53-species set with pressure-dependent pairs (third body and falloff,
    # about 9 % each of the reaction pairs, as in GRI-Mech-sized mechanisms)
    "c3p": dict(n_species=53, n_reactions=634, elements=["H", "O", "C", "N", "Ar"],
                mech_seed=1003, pdep_seed=1103, pdep_frac=(0.09, 0.09), state_seed=2003,
                n_cells=131072, T=("uniform", 800.0, 2200.0), P=("const", ATM),
                Y=("majors", 5, 0.90, 0.99), dt=1e-6, rtol=1e-6, atol=1e-10, ea_max=2e5,
                T_range=(750.0, 2300.0), P_max=ATM, s_target=30,
                label="53sp/634rx with third-body and falloff pairs, 131072 cells, dt 1e-6"),
    "c4": dict(n_species=111, n_reactions=1566, elements=["H", "O", "C", "N", "Ar"],
               mech_seed=1004, state_seed=2004, n_cells=65536,
               T=("bimodal", 800.0, 2400.0, 20.0), P=("const", ATM), Y=("dirichlet",),
               dt=1e-5, rtol=1e-6, atol=1e-10, ea_max=3e5, T_range=(700.0, 2500.0),
               P_max=ATM, s_target=200, limits={"C": 3, "H": 8, "O": 3, "N": 2},
               max_atoms=8, label="111sp/1566rx, 65536 cells, dt 1e-5"),
    # the 111-species set with third-body and falloff pairs (as c3p)
    "c4p": dict(n_species=111, n_reactions=1566, elements=["H", "O", "C", "N", "Ar"],
                mech_seed=1004, pdep_seed=1104, pdep_frac=(0.09, 0.09), state_seed=2004,
                n_cells=65536, T=("bimodal", 800.0, 2400.0, 20.0), P=("const", ATM),
                Y=("dirichlet",), dt=1e-5, rtol=1e-6, atol=1e-10, ea_max=3e5,
                T_range=(700.0, 2500.0), P_max=ATM, s_target=200,
                limits={"C": 3, "H": 8, "O": 3, "N": 2}, max_atoms=8,
                label="111sp/1566rx with third-body and falloff pairs, 65536 cells, dt 1e-5"),
}


@functools.lru_cache(maxsize=None)
def _cached_mech(name):
    c = CONFIGS[name]
    kw = {}
    if "limits" in c:
        kw["limits"] = c["limits"]
        kw["max_atoms"] = c["max_atoms"]
    m = make_mechanism(c["n_species"], c["n_reactions"], c["elements"], c["mech_seed"],
                       ea_max=c["ea_max"], T_lo=c["T_range"][0], T_hi=c["T_range"][1],
                       P_max=c["P_max"], dt=c["dt"], s_target=c["s_target"],
                       name=name, **kw)
    if "pdep_seed" in c:
        m = add_pressure_dependence(m, c["pdep_seed"], c["pdep_frac"][0], c["pdep_frac"][1],
                                    T_ref=math.sqrt(c["T_range"][0] * c["T_range"][1]),
                                    P_ref=c["P_max"])
    if c["Y"][0] == "majors":
        rng = np.random.Generator(np.random.PCG64(c["mech_seed"] + 7))
        m["major_species"] = sorted(rng.choice(c["n_species"] - 1, size=c["Y"][1],
                                               replace=False).tolist())
    return m


PDEP_PLAIN, PDEP_THIRD_BODY, PDEP_LINDEMANN, PDEP_TROE = 0, 1, 2, 3


def add_pressure_dependence(mech, seed, frac_tb, frac_fo, *, T_ref, P_ref, n_sets=3):
    """A copy of a pair-structured mechanism in which a seeded fraction of the
    forward/reverse pairs become third-body pairs (rate k [M] prod C) and
    falloff pairs (Lindemann or Troe), the pressure-dependent forms the paper
    also evaluates (Sec. 2.2, after E:rxn-rate; Chemkin conventions).

    Added keys: pdep [nR] (0 plain, 1 third body, 2 Lindemann, 3 Troe),
    eff [nR][nS] third-body efficiencies (n_sets distinct vectors: six species
    with efficiency in {0.7, 1.5, 2, 3, 6, 12}, the rest 1), A0/beta0/Ea0 [nR]
    low-pressure limits, troe [nR][4] (a, T***, T*, T**; T** = 0: term absent).
    Both reactions of a pair get the same kind, efficiencies and Troe
    parameters.  Third body: A is divided by C_ref * e_max (C_ref the total
    concentration at T_ref, P_ref; e_max the largest efficiency) so the
    effective rate stays under the original stiffness bound.  Falloff: k_inf is
    the pair's original rate; k_0 = k_inf * 10^U(-1, 1) / C_ref for each
    direction (the same factor, so the reverse k_0 / k_inf ratio matches the
    forward one and the Appendix A fit of the reverse carries over); the
    falloff rate never exceeds k_inf."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in mech.items()}
    nS, nR = m["n_species"], m["n_reactions"]
    n_pairs = nR // 2
    c_ref = P_ref * 10.0 / (R_ERG * T_ref)
    sets = np.ones((n_sets, nS))
    for q in range(n_sets):
        sp = rng.choice(nS, size=min(6, nS), replace=False)
        sets[q, sp] = rng.choice([0.7, 1.5, 2.0, 3.0, 6.0, 12.0], size=len(sp))
    pdep = np.zeros(nR, np.int32)
    eff = np.ones((nR, nS))
    A0 = np.zeros(nR)
    beta0 = np.zeros(nR)
    Ea0 = np.zeros(nR)
    troe = np.zeros((nR, 4))
    order = rng.permutation(n_pairs)
    n_tb = int(round(frac_tb * n_pairs))
    n_fo = int(round(frac_fo * n_pairs))
    for k, pr in enumerate(order[:n_tb + n_fo]):
        j = 2 * int(pr)
        q = int(rng.integers(n_sets))
        if k < n_tb:
            kind = PDEP_THIRD_BODY
            for jj in (j, j + 1):
                m["A"][jj] = m["A"][jj] / (c_ref * sets[q].max())
        else:
            kind = PDEP_TROE if rng.random() < 2.0 / 3.0 else PDEP_LINDEMANN
            fac = 10.0 ** rng.uniform(-1.0, 1.0) / c_ref
            for jj in (j, j + 1):
                A0[jj] = m["A"][jj] * fac
                beta0[jj] = m["beta"][jj]
                Ea0[jj] = m["Ea"][jj]
            if kind == PDEP_TROE:
                t = (rng.uniform(0.1, 0.9), 10.0 ** rng.uniform(1.0, 3.0),
                     10.0 ** rng.uniform(3.0, 4.0),
                     rng.uniform(1000.0, 8000.0) if rng.random() < 0.5 else 0.0)
                troe[j] = troe[j + 1] = t
        pdep[j] = pdep[j + 1] = kind
        eff[j] = eff[j + 1] = sets[q]
    m.update(pdep=pdep, eff=eff, A0=A0, beta0=beta0, Ea0=Ea0, troe=troe,
             name=mech.get("name", "mech") + "_pdep")
    return m


def config_mechanism(name):
    """The seeded mechanism of a named configuration (c1..c4)."""
    return _cached_mech(name)


def config_states(name, n_cells=None, order="shuffled", seed=None):
    """Seeded states of a configuration; n_cells defaults to its full size."""
    c = CONFIGS[name]
    n = c["n_cells"] if n_cells is None else n_cells
    return make_states(config_mechanism(name), n, c["state_seed"] if seed is None else seed,
                       T_dist=c["T"], P_dist=c["P"], Y_dist=c["Y"], order=order)


# ---- served workload: Poisson request trace --------------------------------

C5_SEED = 3005


@functools.lru_cache(maxsize=None)
def c5_mechanism(kind, i):
    """kind 13 or 53; i in 0..3: the served workload's mechanism sets."""
    base = "c2" if kind == 13 else "c3"
    c = CONFIGS[base]
    m = make_mechanism(c["n_species"], c["n_reactions"], c["elements"], 3100 + 100 * (kind == 53) + i,
                       ea_max=c["ea_max"], T_lo=c["T_range"][0], T_hi=c["T_range"][1],
                       P_max=c["P_max"], dt=c["dt"], s_target=c["s_target"],
                       name="c5_%dsp_%d" % (kind, i))
    if c["Y"][0] == "majors":
        m["major_species"] = list(range(c["Y"][1]))
    return m


def c5_trace(n_requests=2000, rate=200.0, seed=C5_SEED, log2_lo=10.0, log2_hi=16.0):
    """Request list: arrival time (s), mechanism (kind, i), n_cells, dt, state seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    out = []
    for r in range(n_requests):
        kind = 13 if rng.random() < 0.5 else 53
        i = int(rng.integers(4))
        n = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
        dt = 1e-6 if rng.random() < 0.5 else 1e-5
        out.append({"id": r, "t_arrival": float(t[r]), "mech": (kind, i), "n_cells": n,
                    "dt": dt, "state_seed": int(rng.integers(1 << 31))})
    return out


def c5_states(req):
    base = "c2" if req["mech"][0] == 13 else "c3"
    c = CONFIGS[base]
    return make_states(c5_mechanism(*req["mech"]), req["n_cells"], req["state_seed"],
                       T_dist=c["T"], P_dist=c["P"], Y_dist=c["Y"])
