"""Hand-built tiny mechanisms for closed-form pins (dict layout of synth), and
seeded synthetic ones at the kernels' largest state sizes."""
import functools

import numpy as np

from paper_1309_2710_amd.synth import R_J, ATM


def tiny(species_W, reactions, nasa=None, T_mid=1000.0):
    """species_W: list of W; reactions: list of (reac list, prod list, A, beta, Ea).
    nasa: per species (low7, high7) or a single 7-vector used for both ranges."""
    nS = len(species_W)
    nR = len(reactions)
    reac = np.full((nR, 3), -1, np.int32)
    prod = np.full((nR, 3), -1, np.int32)
    A = np.zeros(nR); beta = np.zeros(nR); Ea = np.zeros(nR)
    for j, (r, p, a, b, e) in enumerate(reactions):
        reac[j, :len(r)] = r
        prod[j, :len(p)] = p
        A[j], beta[j], Ea[j] = a, b, e
    lo = np.zeros((nS, 7)); hi = np.zeros((nS, 7))
    for i in range(nS):
        if nasa is None:
            c = np.array([3.5, 0, 0, 0, 0, 0, 0.0])
            lo[i] = hi[i] = c
        else:
            v = nasa[i]
            if isinstance(v, tuple):
                lo[i], hi[i] = v
            else:
                lo[i] = hi[i] = v
    return {"n_species": nS, "n_reactions": nR, "W": np.asarray(species_W, float),
            "nasa_low": lo, "nasa_high": hi, "T_mid": np.full(nS, T_mid),
            "reac": reac, "prod": prod, "A": A, "beta": beta, "Ea": Ea}


def a_to_b(k=1e6, W=10.0):
    """A -> B, identical W and thermo: dT/dt = 0 and dY_A/dt = -k Y_A."""
    return tiny([W, W], [([0], [1], k, 0.0, 0.0)])


def a_b_c(k1, k2, W=10.0):
    """A -> B -> C at constant T (identical thermo)."""
    return tiny([W, W, W], [([0], [1], k1, 0.0, 0.0), ([1], [2], k2, 0.0, 0.0)])


def nonlinear3(W=(10.0, 20.0, 30.0)):
    """A + B -> C, C -> A + B with distinct thermo: nonlinear, T varies."""
    n = [np.array([3.0, 1e-3, 0, 0, 0, -2000.0, 0]),
         np.array([3.5, 5e-4, 0, 0, 0, 1000.0, 0]),
         np.array([4.5, 2e-4, 0, 0, 0, -6000.0, 0])]
    return tiny(list(W), [([0, 1], [2], 1e12, 0.5, 4e4), ([2], [0, 1], 1e9, 0.0, 8e4)],
                nasa=n)


@functools.lru_cache(maxsize=None)
def seeded(n_species):
    """Seeded synthetic mechanisms sized to fill four slots per lane: 255
    species (64 lanes) and 31 species (8 lanes)."""
    from paper_1309_2710_amd import synth
    if n_species == 255:
        return synth.make_mechanism(255, 600, ["H", "O", "C", "N", "Ar"], 4242,
                                    limits={"C": 4, "H": 10, "O": 4, "N": 2}, max_atoms=12)
    assert n_species == 31
    return synth.make_mechanism(31, 120, ["H", "O", "C", "N"], 3131,
                                limits={"C": 2, "H": 4, "O": 2, "N": 2}, max_atoms=6)


def seeded_states(m, n, seed):
    from paper_1309_2710_amd import synth
    return synth.make_states(m, n, seed, T_dist=("uniform", 900.0, 1800.0),
                             P_dist=("const", ATM), Y_dist=("dirichlet",))
