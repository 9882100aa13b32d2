"""Shared test fixtures: block builders (oracle for exact blocks, seeded generators for synthetic ones)."""
import numpy as np

from dmrg_inputs import random_integrals
from dmrg_inputs.synthetic import synthetic_problem
from oracle.fock import exact_block, random_bases, truncate
from oracle.hamiltonian import spin_orbital_integrals


def exact_problem(L, seed, n_alpha=None, n_beta=None, trunc=None, site=None):
    """Integrals + exact (optionally randomly truncated) blocks from the oracle's Fock space at the
    middle bond, or at the bond (site, site + 1) (0-based; site 0 and L - 2 leave a block empty)."""
    h, eri = random_integrals(L, seed)
    t, w = spin_orbital_integrals(h, eri)
    s1 = L // 2 - 1 if site is None else site
    s2 = s1 + 1
    left = exact_block(list(range(0, s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    right = exact_block(list(range(s2 + 1, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s2])
    if trunc is not None:
        left = truncate(left, random_bases(left, trunc, seed + 100))
        right = truncate(right, random_bases(right, trunc, seed + 200))
    na = L // 2 if n_alpha is None else n_alpha
    nb = L // 2 if n_beta is None else n_beta
    return h, eri, left, right, na, nb, s1


def synth(L, M, sigma, seed, n_alpha=None, n_beta=None):
    na = (L + 1) // 2 if n_alpha is None else n_alpha
    nb = L // 2 if n_beta is None else n_beta
    h, eri, left, right, site = synthetic_problem(L, na, nb, M, sigma, seed)
    return h, eri, left, right, na, nb, site


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
