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


# Error model of the split-BF16 H.psi. Each operand x is held as x_hi + x_lo with 8 significant bits
# each (round to nearest), so x - x_hi - x_lo is at most 2^-17 |x|, and a product a.b is formed as
# a_hi b_hi + a_hi b_lo + a_lo b_hi: off by at most about (2 * 2^-17 + 2^-18) |a| |b|. A task chains
# two such GEMMs (the intermediate is split again) and partial sums run in FP32 (2^-24 per add), so
# every output element satisfies |y - y_ref| <= ~2^-15 * sum over its summands of |f| |A| |X| |B|^T
# (the oracle's ``magnitude``). The bar is 2^-12 of that sum: an 8x margin over the model, while a
# dropped task or a wrong row changes its elements by a whole summand (~1/#summands of the sum).
SPLIT_BOUND = 2.0 ** -12


def assert_split_bound(y, ref, mag, what=""):
    """Every element of the split result within SPLIT_BOUND * magnitude of the oracle's value."""
    ratio = np.abs(y - ref) / np.maximum(mag, 1e-300)
    worst = float(ratio.max(initial=0.0))
    print(f"[split bound] {what}: max |y - ref| / magnitude = {worst:.2e} (bar {SPLIT_BOUND:.2e})", flush=True)
    assert worst <= SPLIT_BOUND, (what, worst)
    return worst
