"""Random-integral Hamiltonians for the synthetic workloads.

The paper's molecules (Fe(II)-porphyrin CAS(32,34), anthracene tetramer CAS(63,63), FeMoco
CAS(113,76); Section 3) are not available, so every workload uses seeded random integrals with the
structure of a real-orbital electronic Hamiltonian (Eq. H2q, Section 2.1):

* ``h``: symmetric, upper triangle (incl. diagonal, row-major) drawn in one ``normal(0, 1)`` call
  and mirrored; then ``h[p, p] -= 2 p / L`` for 0-based ``p``.
* ``eri``: chemist-notation ``(pq|rs) = sum_k B_k[p,q] B_k[r,s]`` with 16 symmetric factors ``B_k``
  (upper triangles drawn with ``normal(0, 0.3)``, i.e. sigma = 0.3), giving the 8-fold permutational
  symmetry of real orbitals and a positive semi-definite pair matrix.

The generator is ``numpy.random.Generator(PCG64(seed))``; draw order: ``h`` first, then ``B_0..B_15``.
"""
import numpy as np

N_FACTORS = 16


def _sym_from_upper(rng, n, scale):
    iu = np.triu_indices(n)
    m = np.zeros((n, n))
    m[iu] = rng.normal(0.0, scale, size=iu[0].size)
    return m + np.triu(m, 1).T


def random_integrals(L, seed):
    """Return ``(h, eri)``: ``h`` of shape (L, L), ``eri`` of shape (L, L, L, L), both float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = _sym_from_upper(rng, L, 1.0)
    h[np.arange(L), np.arange(L)] -= 2.0 * np.arange(L) / L
    B = np.stack([_sym_from_upper(rng, L, 0.3) for _ in range(N_FACTORS)])
    eri = np.einsum("kpq,krs->pqrs", B, B)
    return h, eri


def random_vector(n, seed):
    """Seeded standard-normal vector of length ``n`` (float64, not normalised)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, 1.0, size=n)
