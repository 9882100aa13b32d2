"""Spin-orbital form of the electronic Hamiltonian, Eq. H2q (Section 2.1).

Eq. H2q has no 1/2 and names no index convention for ``v_pqrs``; the integrals of the workloads
are chemist-notation ``(pq|rs)``. Reading used throughout: ``v_pqrs = (ps|qr) / 2``, i.e.

    H = sum_{PQ} t_PQ c+_P c_Q + 1/2 sum_{PQRS} w_PQRS c+_P c+_Q c_R c_S,
    t_PQ   = h_pq  delta(sP, sQ),
    w_PQRS = (ps|qr) delta(sP, sS) delta(sQ, sR),

with spin-orbital id ``P = 2 p + sP`` (sP = 0 alpha, 1 beta) and Jordan-Wigner order
1a, 1b, 2a, 2b, ... along the orbital lattice. There is no core energy.
Pinned by the one-orbital closed form E = 2 h_11 + (11|11) (tests/test_oracle_fci.py).
"""
import numpy as np


def spin_orbital_integrals(h, eri):
    """Return ``(t, w)`` of shapes (2L, 2L) and (2L, 2L, 2L, 2L)."""
    L = h.shape[0]
    n = 2 * L
    t = np.zeros((n, n))
    for s in (0, 1):
        t[s::2, s::2] = h
    w = np.zeros((n, n, n, n))
    # w[P,Q,R,S] = (p s | q r) when spin(P) == spin(S) and spin(Q) == spin(R)
    ps_qr = np.transpose(eri, (0, 2, 3, 1))  # [p, q, r, s] -> (ps|qr)
    for sp in (0, 1):
        for sq in (0, 1):
            w[sp::2, sq::2, sq::2, sp::2] = ps_qr
    return t, w
