"""Brute-force full configuration interaction in the (N_alpha, N_beta) sector (Section 2.1, Eq. H2q).

Determinants are integers whose bit ``2p + s`` marks spin-orbital (p, s); the Jordan-Wigner order
is ascending bit index, so ``c+_P |n>`` carries ``(-1)^(number of occupied bits below P)``.

The Hamiltonian is applied in the spin-summed form of Eq. H2q (with the reading of
``oracle.hamiltonian``):

    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps),
    E_pq = sum_s c+_{ps} c_{qs},

which is an independent route from the spin-orbital ``w`` tensor used by the DMRG expansion.
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def determinants(L, n_alpha, n_beta):
    """Sorted array of determinant bit strings with the given electron counts."""
    dets = []
    for occ_a in itertools.combinations(range(L), n_alpha):
        ma = sum(1 << (2 * p) for p in occ_a)
        for occ_b in itertools.combinations(range(L), n_beta):
            dets.append(ma | sum(1 << (2 * p + 1) for p in occ_b))
    return np.array(sorted(dets), dtype=np.int64)


def _popcount(x):
    return np.bitwise_count(x.astype(np.uint64)).astype(np.int64)


def apply_excitation(dets, P, Q):
    """Apply c+_P c_Q to every determinant. Returns (mask, new_dets, sign) for those that survive."""
    bitQ = np.int64(1) << Q
    bitP = np.int64(1) << P
    has_q = (dets & bitQ) != 0
    d1 = dets ^ bitQ
    sign_q = 1 - 2 * (_popcount(dets & (bitQ - 1)) & 1)
    if P == Q:
        ok = has_q
        new = dets
        sign = np.ones_like(dets)
    else:
        ok = has_q & ((d1 & bitP) == 0)
        new = d1 | bitP
        sign = sign_q * (1 - 2 * (_popcount(d1 & (bitP - 1)) & 1))
    return ok, new, sign


def excitation_operators(L, dets):
    """Spin-summed E_pq as sparse (dim x dim) matrices on the determinant list ``dets``."""
    dim = dets.size
    E = {}
    for p in range(L):
        for q in range(L):
            rows, cols, vals = [], [], []
            for s in (0, 1):
                ok, new, sign = apply_excitation(dets, 2 * p + s, 2 * q + s)
                idx = np.nonzero(ok)[0]
                rows.append(np.searchsorted(dets, new[idx]))
                cols.append(idx)
                vals.append(sign[idx].astype(np.float64))
            E[p, q] = sp.csr_matrix(
                (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(dim, dim))
    return E


class FCI:
    """FCI Hamiltonian of (h, eri) restricted to (n_alpha, n_beta)."""

    def __init__(self, h, eri, n_alpha, n_beta):
        self.L = h.shape[0]
        self.h, self.eri = h, eri
        self.dets = determinants(self.L, n_alpha, n_beta)
        self.dim = self.dets.size
        self.E = excitation_operators(self.L, self.dets)
        L = self.L
        # k_ps = h_ps - 1/2 sum_q (pq|qs)
        self.k = h - 0.5 * np.einsum("pqqs->ps", eri)
        self.g = eri.reshape(L * L, L * L)

    def matvec(self, x):
        """H x for x of shape (dim,) or (dim, nvec)."""
        L = self.L
        x2 = x.reshape(self.dim, -1)
        phi = np.stack([self.E[r, s] @ x2 for r in range(L) for s in range(L)])  # (L^2, dim, nv)
        chi = np.tensordot(self.g, phi, axes=(1, 0))                              # (L^2, dim, nv)
        y = np.zeros_like(x2)
        for p in range(L):
            for q in range(L):
                y += self.E[p, q] @ (self.k[p, q] * x2 + 0.5 * chi[p * L + q])
        return y.reshape(x.shape)

    def sparse_matrix(self):
        """Explicit sparse H (only sensible for small dim)."""
        L = self.L
        H = sp.csr_matrix((self.dim, self.dim))
        for p in range(L):
            for q in range(L):
                H = H + self.k[p, q] * self.E[p, q]
                inner = sp.csr_matrix((self.dim, self.dim))
                for r in range(L):
                    for s in range(L):
                        if self.eri[p, q, r, s] != 0.0:
                            inner = inner + self.eri[p, q, r, s] * self.E[r, s]
                H = H + 0.5 * (self.E[p, q] @ inner)
        return H

    def ground_state(self, tol=1e-13):
        """Lowest eigenpair (energy, vector) by Lanczos on the matvec (dense eigh for dim <= 400)."""
        if self.dim <= 400:
            H = self.sparse_matrix().toarray()
            e, v = np.linalg.eigh(H)
            return e[0], v[:, 0]
        op = spla.LinearOperator((self.dim, self.dim), matvec=self.matvec, dtype=np.float64)
        e, v = spla.eigsh(op, k=1, which="SA", tol=tol, ncv=min(self.dim - 1, 40))
        return e[0], v[:, 0]
