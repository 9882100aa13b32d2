"""Pins of the oracle's reduced density matrices, truncation and Eq. renorm_mat (Section 2.1).

* Schmidt values: with exact blocks the FCI ground state, projected onto the superblock basis, is an
  eigenvector of the superblock H.psi and the same state in another basis of each half, so the
  eigenvalues of rho^L must be the squared singular values of the FCI vector cut between orbitals
  <= s1 and >= s2, computed straight from the determinant bit strings (no block, layout or site
  convention involved). Also the discarded weight of every M.
* Eckart-Young: on a random psi over truncated blocks, the discarded weight of the global M-cut
  equals the tail sum of squared singular values of the dense psi matrix, and O O^T psi equals the
  dense rank-M reconstruction.
* Invariants: trace rho^L = trace rho^R = |psi|^2; rho^L_q and rho^R_{N-q} share their nonzero
  spectrum; M at the full dimension keeps psi exactly.
* Eq. renorm_mat: expectation values of the left site's and left block's electron numbers, from
  rho^L and from the renormalized operators with the transformed psi, equal those of the FCI vector
  (determinant occupations) and the psi blocks themselves.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle import renorm
from oracle.fci import FCI
from oracle.fock import project
from oracle.hpsi import OracleHop
from oracle.layout import SITE_QN
from helpers import exact_problem


def _ground_states(L, site, na, nb, seed):
    h, eri, left, right, na, nb, s1 = exact_problem(L, seed, n_alpha=na, n_beta=nb, site=site)
    hop = OracleHop(h, eri, left, right, na, nb, s1)
    fci = FCI(h, eri, na, nb)
    e, c = fci.ground_state()
    # exact blocks: the block bases span each half's Fock space, so projection is a change of basis
    psi = project(hop.layout, c, left, right, s1, s1 + 1, fci.dets)
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    y = hop.apply(psi)
    assert np.abs(y - e * psi).max() < 1e-9           # an eigenvector of the superblock H.psi
    return hop, left, right, na, nb, s1, psi, fci, c


def _fci_schmidt(dets, c, s1):
    """Singular values of the FCI vector as a matrix (orbitals <= s1) x (orbitals > s1)."""
    cut = 2 * (s1 + 1)
    rows = dets & ((1 << cut) - 1)
    cols = dets >> cut
    ru, ri = np.unique(rows, return_inverse=True)
    cu, ci = np.unique(cols, return_inverse=True)
    C = np.zeros((ru.size, cu.size))
    C[ri, ci] = c
    return np.linalg.svd(C, compute_uv=False)


def _spectrum(rho):
    return np.sort(np.concatenate([np.linalg.eigvalsh(r) for r in rho.values()]))[::-1]


@pytest.fixture(scope="module", params=[(8, None, 4, 4), (6, 1, 3, 3), (7, 4, 4, 3)], ids=["L8_mid", "L6_s1", "L7_s4"])
def exact_gs(request):
    L, site, na, nb = request.param
    return _ground_states(L, site, na, nb, seed=2)


def test_rdm_eigenvalues_are_fci_schmidt_values(exact_gs):
    hop, left, right, na, nb, s1, psi, fci, c = exact_gs
    P = renorm.psi_matrices(hop.layout, left, right, na, nb, psi)
    w = _spectrum(renorm.rdm_left(P))
    s2 = _fci_schmidt(fci.dets, c, s1) ** 2
    n = max(w.size, s2.size)
    w = np.pad(w, (0, n - w.size))
    s2 = np.pad(np.sort(s2)[::-1], (0, n - s2.size))
    assert abs(w.sum() - 1.0) < 1e-12
    assert np.abs(w - s2).max() < 1e-8
    wr = _spectrum(renorm.rdm_right(P, na, nb))
    assert np.abs(np.pad(wr, (0, max(0, n - wr.size)))[:n] - s2).max() < 1e-8
    for M in (1, 4, 16, 64):
        _, kept, disc = renorm.select(renorm.rdm_left(P), M)
        assert len(kept) == min(M, w.size)
        assert abs(disc - s2[M:].sum()) < 1e-8


def test_renorm_mat_preserves_number_expectations(exact_gs):
    hop, left, right, na, nb, s1, psi, fci, c = exact_gs
    P = renorm.psi_matrices(hop.layout, left, right, na, nb, psi)
    rho = renorm.rdm_left(P)
    O, _, disc = renorm.select(rho, sum(r.shape[0] for r in rho.values()))
    assert abs(disc) < 1e-12
    Pt = renorm.transform_psi(P, O)
    for spin in (0, 1):
        # FCI: occupation of spin-orbital (s1, spin), and of the left block's orbitals (< s1)
        occ = ((fci.dets >> (2 * s1 + spin)) & 1).astype(float)
        n_site = float(np.sum(occ * c * c))
        blk = np.zeros(fci.dets.size)
        for p in range(s1):
            blk += (fci.dets >> (2 * p + spin)) & 1
        n_blk = float(np.sum(blk * c * c))
        for A, ref in ((renorm.site_number_left(left, spin), n_site), (renorm.block_number_left(left, spin), n_blk)):
            via_rho = sum(float(np.trace(rho[q] @ A[(q, q)])) for q in rho)
            Ar = renorm.renormalize(A, O, O)
            via_renorm = sum(float(np.trace(Pt[q].T @ Ar[(q, q)] @ Pt[q])) for q in Pt)
            assert abs(via_rho - ref) < 1e-9 and abs(via_renorm - ref) < 1e-9
    # the psi blocks directly: <n_site alpha> = sum over blocks of occupation(b) |X|^2
    direct = sum(SITE_QN[b][0] * float(np.sum(hop.layout.view(psi, i) ** 2))
                 for i, (a, b, cc, d, off, ma, md) in enumerate(hop.layout.blocks))
    occ = ((fci.dets >> (2 * s1)) & 1).astype(float)
    assert abs(direct - float(np.sum(occ * c * c))) < 1e-9


@pytest.fixture(scope="module")
def random_psi():
    h, eri, left, right, na, nb, s1 = exact_problem(8, 1, trunc=24)
    hop = OracleHop(h, eri, left, right, na, nb, s1)
    psi = random_vector(hop.layout.size, 12)
    psi /= np.linalg.norm(psi)
    P = renorm.psi_matrices(hop.layout, left, right, na, nb, psi)
    return hop, left, right, na, nb, psi, P


def _dense(P):
    """Block-diagonal dense psi matrix over all enlarged-left x enlarged-right sectors."""
    R = sum(m.shape[0] for m in P.values())
    C = sum(m.shape[1] for m in P.values())
    D = np.zeros((R, C))
    r = c = 0
    for m in P.values():
        D[r:r + m.shape[0], c:c + m.shape[1]] = m
        r += m.shape[0]
        c += m.shape[1]
    return D


def test_layout_maps_every_block_once(random_psi):
    hop, left, right, na, nb, psi, P = random_psi
    assert abs(sum(float(np.sum(m * m)) for m in P.values()) - 1.0) < 1e-13
    _, ldims = renorm.enlarged_left_basis(left)
    assert sum(ldims.values()) == 4 * int(left.dim.sum())       # the 4M-dimensional enlarged basis


def test_traces_and_shared_spectra(random_psi):
    hop, left, right, na, nb, psi, P = random_psi
    rl, rr = renorm.rdm_left(P), renorm.rdm_right(P, na, nb)
    assert abs(sum(np.trace(r) for r in rl.values()) - 1.0) < 1e-12
    assert abs(sum(np.trace(r) for r in rr.values()) - 1.0) < 1e-12
    for q, r in rl.items():
        qr = (na - q[0], nb - q[1])
        if qr not in rr:
            assert not np.any(r)
            continue
        a = np.sort(np.linalg.eigvalsh(r))[::-1]
        b = np.sort(np.linalg.eigvalsh(rr[qr]))[::-1]
        k = min(a.size, b.size)
        assert np.abs(a[:k] - b[:k]).max() < 1e-13
        assert np.abs(a[k:]).max(initial=0) < 1e-13 and np.abs(b[k:]).max(initial=0) < 1e-13


@pytest.mark.parametrize("M", [1, 5, 17, 40, 96])
def test_global_cut_is_eckart_young(random_psi, M):
    hop, left, right, na, nb, psi, P = random_psi
    D = _dense(P)
    U, s, Vt = np.linalg.svd(D, full_matrices=False)
    O, kept, disc = renorm.select(renorm.rdm_left(P), M)
    assert abs(disc - float(np.sum(s[M:] ** 2))) < 1e-12
    assert sum(o.shape[1] for o in O.values()) == min(M, D.shape[0])
    for o in O.values():
        assert np.abs(o.T @ o - np.eye(o.shape[1])).max() < 1e-12
    proj = {q: O[q] @ (O[q].T @ P[q]) if q in O else np.zeros_like(P[q]) for q in P}
    best = (U[:, :M] * s[:M]) @ Vt[:M]
    assert np.abs(_dense(proj) - best).max() < 1e-10
    assert abs(float(np.sum((D - _dense(proj)) ** 2)) - disc) < 1e-12


def test_full_dimension_keeps_psi(random_psi):
    hop, left, right, na, nb, psi, P = random_psi
    rho = renorm.rdm_left(P)
    n = sum(r.shape[0] for r in rho.values())
    O, kept, disc = renorm.select(rho, n)
    assert len(kept) == n and abs(disc) < 1e-13
    Pt = renorm.transform_psi(P, O)
    for q in P:
        assert O[q].shape == (P[q].shape[0], P[q].shape[0])
        assert np.abs(O[q] @ Pt[q] - P[q]).max() < 1e-13


def test_per_sector_cut_is_not_the_global_cut(random_psi):
    """Planted reading error: keeping M states in every sector instead of M overall changes the
    discarded weight that the Eckart-Young pin checks."""
    hop, left, right, na, nb, psi, P = random_psi
    rho = renorm.rdm_left(P)
    M = 5
    s = np.linalg.svd(_dense(P), compute_uv=False)
    per_sector = sum(float(np.sum(np.sort(np.linalg.eigvalsh(r))[::-1][M:])) for r in rho.values())
    assert abs(per_sector - float(np.sum(s[M:] ** 2))) > 1e-3
