"""Pins of the FCI oracle and of the Hamiltonian reading (Eq. H2q) against closed forms."""
import numpy as np
import pytest

from dmrg_inputs import random_integrals
from oracle.fci import FCI, determinants
from oracle.hamiltonian import spin_orbital_integrals


def test_one_orbital_closed_form():
    # L = 1, N = 2: |updown> has E = 2 h_11 + (11|11)   (reading v_pqrs = (ps|qr)/2)
    h = np.array([[-1.3]])
    eri = np.array([[[[0.7]]]])
    e, _ = FCI(h, eri, 1, 1).ground_state()
    assert abs(e - (2 * h[0, 0] + eri[0, 0, 0, 0])) < 1e-14
    e1, _ = FCI(h, eri, 1, 0).ground_state()
    assert abs(e1 - h[0, 0]) < 1e-14


def test_two_orbital_triplet_closed_form():
    # L = 2, (N_alpha, N_beta) = (2, 0): one determinant, E = h11 + h22 + (11|22) - (12|21)
    h, eri = random_integrals(2, 11)
    e, _ = FCI(h, eri, 2, 0).ground_state()
    ref = h[0, 0] + h[1, 1] + eri[0, 0, 1, 1] - eri[0, 1, 1, 0]
    assert abs(e - ref) < 1e-13


def test_noninteracting_diagonal_closed_form():
    L = 6
    hd = np.array([0.3, -1.2, 0.8, -0.4, 2.0, -0.9])
    h = np.diag(hd)
    eri = np.zeros((L,) * 4)
    e, _ = FCI(h, eri, 3, 2).ground_state()
    s = np.sort(hd)
    assert abs(e - (s[:3].sum() + s[:2].sum())) < 1e-12


def test_noninteracting_offdiagonal_orbital_energies():
    # eri = 0: E = sum of the N_alpha lowest eigenvalues of h + the N_beta lowest
    h, _ = random_integrals(6, 3)
    eri = np.zeros((6,) * 4)
    e, _ = FCI(h, eri, 3, 3).ground_state()
    ev = np.linalg.eigvalsh(h)
    assert abs(e - 2 * ev[:3].sum()) < 1e-11


def test_integral_symmetries():
    h, eri = random_integrals(5, 0)
    assert np.allclose(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (1, 0, 3, 2), (3, 2, 1, 0)]:
        assert np.allclose(eri, np.transpose(eri, perm))
    g = eri.reshape(25, 25)
    assert np.linalg.eigvalsh(g).min() > -1e-12       # PSD pair matrix (sum of 16 outer products)


def test_spin_orbital_tensor_matches_chemist_form():
    h, eri = random_integrals(3, 2)
    t, w = spin_orbital_integrals(h, eri)
    # w[P,Q,R,S] = (ps|qr) for sP = sS, sQ = sR
    assert w[2 * 0 + 0, 2 * 1 + 1, 2 * 2 + 1, 2 * 1 + 0] == pytest.approx(eri[0, 1, 1, 2])
    assert w[2 * 0 + 0, 2 * 1 + 1, 2 * 2 + 0, 2 * 1 + 1] == 0.0
    assert np.allclose(w, np.transpose(w, (1, 0, 3, 2)))   # w_PQRS = w_QPSR


def test_fci_matvec_matches_sparse_and_is_symmetric():
    h, eri = random_integrals(5, 4)
    f = FCI(h, eri, 2, 3)
    H = f.sparse_matrix().toarray()
    assert np.abs(H - H.T).max() < 1e-12
    x = np.random.default_rng(0).normal(size=f.dim)
    assert np.abs(f.matvec(x) - H @ x).max() < 1e-11


def test_sector_dimension():
    assert determinants(8, 4, 4).size == 4900
    assert determinants(10, 5, 4).size == 252 * 210
