"""Pins of the oracle's two-site H.psi, diag(H) and Davidson against brute-force FCI and invariants."""
import os

import numpy as np
import pytest

from dmrg_inputs import random_integrals, random_vector
from oracle import terms
from oracle.davidson import davidson
from oracle.fci import FCI
from oracle.fock import FockSpace, embed, exact_block, project, random_bases, truncate
from oracle.hamiltonian import spin_orbital_integrals
from oracle.hpsi import OracleHop

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def middle_bond_blocks(L, seed, trunc=None):
    """Exact (or randomly truncated) blocks at the middle bond i = floor(L/2) (1-based)."""
    h, eri = random_integrals(L, seed)
    t, w = spin_orbital_integrals(h, eri)
    s1 = L // 2 - 1
    s2 = s1 + 1
    left = exact_block(list(range(0, s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    right = exact_block(list(range(s2 + 1, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s2])
    if trunc is not None:
        left = truncate(left, random_bases(left, trunc, seed + 100))
        right = truncate(right, random_bases(right, trunc, seed + 200))
    return h, eri, left, right, s1, s2


def test_golden_creation_matrices():
    """Eq. creation_ops as printed equals the site matrices used here, in the basis order (0,dn,up,updn)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "creation_ops.txt")) if not l.startswith("#")]
    up = np.array([[float(v) for v in r] for r in rows[1:5]])
    dn = np.array([[float(v) for v in r] for r in rows[6:10]])
    perm = np.eye(4)[[0, 2, 1, 3]]                # (0, up, dn, updn) -> (0, dn, up, updn)
    assert np.array_equal(perm @ terms.A_UP @ perm.T, up)
    assert np.array_equal(perm @ terms.A_DN @ perm.T, dn)


def test_site_car():
    I = np.eye(4)
    ops = {s: terms.site_op(True, s) for s in (0, 1)}
    for s in (0, 1):
        for r in (0, 1):
            a, ad = ops[s].T, ops[r]
            assert np.allclose(a @ ad + ad @ a, I * (s == r))
            assert np.allclose(ops[s] @ ops[r] + ops[r] @ ops[s], 0)
    # parity anticommutes with every site fermion operator
    for s in (0, 1):
        assert np.allclose(terms.SITE_PARITY @ ops[s], -ops[s] @ terms.SITE_PARITY)


def test_fock_space_car():
    F = FockSpace(2)
    for m in range(4):
        for n in range(4):
            acomm = (F.cd(m) @ F.c(n) + F.c(n) @ F.cd(m)).toarray()
            assert np.allclose(acomm, np.eye(16) * (m == n))
            assert np.allclose((F.c(m) @ F.c(n) + F.c(n) @ F.c(m)).toarray(), 0)


@pytest.mark.parametrize("L", [8])
def test_hpsi_equals_fci_exact_blocks(L):
    """Config 0 shape: exact 64-state blocks; the superblock space is the FCI space (4900)."""
    h, eri, left, right, s1, s2 = middle_bond_blocks(L, 0)
    hop = OracleHop(h, eri, left, right, L // 2, L // 2, s1)
    fci = FCI(h, eri, L // 2, L // 2)
    assert hop.layout.size == fci.dim == 4900
    assert len(hop.layout.blocks) == 196
    x = random_vector(hop.layout.size, 5)
    y = hop.apply(x)
    X = embed(hop.layout, x, left, right, s1, s2, fci.dets)
    yref = project(hop.layout, fci.matvec(X), left, right, s1, s2, fci.dets)
    assert np.abs(y - yref).max() < 1e-12 * np.abs(yref).max()


@pytest.mark.slow
def test_hpsi_equals_fci_exact_blocks_L10():
    h, eri, left, right, s1, s2 = middle_bond_blocks(10, 1)
    hop = OracleHop(h, eri, left, right, 5, 4, s1)
    fci = FCI(h, eri, 5, 4)
    x = random_vector(hop.layout.size, 6)
    X = embed(hop.layout, x, left, right, s1, s2, fci.dets)
    yref = project(hop.layout, fci.matvec(X), left, right, s1, s2, fci.dets)
    assert np.abs(hop.apply(x) - yref).max() < 1e-12 * np.abs(yref).max()


@pytest.mark.parametrize("L,s1,na,nb", [(2, 0, 1, 1), (4, 0, 2, 2), (4, 2, 2, 2), (5, 0, 3, 2), (6, 4, 3, 3),
                                        (8, 3, 6, 2), (9, 2, 5, 3), (6, 2, 5, 5), (6, 2, 1, 0)])
def test_hpsi_equals_fci_edge_and_uneven_bonds(L, s1, na, nb):
    """Edge bonds: a block with no orbitals holds only the vacuum (one sector of dimension 1), so the
    superblock is still the whole FCI space. Also, with exact blocks: strong spin imbalance (6, 2), an
    off-centre bond of odd L, two holes (5, 5) in 6 orbitals, and a single electron."""
    h, eri = random_integrals(L, 3)
    t, w = spin_orbital_integrals(h, eri)
    s2 = s1 + 1
    left = exact_block(list(range(0, s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    right = exact_block(list(range(s2 + 1, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s2])
    hop = OracleHop(h, eri, left, right, na, nb, s1)
    fci = FCI(h, eri, na, nb)
    assert hop.layout.size == fci.dim
    x = random_vector(hop.layout.size, 5)
    X = embed(hop.layout, x, left, right, s1, s2, fci.dets)
    yref = project(hop.layout, fci.matvec(X), left, right, s1, s2, fci.dets)
    assert np.abs(hop.apply(x) - yref).max() < 1e-12 * np.abs(yref).max()


def test_hpsi_projected_fci_truncated_blocks():
    """Truncated bases: H_sb = P^T H_FCI P with P the isometric embedding (Section 2.1, Eq. h_mat)."""
    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 2, trunc=24)
    hop = OracleHop(h, eri, left, right, 4, 3, s1)
    fci = FCI(h, eri, 4, 3)
    x = random_vector(hop.layout.size, 7)
    X = embed(hop.layout, x, left, right, s1, s2, fci.dets)
    yref = project(hop.layout, fci.matvec(X), left, right, s1, s2, fci.dets)
    assert np.abs(hop.apply(x) - yref).max() < 1e-12 * np.abs(yref).max()


def test_hermiticity_and_linearity_truncated():
    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 3, trunc=30)
    hop = OracleHop(h, eri, left, right, 4, 4, s1)
    n = hop.layout.size
    x, y = random_vector(n, 1), random_vector(n, 2)
    hx, hy = hop.apply(x), hop.apply(y)
    assert abs(x @ hy - hx @ y) < 1e-12 * np.linalg.norm(hx) * np.linalg.norm(y)
    assert np.abs(hop.apply(2.0 * x - 3.0 * y) - (2.0 * hx - 3.0 * hy)).max() < 1e-11 * np.abs(hx).max()


def test_diagonal_matches_unit_vectors():
    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 4, trunc=20)
    hop = OracleHop(h, eri, left, right, 4, 4, s1)
    D = hop.diagonal()
    rng = np.random.default_rng(0)
    idx = rng.choice(hop.layout.size, 25, replace=False)
    E = np.zeros((hop.layout.size, idx.size))
    E[idx, np.arange(idx.size)] = 1.0
    HE = hop.apply(E)
    assert np.abs(HE[idx, np.arange(idx.size)] - D[idx]).max() < 1e-12 * (1 + np.abs(D).max())


def test_davidson_config0_equals_fci():
    """Config 0: L=8, (4,4), M=64, Davidson to 1e-10 at the middle bond equals the FCI energy."""
    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 0)
    hop = OracleHop(h, eri, left, right, 4, 4, s1)
    fci = FCI(h, eri, 4, 4)
    e_fci, _ = fci.ground_state()
    H = hop.apply(np.eye(hop.layout.size))       # explicit operator, columns H e_i
    res = davidson(lambda v: H @ v, hop.diagonal(), random_vector(hop.layout.size, 0), tol=1e-10)
    assert res["converged"]
    assert abs(res["energy"] - e_fci) < 1e-10


def test_davidson_equals_dense_eigh():
    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 5, trunc=16)
    hop = OracleHop(h, eri, left, right, 4, 4, s1)
    n = hop.layout.size
    H = hop.apply(np.eye(n))
    assert np.abs(H - H.T).max() < 1e-11
    e0 = np.linalg.eigvalsh(H)[0]
    v = random_vector(n, 3)
    assert np.abs(H @ v - hop.apply(v)).max() < 1e-11 * np.abs(H).max()
    res = davidson(hop.apply, hop.diagonal(), v, tol=1e-9)
    assert abs(res["energy"] - e0) < 1e-10


def test_variational_truncation():
    """Truncated-block energies are upper bounds of the FCI energy and fall as M grows."""
    energies = []
    for M in (12, 24, 48):
        h, eri, left, right, s1, s2 = middle_bond_blocks(8, 6, trunc=M)
        hop = OracleHop(h, eri, left, right, 4, 4, s1)
        H = hop.apply(np.eye(hop.layout.size))
        res = davidson(lambda v: H @ v, hop.diagonal(), random_vector(hop.layout.size, 1), tol=1e-9)
        energies.append(res["energy"])
    h, eri = random_integrals(8, 6)
    e_fci, _ = FCI(h, eri, 4, 4).ground_state()
    assert all(e >= e_fci - 1e-9 for e in energies)


def test_planted_sign_mistake_is_caught(monkeypatch):
    """A plausible mistake in the oracle (dropping the JW parity on the site strings) fails the FCI pin."""
    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 0)
    monkeypatch.setattr(terms, "SITE_PARITY", np.eye(4))
    hop = OracleHop(h, eri, left, right, 4, 4, s1)
    fci = FCI(h, eri, 4, 4)
    x = random_vector(hop.layout.size, 5)
    X = embed(hop.layout, x, left, right, s1, s2, fci.dets)
    yref = project(hop.layout, fci.matvec(X), left, right, s1, s2, fci.dets)
    assert np.abs(hop.apply(x) - yref).max() > 1e-3


def test_planted_integral_convention_mistake_is_caught(monkeypatch):
    """Reading v_pqrs as (pq|rs)/2 instead of (ps|qr)/2 fails the FCI pin."""
    import oracle.hpsi as hpsi_mod

    def wrong(h, eri):
        t, w = spin_orbital_integrals(h, eri)
        L = h.shape[0]
        w2 = np.zeros_like(w)
        for sp in (0, 1):
            for sq in (0, 1):
                w2[sp::2, sq::2, sq::2, sp::2] = eri
        return t, w2

    h, eri, left, right, s1, s2 = middle_bond_blocks(8, 0)
    monkeypatch.setattr(hpsi_mod, "spin_orbital_integrals", wrong)
    hop = OracleHop(h, eri, left, right, 4, 4, s1)
    fci = FCI(h, eri, 4, 4)
    x = random_vector(hop.layout.size, 5)
    X = embed(hop.layout, x, left, right, s1, s2, fci.dets)
    yref = project(hop.layout, fci.matvec(X), left, right, s1, s2, fci.dets)
    assert np.abs(hop.apply(x) - yref).max() > 1e-3
