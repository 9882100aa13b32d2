"""Pins of the oracle's grown-block operators and of one renormalization step (Section 2.1).

* Blocking: with an exact block X, every operator of the grown block X + s built from X's stored
  operators and the site matrices (H, C, A, B, S) equals the exact operator of the grown orbital set
  (built independently in its full Fock space), after mapping |l>|s> onto the grown Fock states.
  Bonds: L = 6 (2 | 3), L = 8 (3 | 4), L = 5 (0 | 1: X holds the vacuum only) and (1 | 2).
* Planted mistake: dropping X's parity from the site operators breaks the pin.
* One renormalization step: ground state at the bond (2, 3) of L = 6 from FCI, rho^L, truncation to
  M states, Eq. renorm_mat for every grown-block operator; the superblock at the next bond (3, 4)
  then has the FCI ground-state energy when nothing is discarded, and for smaller M an energy
  between E_FCI (variational bound) and the energy of the truncated state O O^T psi, which that
  superblock space contains.
* The same step for the state itself: O O^T psi written in the next bond's basis (renormalized left
  block, the old right site as the new left site, the old exact right block split into a site and a
  block) has, under the next bond's H.psi, exactly the energy and norm it has at the current bond;
  at full M it is an eigenvector with the FCI energy.
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals
from oracle import renorm
from oracle.blocking import GrownLeft
from oracle.fci import FCI
from oracle.fock import exact_block, project
from oracle.hamiltonian import spin_orbital_integrals
from oracle.hpsi import OracleHop


def _dense(block, op):
    off = np.concatenate([[0], np.cumsum(block.dim)]).astype(np.int64)
    D = np.zeros((off[-1], off[-1]))
    if op is not None:
        for (so, si), m in op.blocks.items():
            D[off[so]:off[so + 1], off[si]:off[si + 1]] = m
    return D


def _setup(L, site, seed=3):
    h, eri = random_integrals(L, seed)
    t, w = spin_orbital_integrals(h, eri)
    X = exact_block(list(range(site)), "left", t, w, [P for P in range(2 * L) if P // 2 >= site])
    G = exact_block(list(range(site + 1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= site + 1])
    g = GrownLeft(X, t, w, site)
    # |l>|s> -> grown Fock state: X's bits below the site's (alpha = bit 0, beta = bit 1 of the site)
    xoff = np.concatenate([[0], np.cumsum(X.dim)]).astype(np.int64)
    goff = np.concatenate([[0], np.cumsum(G.dim)]).astype(np.int64)
    pi = np.zeros(g.n, dtype=np.int64)
    for a in range(X.n_sec):
        for l in range(int(X.dim[a])):
            bits = int(X.fock.sector_states[a][l])
            for s in range(4):
                gb = bits | (s << (2 * site))
                pi[4 * (xoff[a] + l) + s] = goff[G.fock.sector_of[gb]] + G.fock.pos_in[gb]
    assert np.array_equal(np.sort(pi), np.arange(g.n))
    return g, G, pi


def _exact(G, pi, kind, i0=-1, i1=-1):
    op = G.get(kind, i0, i1)
    if op is None and kind == "B" and G.get("B", i1, i0) is not None:
        return _dense(G, G.get("B", i1, i0)).T[np.ix_(pi, pi)]
    return _dense(G, op)[np.ix_(pi, pi)]


@pytest.mark.parametrize("L,site", [(6, 2), (8, 3), (5, 0), (5, 1)])
def test_blocked_operators_equal_exact_grown_block(L, site):
    g, G, pi = _setup(L, site)
    scale = np.abs(_exact(G, pi, "H")).max()
    assert np.abs(g.H() - _exact(G, pi, "H")).max() < 1e-13 * scale
    for P in g.modes:
        assert np.abs(g.C(P) - _exact(G, pi, "C", P)).max() < 1e-14
        for Q in g.modes:
            if P < Q:
                assert np.abs(g.A(P, Q) - _exact(G, pi, "A", P, Q)).max() < 1e-14
            assert np.abs(g.B(P, Q) - _exact(G, pi, "B", P, Q)).max() < 1e-14
    for W in range(2 * site + 2, 2 * L):
        assert np.abs(g.S(W) - _exact(G, pi, "S", W)).max() < 1e-13 * scale


def test_planted_missing_parity_is_caught():
    g, G, pi = _setup(6, 2)
    g.par = np.eye(g.nx)              # site operators no longer pass X's fermions
    assert np.abs(g.H() - _exact(G, pi, "H")).max() > 1e-3
    assert np.abs(g.C(g.smodes[0]) - _exact(G, pi, "C", g.smodes[0])).max() > 0.5


def _unflatten(layout, left, right, na, nb, P):
    """Inverse of renorm.psi_matrices: sector matrices back to the flat psi of the layout."""
    lparts, _ = renorm.enlarged_left_basis(left)
    rparts, _ = renorm.enlarged_right_basis(right)
    lstart = {(a, b): st for q in lparts for (a, b, st, m) in lparts[q]}
    rstart = {(c, d): st for q in rparts for (c, d, st, m) in rparts[q]}
    out = np.zeros(layout.size)
    for a, b, c, d, off, ma, md in layout.blocks:
        q = (int(left.qn[a][0]) + (b in (1, 3)), int(left.qn[a][1]) + (b in (2, 3)))
        r0, c0 = lstart[(a, b)], rstart[(c, d)]
        out[off:off + ma * md] = P[q][r0:r0 + ma, c0:c0 + md].ravel()
    return out


@pytest.fixture(scope="module")
def step():
    L, s1, na, nb = 6, 2, 3, 3
    h, eri = random_integrals(L, 5)
    t, w = spin_orbital_integrals(h, eri)
    left = exact_block(list(range(s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    right = exact_block(list(range(s1 + 2, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s1 + 1])
    hop = OracleHop(h, eri, left, right, na, nb, s1)
    fci = FCI(h, eri, na, nb)
    e_fci, c = fci.ground_state()
    psi = project(hop.layout, c, left, right, s1, s1 + 1, fci.dets)
    P = renorm.psi_matrices(hop.layout, left, right, na, nb, psi)
    rho = renorm.rdm_left(P)
    right_next = exact_block(list(range(s1 + 3, L)), "right", t, w, [P_ for P_ in range(2 * L) if P_ // 2 <= s1 + 2])
    return dict(h=h, eri=eri, t=t, w=w, left=left, right=right, right_next=right_next, hop=hop, na=na, nb=nb,
                s1=s1, e_fci=e_fci, P=P, rho=rho)


def _next_bond_energy(st, M):
    O, kept, disc = renorm.select(st["rho"], M)
    grown = GrownLeft(st["left"], st["t"], st["w"], st["s1"]).renormalized_block(O)
    nxt = OracleHop(st["h"], st["eri"], grown, st["right_next"], st["na"], st["nb"], st["s1"] + 1)
    Hm = nxt.apply(np.eye(nxt.layout.size))
    assert np.abs(Hm - Hm.T).max() < 1e-11
    return float(np.linalg.eigvalsh(Hm)[0]), O, disc


def test_renormalization_step_full_M_keeps_the_fci_energy(step):
    n = sum(r.shape[0] for r in step["rho"].values())
    e, O, disc = _next_bond_energy(step, n)
    assert abs(disc) < 1e-12
    assert abs(e - step["e_fci"]) < 1e-10


@pytest.mark.parametrize("M", [6, 12, 24])
def test_renormalization_step_truncated_is_bracketed(step, M):
    e, O, disc = _next_bond_energy(step, M)
    # energy of the truncated state O O^T psi at the current bond (contained in the next bond's space)
    Pt = {q: (O[q] @ (O[q].T @ step["P"][q]) if q in O else np.zeros_like(step["P"][q])) for q in step["P"]}
    x = _unflatten(step["hop"].layout, step["left"], step["right"], step["na"], step["nb"], Pt)
    e_trunc = float(x @ step["hop"].apply(x) / (x @ x))
    assert disc > 0
    assert step["e_fci"] - 1e-10 <= e <= e_trunc + 1e-10


def _split_exact_right(old, new):
    """Old exact right block -> its first orbital (the new right site) x the new right block."""
    def split(d, r):
        bits = int(old.fock.sector_states[d][r])
        s, rest = bits & 3, bits >> 2          # site bits come first in the Jordan-Wigner order
        return s, int(new.fock.sector_of[rest]), int(new.fock.pos_in[rest]), 1.0
    return split


@pytest.mark.parametrize("M", [6, 12, 24, 64])
def test_renormalization_step_carries_the_state(step, M):
    O, kept, disc = renorm.select(step["rho"], M)
    grown = GrownLeft(step["left"], step["t"], step["w"], step["s1"]).renormalized_block(O)
    nxt = OracleHop(step["h"], step["eri"], grown, step["right_next"], step["na"], step["nb"], step["s1"] + 1)
    psi_t = renorm.transform_psi(step["P"], O)
    split = _split_exact_right(step["right"], step["right_next"])
    y = renorm.next_bond_psi(nxt.layout, psi_t, step["right"], step["na"], step["nb"], split)
    # the same state at the current bond
    Pt = {q: (O[q] @ psi_t[q] if q in O else np.zeros_like(step["P"][q])) for q in step["P"]}
    x = _unflatten(step["hop"].layout, step["left"], step["right"], step["na"], step["nb"], Pt)
    assert abs(y @ y - x @ x) < 1e-12 and abs(y @ y - (1.0 - disc)) < 1e-12
    e_next = float(y @ nxt.apply(y) / (y @ y))
    e_cur = float(x @ step["hop"].apply(x) / (x @ x))
    assert abs(e_next - e_cur) < 1e-10
    if M == 64:
        assert abs(disc) < 1e-12
        assert np.abs(nxt.apply(y) - step["e_fci"] * y).max() < 1e-9


# ---------------------------------------------------------------- growth by the Fock-space route
@pytest.mark.parametrize("trunc", [None, 5])
def test_fock_route_growth_equals_stored_operator_route(step, trunc):
    """Two derivations of the grown, renormalized left block agree: GrownLeft (from the block's stored
    operators and the site matrices) and grown_block (exact operators of the grown orbital set in its
    own Fock space, projected); on the exact block and on a randomly truncated one."""
    from oracle.blocking import grown_block
    from oracle.fock import random_bases, truncate
    left = step["left"] if trunc is None else truncate(step["left"], random_bases(step["left"], trunc, 9))
    _, edims = renorm.enlarged_left_basis(left)
    rng = np.random.default_rng(2)
    O = {q: np.linalg.qr(rng.normal(size=(d, d)))[0][:, :max(1, (2 * d) // 3)] for q, d in edims.items()}
    a = GrownLeft(left, step["t"], step["w"], step["s1"]).renormalized_block(O)
    b = grown_block("left", left, step["s1"], O, step["t"], step["w"])
    assert a.qn.tolist() == b.qn.tolist() and a.dim.tolist() == b.dim.tolist()
    n = 0
    for op in a.ops:
        ob = b.get(op.kind, op.i0, op.i1)
        assert np.abs(_dense(a, op) - _dense(b, ob)).max() < 1e-13, op.key
        n += 1
    assert n > 50


@pytest.fixture(scope="module")
def back_step(step):
    """The backward direction at the same bond: rho^R of the FCI ground state, and the right block
    grown by the right site s2 = 3 into orbitals 3 .. 5 (the right block of the bond (1, 2))."""
    rho = renorm.rdm_right(step["P"], step["na"], step["nb"])
    left_prev = exact_block(list(range(step["s1"] - 1)), "left", step["t"], step["w"],
                            [P for P in range(12) if P // 2 >= step["s1"] - 1])
    return dict(rho=rho, left_prev=left_prev)


def _prev_bond_energy(step, back, M):
    from oracle.blocking import grown_block
    O, kept, disc = renorm.select(back["rho"], M)
    grown = grown_block("right", step["right"], step["s1"] + 1, O, step["t"], step["w"])
    prv = OracleHop(step["h"], step["eri"], back["left_prev"], grown, step["na"], step["nb"], step["s1"] - 1)
    Hm = prv.apply(np.eye(prv.layout.size))
    assert np.abs(Hm - Hm.T).max() < 1e-11
    return float(np.linalg.eigvalsh(Hm)[0]), disc


def test_backward_step_full_M_keeps_the_fci_energy(step, back_step):
    n = sum(r.shape[0] for r in back_step["rho"].values())
    e, disc = _prev_bond_energy(step, back_step, n)
    assert abs(disc) < 1e-12
    assert abs(e - step["e_fci"]) < 1e-10


def test_backward_step_truncated_is_variational_and_monotone(step, back_step):
    es = [_prev_bond_energy(step, back_step, M)[0] for M in (4, 8, 16, 32)]
    assert all(e >= step["e_fci"] - 1e-10 for e in es)
    assert all(es[i + 1] <= es[i] + 1e-10 for i in range(len(es) - 1))
    assert es[0] > step["e_fci"] + 1e-6
