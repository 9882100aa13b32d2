"""Pins of two oracle helpers (CPU): the share mode of ``OracleHop`` (one device's share of the sum
over operator combinations, Section 2.2.1) and ``OracleHop.magnitude`` (the size of the summands of
every output element, the scale of the split-precision error bound).

Share mode is defined by Hamiltonian terms: a term (left operator) x (site part) x (right operator)
belongs to a share when its left and right block operators are both supplied. Pins:
* with every operator supplied the share is the whole H.psi;
* with exact blocks (every stored operator is the exact one), leaving out the left operators A_01
  and A_01^T (P_01 on the right pairs only with them), or B_02 and B_20, removes exactly the
  Hamiltonian terms whose left-block substring is that operator: H.psi - share.psi, embedded in the
  determinant space, equals those terms of Eq. H2q applied determinant by determinant (brute force
  with Jordan-Wigner signs, independent of the block machinery).
Magnitude pins: |H x| <= magnitude(x) element by element (triangle inequality), magnitude depends on
|x| only and is positively homogeneous and additive on non-negative vectors; a planted mistake
(the absolute value of f dropped) violates the first pin.
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals, random_vector
from dmrg_inputs.blocks import Block
from oracle.fci import determinants
from oracle.fock import embed, exact_block
from oracle.hamiltonian import spin_orbital_integrals
from oracle.hpsi import OracleHop

L, S1, NA, NB = 6, 2, 3, 3


@pytest.fixture(scope="module")
def exact6():
    h, eri = random_integrals(L, 17)
    t, w = spin_orbital_integrals(h, eri)
    left = exact_block(list(range(S1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= S1])
    right = exact_block(list(range(S1 + 2, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= S1 + 1])
    return h, eri, t, w, left, right


def without(block, drop):
    """The block with the operators (kind, i0, i1) in ``drop`` removed."""
    ops = [op for op in block.ops if (op.kind, op.i0, op.i1) not in drop]
    out = Block(side=block.side, orbitals=block.orbitals, qn=block.qn, dim=block.dim, ops=ops)
    out.fock = block.fock
    return out


def apply_terms(terms, x, dets):
    """sum over (coeff, ops) of coeff * ops applied to the determinant vector x, ops = [(dagger, P)]
    applied right to left with the sign (-1)^(occupied modes below P)."""
    y = np.zeros_like(x)
    index = {int(d): i for i, d in enumerate(dets)}
    for coeff, ops in terms:
        for i, d0 in enumerate(dets):
            if x[i] == 0.0:
                continue
            d, sign = int(d0), 1.0
            for dag, P in reversed(ops):
                bit = 1 << P
                if bool(d & bit) == dag:
                    sign = 0.0
                    break
                if bin(d & (bit - 1)).count("1") % 2:
                    sign = -sign
                d ^= bit
            if sign != 0.0:
                y[index[d]] += coeff * sign * x[i]
    return y


def h2q_terms(t, w):
    """Every term of Eq. H2q (spin-orbital form): (coefficient, operator string)."""
    terms = [(t[P, Q], [(True, P), (False, Q)]) for P, Q in zip(*np.nonzero(t))]
    terms += [(0.5 * w[P, Q, R, S], [(True, P), (True, Q), (False, R), (False, S)])
              for P, Q, R, S in zip(*np.nonzero(w))]
    return terms


def left_substring(ops):
    """(creators, annihilators) of the term's left-block operators, or None if every operator is in
    the left block (then the term belongs to the left block's Hamiltonian)."""
    left = [(d, P) for d, P in ops if P // 2 < S1]
    if len(left) == len(ops):
        return None
    return (tuple(sorted(P for d, P in left if d)), tuple(sorted(P for d, P in left if not d)))


def test_share_with_every_operator_is_the_whole_hpsi(exact6):
    h, eri, t, w, left, right = exact6
    x = random_vector(OracleHop(h, eri, left, right, NA, NB, S1).layout.size, 3)
    full = OracleHop(h, eri, left, right, NA, NB, S1).apply(x)
    share = OracleHop(h, eri, left, right, NA, NB, S1, share=True).apply(x)
    assert np.array_equal(full, share)


@pytest.mark.parametrize("drop_left,drop_right,missing", [
    ({("A", 0, 1)}, {("P", 0, 1)}, {((0, 1), ()), ((), (0, 1))}),
    ({("B", 0, 2), ("B", 2, 0)}, set(), {((0,), (2,)), ((2,), (0,))}),
])
def test_share_leaves_out_exactly_the_terms_of_the_missing_operators(exact6, drop_left, drop_right, missing):
    h, eri, t, w, left, right = exact6
    lp, rp = without(left, drop_left), without(right, drop_right)
    full_hop = OracleHop(h, eri, left, right, NA, NB, S1)
    x = random_vector(full_hop.layout.size, 5)
    diff = full_hop.apply(x) - OracleHop(h, eri, lp, rp, NA, NB, S1, share=True).apply(x)
    dets = determinants(L, NA, NB)
    terms = [(c, ops) for c, ops in h2q_terms(t, w) if left_substring(ops) in missing]
    assert terms
    want = apply_terms(terms, embed(full_hop.layout, x, left, right, S1, S1 + 1, dets), dets)
    got = embed(full_hop.layout, diff, left, right, S1, S1 + 1, dets)
    assert np.abs(got).max() > 1e-3
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_magnitude_bounds_and_scaling(exact6):
    h, eri, t, w, left, right = exact6
    oh = OracleHop(h, eri, left, right, NA, NB, S1)
    x = random_vector(oh.layout.size, 7)
    z = random_vector(oh.layout.size, 8)
    m = oh.magnitude(x)
    assert np.all(np.abs(oh.apply(x)) <= m * (1 + 1e-12) + 1e-300)
    assert np.array_equal(m, oh.magnitude(-x)) and np.array_equal(m, oh.magnitude(np.abs(x)))
    assert np.allclose(oh.magnitude(2.5 * x), 2.5 * m, rtol=1e-14, atol=0)
    assert np.allclose(oh.magnitude(np.abs(x) + np.abs(z)), m + oh.magnitude(z), rtol=1e-12, atol=0)
    # the bound is not vacuous: summands of one output element rarely all share a sign
    assert np.median(np.abs(oh.apply(x)) / np.maximum(m, 1e-300)) < 0.9


def test_planted_magnitude_mistake_is_caught(exact6, monkeypatch):
    h, eri, t, w, left, right = exact6
    oh = OracleHop(h, eri, left, right, NA, NB, S1)
    x = random_vector(oh.layout.size, 7)
    y = np.abs(oh.apply(x))
    # f without its absolute value: negative summands now subtract
    monkeypatch.setattr("oracle.hpsi.abs", lambda v: v, raising=False)
    assert np.any(y > oh.magnitude(x) * (1 + 1e-12))
