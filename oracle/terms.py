"""Expansion of H into operator combinations alpha = A_l x A_sl x A_sr x A_r (Section 2.2.1).

The superblock is left block | left site s1 | right site s2 | right block (Section 2.1, Fig. 1).
Every term of H (Eq. H2q in the spin-orbital reading of ``oracle.hamiltonian``) is taken one at a
time and written literally as a product of part-local operators:

1. a term whose indices all lie in one block is part of that block's Hamiltonian H_l or H_r;
2. otherwise its creation/annihilation operators are stably reordered into part order
   (left, s1, s2, right) and the permutation sign is kept (fermionic anticommutation);
3. the left-block substring becomes a stored operator (c+, c, A = c+c+, A^T, B = c+c) when it has
   at most two operators; a three-operator substring, summed over its block indices, must equal a
   multiple of the stored complementary-type operator S_W (or S_W^T); the right-block substring is
   c+ / c when it has one operator and otherwise, summed over its block indices, must equal a
   multiple of a stored complementary operator U, U^T, P, P^T or Q. These pre-summed operators
   (Section 2.1, pre-summed example and its footnote) are identified by accumulating the
   coefficient tensor over the summed indices and comparing it with the operator's definition;
   any mismatch raises.
4. site substrings become 4x4 matrices built from the site creation matrices (Eq. creation_ops,
   read in the basis order 0, up, down, updown with |updown> = a+_up a+_dn |0>).

The matrix of a product O_l O_1 O_2 O_r (fermion parities p_l, p_1, p_2, p_r) on the product basis
|l>|s1>|s2>|r> is (O_l P_l^(p_1+p_2+p_r)) x (O_1 P_1^(p_2+p_r)) x (O_2 P_2^(p_r)) x O_r, with P the
parity (-1)^n of the ket: each operator passes the creation strings of the parts to its left.

Combinations sharing the site matrices and the right-block operator are merged by summing their
left-block operators (the on-the-fly pre-summation of Section 2.2.3), giving the alpha list that
``oracle.hpsi`` applies with Eq. dgemm.
"""
from collections import defaultdict

import numpy as np

LEFT, SITE1, SITE2, RIGHT = 0, 1, 2, 3

# Site matrices in the basis (0, up, down, updown): a+_up = E10 + E32, a+_dn = E20 - E31.
A_UP = np.zeros((4, 4)); A_UP[1, 0] = 1.0; A_UP[3, 2] = 1.0
A_DN = np.zeros((4, 4)); A_DN[2, 0] = 1.0; A_DN[3, 1] = -1.0
SITE_PARITY = np.diag([1.0, -1.0, -1.0, 1.0])


def site_op(dag, mode):
    m = A_UP if mode % 2 == 0 else A_DN
    return m if dag else m.T


def site_matrix(string):
    M = np.eye(4)
    for dag, mode in string:
        M = M @ site_op(dag, mode)
    return M


def _perm_sign(parts):
    inv = 0
    for i in range(len(parts)):
        for j in range(i + 1, len(parts)):
            if parts[i] > parts[j]:
                inv += 1
    return -1.0 if inv % 2 else 1.0


def _left_individual(sub):
    """Left-block substring of <= 2 operators -> (op descriptor, sign) or None if identically zero."""
    if len(sub) == 0:
        return ("I", -1, -1, False), 1.0
    if len(sub) == 1:
        dag, P = sub[0]
        return ("C", P, -1, not dag), 1.0
    (d0, P), (d1, Q) = sub
    if d0 and d1:                     # c+_P c+_Q
        if P == Q:
            return None
        return (("A", P, Q, False), 1.0) if P < Q else (("A", Q, P, False), -1.0)
    if not d0 and not d1:             # c_P c_Q = (c+_Q c+_P)^T
        if P == Q:
            return None
        return (("A", Q, P, True), 1.0) if Q < P else (("A", P, Q, True), -1.0)
    if d0 and not d1:                 # c+_P c_Q
        return ("B", P, Q, False), 1.0
    raise AssertionError("substring not normal-ordered")


def _right_individual(sub):
    if len(sub) == 0:
        return ("I", -1, -1, False)
    assert len(sub) == 1
    dag, Z = sub[0]
    return ("C", Z, -1, not dag)


def _n_ops(desc):
    kind, i0, i1, _ = desc
    return {"I": 0, "C": 1, "A": 2, "B": 2, "S": 3, "U": 3, "P": 2, "Q": 2, "H": 0}[kind]


def _antisym(T, axes):
    return T - np.swapaxes(T, *axes)


class _Pending:
    """Coefficient tensor of a block substring whose indices are summed into a stored operator."""

    def __init__(self, nidx, n):
        self.T = np.zeros((n,) * nidx)

    def add(self, idx, v):
        self.T[idx] += v


def expand(t, w, n_orb, s1, tol=1e-11):
    """Return the merged alpha list for the bond with left site ``s1`` (right site s1+1).

    Each alpha is a dict with keys ``left`` (list of (coeff, op descriptor)), ``s1``, ``s2``
    (site substrings), ``right`` (op descriptor) and ``coeff`` (overall scalar, 1 after merging),
    where an op descriptor is ``(kind, i0, i1, transposed)``.
    """
    n = 2 * n_orb
    s2 = s1 + 1
    part = np.array([LEFT if P // 2 < s1 else SITE1 if P // 2 == s1 else SITE2 if P // 2 == s2
                     else RIGHT for P in range(n)])
    individual = defaultdict(float)         # (Ldesc, s1str, s2str, Rdesc) -> coefficient
    pend_right = {}                         # (Ldesc, s1str, s2str, pattern) -> _Pending
    pend_left = {}                          # (pattern, s1str, s2str, Rdesc) -> _Pending

    def process(coeff, ops):
        parts = [part[i] for _, i in ops]
        if all(p == LEFT for p in parts) or all(p == RIGHT for p in parts):
            return                          # part of H_l or H_r
        order = sorted(range(len(ops)), key=lambda k: parts[k])
        sign = _perm_sign(parts)
        subs = [[ops[k] for k in order if parts[k] == p] for p in range(4)]
        s1str, s2str = tuple(subs[SITE1]), tuple(subs[SITE2])
        lsub, rsub = subs[LEFT], subs[RIGHT]
        c = coeff * sign
        if len(lsub) == 3:
            pattern = tuple(d for d, _ in lsub)
            rdesc = _right_individual(rsub)
            key = (pattern, s1str, s2str, rdesc)
            if key not in pend_left:
                pend_left[key] = _Pending(3, n)
            pend_left[key].add(tuple(i for _, i in lsub), c)
            return
        li = _left_individual(lsub)
        if li is None:
            return
        ldesc, lsign = li
        c *= lsign
        if len(rsub) >= 2:
            pattern = tuple(d for d, _ in rsub)
            key = (ldesc, s1str, s2str, pattern)
            if key not in pend_right:
                pend_right[key] = _Pending(len(rsub), n)
            pend_right[key].add(tuple(i for _, i in rsub), c)
            return
        individual[(ldesc, s1str, s2str, _right_individual(rsub))] += c

    for P, Q in zip(*np.nonzero(t)):
        process(t[P, Q], [(True, int(P)), (False, int(Q))])
    for P, Q, R, S in zip(*np.nonzero(w)):
        process(0.5 * w[P, Q, R, S], [(True, int(P)), (True, int(Q)), (False, int(R)), (False, int(S))])

    combos = defaultdict(float)
    for k, v in individual.items():
        if v != 0.0:
            combos[k] += v

    def outside(ldesc, s1str, s2str, rdesc=None):
        cre, ann = [], []
        kind, i0, i1, tr = ldesc
        if kind == "C":
            (ann if tr else cre).append(i0)
        elif kind == "A":
            (ann if tr else cre).extend([i0, i1])
        elif kind == "B":
            cre.append(i0); ann.append(i1)
        for dag, m in list(s1str) + list(s2str):
            (cre if dag else ann).append(m)
        if rdesc is not None and rdesc[0] == "C":
            (ann if rdesc[3] else cre).append(rdesc[1])
        return cre, ann

    in_right = part == RIGHT
    in_left = part == LEFT

    def restrict(D, mask):
        for ax in range(D.ndim):
            shape = [1] * D.ndim
            shape[ax] = -1
            D = D * mask.reshape(shape)
        return D

    def identify(T, D, axes, mask):
        D = restrict(D, mask)
        Ta, Da = (_antisym(T, axes), _antisym(D, axes)) if axes else (T, D)
        dd = float(np.vdot(Da, Da))
        scale = max(np.abs(Ta).max(), np.abs(Da).max(), 1e-300)
        if dd == 0.0:
            if np.abs(Ta).max() > tol * max(scale, 1.0):
                raise ValueError("pre-summed operator does not match any stored definition")
            return 0.0
        lam = float(np.vdot(Ta, Da)) / dd
        if np.abs(Ta - lam * Da).max() > tol * scale:
            raise ValueError("pre-summed operator is not a multiple of the stored definition")
        return lam

    for (ldesc, s1str, s2str, pattern), pend in pend_right.items():
        cre, ann = outside(ldesc, s1str, s2str)
        if pattern == (False, False):
            P, Q = sorted(cre)
            D = w[P, Q, :, :]
            lam, rdesc = identify(pend.T, D, (0, 1), in_right), ("P", P, Q, False)
        elif pattern == (True, True):
            P, Q = sorted(ann)
            D = np.transpose(w[P, Q, :, :])           # coefficient of c+_A c+_B is w[P,Q,B,A]
            lam, rdesc = identify(pend.T, D, (0, 1), in_right), ("P", P, Q, True)
        elif pattern == (True, False):
            (X,), (Y,) = cre, ann
            D = w[X, :, :, Y] - w[X, :, Y, :]
            lam, rdesc = identify(pend.T, D, None, in_right), ("Q", X, Y, False)
        elif pattern == (True, False, False):
            (P,) = cre
            D = w[P, :, :, :]
            lam, rdesc = identify(pend.T, D, (1, 2), in_right), ("U", P, -1, False)
        elif pattern == (True, True, False):
            (P,) = ann
            D = np.transpose(w[P, :, :, :], (2, 1, 0))  # c+_A c+_B c_C : w[P, C, B, A]
            lam, rdesc = identify(pend.T, D, (0, 1), in_right), ("U", P, -1, True)
        else:
            raise AssertionError(pattern)
        if lam != 0.0:
            combos[(ldesc, s1str, s2str, rdesc)] += lam

    for (pattern, s1str, s2str, rdesc), pend in pend_left.items():
        cre, ann = outside(("I", -1, -1, False), s1str, s2str, rdesc)
        if pattern == (True, True, False):
            (W,) = ann
            D = w[:, :, :, W]
            lam, ldesc = identify(pend.T, D, (0, 1), in_left), ("S", W, -1, False)
        elif pattern == (True, False, False):
            (W,) = cre
            D = np.transpose(w[:, :, :, W], (2, 1, 0))  # c+_X c_Y c_Z : w[Z, Y, X, W]
            lam, ldesc = identify(pend.T, D, (1, 2), in_left), ("S", W, -1, True)
        else:
            raise AssertionError(pattern)
        if lam != 0.0:
            combos[(ldesc, s1str, s2str, rdesc)] += lam

    combos[(("H", -1, -1, False), (), (), ("I", -1, -1, False))] += 1.0
    combos[(("I", -1, -1, False), (), (), ("H", -1, -1, False))] += 1.0

    # Pre-sum left-block operators that share site substrings and the right-block operator.
    groups = defaultdict(list)
    for (ldesc, s1str, s2str, rdesc), v in combos.items():
        if v != 0.0:
            groups[(s1str, s2str, rdesc)].append((v, ldesc))
    alphas = []
    for (s1str, s2str, rdesc), left in sorted(groups.items(), key=lambda kv: repr(kv[0])):
        pr, p2, p1 = _n_ops(rdesc) % 2, len(s2str) % 2, len(s1str) % 2
        e2 = pr
        e1 = (p2 + pr) % 2
        eL = (p1 + p2 + pr) % 2
        S1 = site_matrix(s1str) @ np.linalg.matrix_power(SITE_PARITY, e1)
        S2 = site_matrix(s2str) @ np.linalg.matrix_power(SITE_PARITY, e2)
        alphas.append(dict(left=sorted(left, key=repr), s1=s1str, s2=s2str, right=rdesc,
                           S1=S1, S2=S2, eL=eL))
    return alphas
