"""Operators of the grown left block (block X plus the next site s) in the product basis |l>|s>, built
from X's stored normal operators (H, C, A, B, S) and the site matrices of Eq. creation_ops -- the
"operator matrices formed for the enlarged block" that Eq. renorm_mat then truncates (Section 2.1).
TEST INFRASTRUCTURE ONLY (plain FP64 NumPy; see the package header for who may import it).

Each grown-block operator is the sum of its defining operator strings (``dmrg_inputs.blocks`` lists
the definitions). A string is split into its X part and its site part with the sign of moving the
site operators to the right (different modes anticommute). With the Jordan-Wigner order of X before
s, an X operator acts as x (x) 1 and a site operator as P_X (x) a, P_X the parity of X's state, so a
string with m site operators becomes (x_string P_X^m) (x) site_string. An X part is never formed
as a product of X's matrices (its truncated basis is not complete, Section 2.1): one operator is C or
C^T, two are A, A^T or B (with c_R c+_P = delta_RP - c+_P c_R), and the three-operator strings of H
are collected into S: the terms of H with one index on the site add up to S(W) c_W + c+_W S(W)^T
(W on the site), using w_PQRS = w_QPSR. Four X operators are X's own H.

Product index of |l>|s>: 4 * (sector offset of l + position of l) + s, sectors in X's order.
"""
import numpy as np

from dmrg_inputs.blocks import Block, Op
from oracle import renorm
from oracle.terms import SITE_PARITY, site_matrix, site_op


class GrownLeft:
    def __init__(self, block, t, w, site):
        """block: left block X (normal set) over orbitals 0 .. site-1; t, w: spin-orbital integrals."""
        self.X, self.t, self.w, self.site = block, t, w, site
        self.off = np.concatenate([[0], np.cumsum(block.dim)]).astype(np.int64)
        self.nx = int(self.off[-1])
        self.n = 4 * self.nx
        par = np.concatenate([np.full(int(d), (-1.0) ** (int(q[0]) + int(q[1]))) for q, d in zip(block.qn, block.dim)]) \
            if self.nx else np.zeros(0)
        self.par = np.diag(par)
        self.xmodes = list(range(2 * site))
        self.smodes = [2 * site, 2 * site + 1]
        self.modes = self.xmodes + self.smodes

    # ---------------------------------------------------------------- X's stored operators, dense
    def _dense(self, op):
        D = np.zeros((self.nx, self.nx))
        if op is None:
            return D
        for (so, si), m in op.blocks.items():
            D[self.off[so]:self.off[so + 1], self.off[si]:self.off[si + 1]] = m
        return D

    def _x(self, kind, i0=-1, i1=-1):
        op = self.X.get(kind, i0, i1)
        if op is None and kind == "B":                     # B_QP = B_PQ^T (real orbitals)
            alt = self.X.get("B", i1, i0)
            return self._dense(alt).T if alt is not None else np.zeros((self.nx, self.nx))
        return self._dense(op)

    def x_string(self, xs):
        """Matrix of an X-only string of at most two operators, from X's stored operators."""
        if len(xs) == 0:
            return np.eye(self.nx)
        if len(xs) == 1:
            dag, P = xs[0]
            C = self._x("C", P)
            return C if dag else C.T
        if len(xs) == 2:
            (d1, P), (d2, Q) = xs
            if d1 and d2:
                if P == Q:
                    return np.zeros((self.nx, self.nx))
                return self._x("A", P, Q) if P < Q else -self._x("A", Q, P)
            if not d1 and not d2:                          # c_P c_Q = (c+_Q c+_P)^T
                return self.x_string([(1, Q), (1, P)]).T
            if d1:                                         # c+_P c_Q
                return self._x("B", P, Q)
            return (np.eye(self.nx) if P == Q else 0.0) - self._x("B", Q, P)   # c_P c+_Q
        raise ValueError("X strings of three or more operators are only available through S and H")

    def term(self, coef, string):
        """coef * string (a list of (dagger, mode)) as a product-basis matrix."""
        xs = [e for e in string if e[1] < 2 * self.site]
        ss = [e for e in string if e[1] >= 2 * self.site]
        swaps = 0
        for i, e in enumerate(string):                     # site operators moved right past X operators
            if e[1] >= 2 * self.site:
                swaps += sum(1 for f in string[i + 1:] if f[1] < 2 * self.site)
        X = self.x_string(xs) @ np.linalg.matrix_power(self.par, len(ss)) if self.nx else np.zeros((0, 0))
        return coef * (-1.0) ** swaps * np.kron(X, site_matrix(ss))

    # ---------------------------------------------------------------- grown-block operators
    def H(self):
        M = np.kron(self._x("H"), np.eye(4))
        xset = set(self.xmodes)
        for P in self.modes:
            for Q in self.modes:
                if self.t[P, Q] != 0.0 and not (P in xset and Q in xset):
                    M += self.term(self.t[P, Q], [(1, P), (0, Q)])
        for P in self.modes:
            for Q in self.modes:
                for R in self.modes:
                    for S in self.modes:
                        v = self.w[P, Q, R, S]
                        nx = (P in xset) + (Q in xset) + (R in xset) + (S in xset)
                        if v != 0.0 and nx <= 2:
                            M += self.term(0.5 * v, [(1, P), (1, Q), (0, R), (0, S)])
        for W in self.smodes:                              # three X indices: S(W) c_W + c+_W S(W)^T
            Sx = self._x("S", W)
            M += np.kron(Sx @ self.par, site_op(False, W)) + np.kron(self.par @ Sx.T, site_op(True, W))
        return M

    def C(self, P):
        return self.term(1.0, [(1, P)])

    def A(self, P, Q):
        return self.term(1.0, [(1, P), (1, Q)])

    def B(self, P, Q):
        return self.term(1.0, [(1, P), (0, Q)])

    def S(self, W):
        """S'(W) = sum over P, Q, R in X + s of w_PQRW c+_P c+_Q c_R, for W right of the site."""
        xset = set(self.xmodes)
        M = np.kron(self._x("S", W), np.eye(4))
        for P in self.modes:
            for Q in self.modes:
                for R in self.modes:
                    v = self.w[P, Q, R, W]
                    if v != 0.0 and not (P in xset and Q in xset and R in xset):
                        M += self.term(v, [(1, P), (1, Q), (0, R)])
        return M

    # ---------------------------------------------------------------- sector form and renormalization
    def sector_map(self):
        """Product index -> (q, index inside q) in the enlarged-left order of ``oracle.renorm``."""
        parts, dims = renorm.enlarged_left_basis(self.X)
        pos = {}
        for q in parts:
            for a, b, st, m in parts[q]:
                for l in range(m):
                    pos[4 * (int(self.off[a]) + l) + b] = (q, st + l)
        return pos, dims

    def to_sectors(self, M):
        """Dense product-basis matrix -> {(q_out, q_in): block} in the enlarged-left sector bases."""
        pos, dims = self.sector_map()
        idx = {q: np.zeros(dims[q], dtype=np.int64) for q in dims}
        for p, (q, i) in pos.items():
            idx[q][i] = p
        out = {}
        for qo in dims:
            for qi in dims:
                blk = M[np.ix_(idx[qo], idx[qi])]
                if np.any(blk):
                    out[(qo, qi)] = blk
        return out

    def renormalized_block(self, O):
        """The grown block's normal operator set renormalized by O (Eq. renorm_mat), as a Block over
        orbitals 0 .. site whose sectors are the q that keep states, in ascending q."""
        qs = sorted(O)
        sidx = {q: i for i, q in enumerate(qs)}
        L = self.w.shape[0] // 2

        def op(kind, i0, i1, M):
            r = renorm.renormalize(self.to_sectors(M), O, O)
            return Op(kind, i0, i1, {(sidx[a], sidx[b]): m for (a, b), m in r.items() if np.any(m)})

        ops = [op("H", -1, -1, self.H())]
        ops += [op("C", P, -1, self.C(P)) for P in self.modes]
        ops += [op("A", P, Q, self.A(P, Q)) for P in self.modes for Q in self.modes if P < Q]
        ops += [op("B", P, Q, self.B(P, Q)) for P in self.modes for Q in self.modes]
        ops += [op("S", W, -1, self.S(W)) for W in range(2 * self.site + 2, 2 * L)]
        return Block(side="left", orbitals=tuple(range(self.site + 1)), qn=np.array(qs, dtype=np.int32),
                     dim=np.array([O[q].shape[1] for q in qs], dtype=np.int32), ops=ops)


# ---------------------------------------------------------------- growth by the Fock-space route
def _fock_basis(block):
    """(root exact block, per-sector basis columns over the root's sector states) of a block built by
    ``oracle.fock`` (exact, or truncated by projection)."""
    if hasattr(block, "bases"):
        root = block.parent
        ridx = root.sector_index()
        return root, {i: (ridx[(int(q[0]), int(q[1]))], block.bases[i]) for i, q in enumerate(block.qn)}
    return block, {i: (i, np.eye(int(block.dim[i]))) for i in range(block.n_sec)}


def grown_block(side, block, site, O, t, w):
    """The block grown by one site and renormalized by O (Eq. renorm_mat), from the definition: every
    operator of the grown orbital set taken exactly in its own Fock space (``oracle.fock``) and
    projected onto the kept basis. Valid for blocks whose operators are projections of the exact
    ones (exact blocks and their truncations), which is what Section 2.1 asks of stored operators.

    side  : "left" (block = orbitals 0 .. site-1, grown by orbital ``site``) or "right" (block =
            orbitals site+1 .. L-1, grown by orbital ``site``, i.e. the site becomes the first orbital)
    O     : enlarged sector q -> (dim_q, kept_q) orthonormal columns, rows in the enlarged basis of
            ``oracle.renorm.enlarged_left_basis`` / ``enlarged_right_basis`` of ``block``
    Returns the renormalized Block (sectors = the q with kept_q > 0, ascending), with ``bases`` over
    the grown orbitals' Fock space (so it can grow again).
    """
    from oracle.fock import exact_block
    n_modes = t.shape[0]
    L = n_modes // 2
    root, basis = _fock_basis(block)
    k = len(block.orbitals)
    if side == "left":
        orbitals = tuple(range(0, site + 1))
        outside = [P for P in range(n_modes) if P // 2 > site]
        parts, dims = renorm.enlarged_left_basis(block)
    else:
        orbitals = tuple(range(site, L))
        outside = [P for P in range(n_modes) if P // 2 < site]
        parts, dims = renorm.enlarged_right_basis(block)
    grown = exact_block(list(orbitals), side, t, w, outside)
    F = grown.fock
    Froot = getattr(root, "fock", None)
    gidx = {tuple(int(v) for v in q): i for i, q in enumerate(grown.qn)}
    pos = {}                                      # grown Fock state -> (sector, position)
    for i, states in enumerate(F.sector_states):
        for p, s in enumerate(states):
            pos[int(s)] = (i, p)
    bases = [np.zeros((int(d), 0)) for d in grown.dim]
    for q in dims:
        if q not in O or O[q].shape[1] == 0:
            continue
        gi = gidx[q]
        E = np.zeros((int(grown.dim[gi]), dims[q]))   # enlarged basis of sector q over the grown Fock states
        for entry in parts[q]:
            if side == "left":
                a, s, st, m = entry
            else:
                s, a, st, m = entry
            ri, V = basis[a]
            states = Froot.sector_states[ri] if Froot is not None else np.zeros(1, dtype=np.int64)
            for col in range(m):
                for r, x in enumerate(states):
                    if V[r, col] == 0.0:
                        continue
                    # product state -> grown Fock determinant, sign +1 (ascending modes, parts in order)
                    g = (int(x) | (s << (2 * k))) if side == "left" else (s | (int(x) << 2))
                    sec, p = pos[g]
                    assert sec == gi
                    E[p, st + col] += V[r, col]
        bases[gi] = E @ O[q]
    from oracle.fock import truncate
    return truncate(grown, bases)
