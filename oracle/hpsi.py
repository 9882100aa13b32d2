"""Two-site H.psi by sector GEMMs (Eq. dgemm, Section 2.2.1) and the Hamiltonian diagonal.

For every operator combination alpha (from ``oracle.terms``) and every sector block phi^s of the
input, the target block s' and the scalar f(s) follow from the sector change of each operator and
the site-matrix elements, and

    phi~^{s'} += f(s) * A_l^{(alpha, s, s')} . phi^s . (A_r^{(alpha, s, s')})^T .

The left operator of a combination is the pre-sum of stored left-block operators formed by
``oracle.terms``; it is assembled here block by block (Section 2.2.3).
"""
import numpy as np

from .hamiltonian import spin_orbital_integrals
from .layout import Layout
from .terms import expand


def _op_blocks(block, desc):
    """Sector blocks {(so, si): matrix} of a stored operator descriptor (transposed if asked)."""
    kind, i0, i1, tr = desc
    op = block.get(kind, i0, i1)
    if op is None and kind in ("B", "Q"):
        # c+_Q c_P = (c+_P c_Q)^T and likewise for Q: a block may store only one of each pair
        op = block.get(kind, i1, i0)
        tr = not tr
    if op is None:
        raise KeyError(f"{block.side} block lacks operator {kind}({i0},{i1})")
    if not tr:
        return dict(op.blocks)
    return {(si, so): m.T for (so, si), m in op.blocks.items()}


def presum_left(block, terms):
    """sum_k coeff_k * op_k over stored left operators -> {(so, si): matrix}."""
    out = {}
    for coeff, desc in terms:
        if desc[0] == "I":
            blocks = {(i, i): np.eye(int(block.dim[i])) for i in range(block.n_sec)}
        else:
            blocks = _op_blocks(block, desc)
        for k, m in blocks.items():
            if k in out:
                out[k] = out[k] + coeff * m
            else:
                out[k] = coeff * m
    return out


class OracleHop:
    """H.psi at the bond (s1, s1+1) for given left/right blocks, following Section 2.2.1."""

    def __init__(self, h, eri, left, right, n_alpha, n_beta, s1, alphas=None, share=False):
        """share: one device's share of the sum over combinations (Section 2.2.1 distributes them):
        H restricted to the terms (left operator) x (site part) x (right operator) whose left and
        right block operators are both supplied by the blocks -- a pre-summed left operator keeps
        its supplied summands, a combination whose right operator is missing is left out."""
        self.left, self.right = left, right
        self.layout = Layout(left, right, n_alpha, n_beta)
        t, w = spin_orbital_integrals(h, eri)
        self.alphas = alphas if alphas is not None else expand(t, w, h.shape[0], s1)
        if share:
            self.alphas = self._share(self.alphas)
        self._prepare()

    def _supplied(self, block, desc):
        kind, i0, i1, _ = desc
        if kind == "I":
            return True
        if block.get(kind, i0, i1) is not None:
            return True
        return kind in ("B", "Q") and block.get(kind, i1, i0) is not None

    def _share(self, alphas):
        kept = []
        for al in alphas:
            if not self._supplied(self.right, al["right"]):
                continue
            left = [(c, d) for c, d in al["left"] if self._supplied(self.left, d)]
            if left:
                kept.append(dict(al, left=left))
        return kept

    def _prepare(self):
        lnum = self.left.qn.sum(axis=1)
        self.ops = []
        for al in self.alphas:
            if len(al["left"]) == 1 and al["left"][0][1][0] == "I":
                lmat = None
                lcoef = al["left"][0][0]
            else:
                lmat = {si: (so, m) for (so, si), m in presum_left(self.left, al["left"]).items()}
                assert len(lmat) == len(presum_left(self.left, al["left"])), "mixed sector change"
                lcoef = 1.0
            if al["right"][0] == "I":
                rmat = None
            else:
                rmat = {si: (so, m) for (so, si), m in _op_blocks(self.right, al["right"]).items()}
            self.ops.append((lmat, lcoef, rmat, al["S1"], al["S2"], al["eL"]))
        self.lparity = (-1.0) ** lnum

    def tasks(self):
        """List of (source block, target block, f, left matrix or None, right matrix or None)."""
        if getattr(self, "_tasks", None) is None:
            self._tasks = list(self._gen_tasks())
        return self._tasks

    def target_tasks(self, targets):
        """Tasks writing into the given output blocks (not cached)."""
        targets = set(targets)
        return [tk for tk in self._gen_tasks() if tk[1] in targets]

    def _gen_tasks(self):
        index = self.layout.index
        for lmat, lcoef, rmat, S1, S2, eL in self.ops:
            for i, (a, b, c, d, off, ma, md) in enumerate(self.layout.blocks):
                bp = np.nonzero(S1[:, b])[0]
                cp = np.nonzero(S2[:, c])[0]
                if bp.size == 0 or cp.size == 0:
                    continue
                assert bp.size == 1 and cp.size == 1
                bp, cp = int(bp[0]), int(cp[0])
                if lmat is None:
                    ap, A = a, None
                else:
                    if a not in lmat:
                        continue
                    ap, A = lmat[a]
                if rmat is None:
                    dp, B = d, None
                else:
                    if d not in rmat:
                        continue
                    dp, B = rmat[d]
                j = index.get((ap, bp, cp, dp))
                if j is None:
                    raise AssertionError("operator combination leaves the (N_alpha, N_beta) sector")
                f = lcoef * S1[bp, b] * S2[cp, c] * (self.lparity[a] if eL else 1.0)
                yield i, j, f, A, B

    def apply(self, x, targets=None, tasks=None):
        """y = H x (x of shape (n,) or (n, nvec)); with ``targets`` (or a task subset) only those blocks."""
        lay = self.layout
        x2 = x.reshape(lay.size, -1)
        y = np.zeros_like(x2)
        nv = x2.shape[1]
        if tasks is None:
            tasks = self.tasks() if targets is None else self.target_tasks(targets)
        for i, j, f, A, B in tasks:
            _, _, _, _, off, ma, md = lay.blocks[i]
            _, _, _, _, offj, mj, nj = lay.blocks[j]
            X = x2[off:off + ma * md].reshape(ma, md * nv)           # columns (r, v)
            T = X if A is None else A @ X                             # (mj, md * nv)
            if B is not None:
                T = (B @ T.reshape(mj, md, nv).transpose(1, 0, 2).reshape(md, mj * nv))
                T = T.reshape(nj, mj, nv).transpose(1, 0, 2)
            y[offj:offj + mj * nj] += f * T.reshape(mj * nj, nv)
        return y.reshape(x.shape)

    def magnitude(self, x, targets=None, tasks=None):
        """sum over tasks of |f| |A| |X| |B|^T (absolute values taken element by element): the size
        of the summands of every output element, which bounds the rounding error of a summation in
        any order and precision of the same summands (x of shape (n,))."""
        lay = self.layout
        ax = np.abs(x)
        y = np.zeros_like(ax)
        if tasks is None:
            tasks = self.tasks() if targets is None else self.target_tasks(targets)
        for i, j, f, A, B in tasks:
            _, _, _, _, off, ma, md = lay.blocks[i]
            _, _, _, _, offj, mj, nj = lay.blocks[j]
            T = ax[off:off + ma * md].reshape(ma, md)
            if A is not None:
                T = np.abs(A) @ T
            if B is not None:
                T = T @ np.abs(B).T
            y[offj:offj + mj * nj] += abs(f) * T.ravel()
        return y

    def diagonal(self):
        """diag(H): sum over combinations mapping a block to itself of f diag(A_l) diag(A_r)^T."""
        lay = self.layout
        D = np.zeros(lay.size)
        for i, j, f, A, B in self.tasks():
            if i != j:
                continue
            _, _, _, _, off, ma, md = lay.blocks[i]
            da = np.ones(ma) if A is None else np.diag(A)
            db = np.ones(md) if B is None else np.diag(B)
            D[off:off + ma * md] += f * np.outer(da, db).ravel()
        return D

    def flops(self, tasks=None):
        """Algorithmic flops of one H.psi: per task 2 MACs of the cheaper association."""
        lay = self.layout
        total = 0.0
        for i, j, f, A, B in (self.tasks() if tasks is None else tasks):
            ma, md = lay.blocks[i][5], lay.blocks[i][6]
            mj, nj = lay.blocks[j][5], lay.blocks[j][6]
            if A is None and B is None:
                continue
            if A is None:
                total += 2.0 * ma * md * nj
            elif B is None:
                total += 2.0 * mj * ma * md
            else:
                total += 2.0 * min(mj * ma * md + mj * md * nj, ma * md * nj + mj * ma * nj)
        return total
