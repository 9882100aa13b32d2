"""Exact block operators from a block's full Fock space (Section 2.1).

For a block of ``k`` contiguous orbitals the Fock space has 4^k determinants ``|n>`` (bit ``2j+s``
for the j-th orbital of the block, Jordan-Wigner order inside the block = global order restricted to
the block). Every operator the H.psi expansion needs is formed here from its definition by explicit
products of creation/annihilation matrices and integral sums, then cut into (n_alpha, n_beta) sector
blocks. With all 4^k states kept (M = 4^k) every stored operator is exactly the projection of the
true operator, which Section 2.1 requires of the renormalized operators.

A block can also be truncated to a subspace: ``truncate(block, bases)`` projects every operator
onto caller-given orthonormal per-sector bases (``O^T A O`` of Eq. renorm_mat), which keeps the
"projection of the exact operator" property.

The superblock basis |l>|s1>|s2>|r> with Fock-determinant block states maps one-to-one onto global
determinants with sign +1 (each part's creation string is in ascending mode order and the parts are
ordered along the lattice); ``embed`` / ``project`` use that map.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from dmrg_inputs.blocks import Block, Op


def _popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


class FockSpace:
    """Fock space of ``k`` orbitals with sector bookkeeping."""

    def __init__(self, k):
        self.k = k
        self.n_modes = 2 * k
        self.size = 4 ** k
        states = np.arange(self.size, dtype=np.int64)
        even = sum(1 << (2 * j) for j in range(k))
        odd = sum(1 << (2 * j + 1) for j in range(k))
        na = _popcount(states & even)
        nb = _popcount(states & odd)
        self.qn_list = [(a, b) for a in range(k + 1) for b in range(k + 1)]
        self.sector_states = [states[(na == a) & (nb == b)] for (a, b) in self.qn_list]
        self.qn = np.array(self.qn_list, dtype=np.int32)
        self.dim = np.array([s.size for s in self.sector_states], dtype=np.int32)
        # position of each state inside its sector
        self.sector_of = np.zeros(self.size, dtype=np.int64)
        self.pos_in = np.zeros(self.size, dtype=np.int64)
        for i, s in enumerate(self.sector_states):
            self.sector_of[s] = i
            self.pos_in[s] = np.arange(s.size)
        self._c = [self._creation(m) for m in range(self.n_modes)]

    def _creation(self, m):
        states = np.arange(self.size, dtype=np.int64)
        bit = np.int64(1) << m
        ok = (states & bit) == 0
        src = states[ok]
        sign = 1.0 - 2.0 * (_popcount(src & (bit - 1)) & 1)
        return sp.csr_matrix((sign, (src | bit, src)), shape=(self.size, self.size))

    def c(self, m):
        """c+ of local mode m (sparse, size x size)."""
        return self._c[m]

    def cd(self, m):
        """Annihilator c of local mode m."""
        return self._c[m].T.tocsr()

    def sector_blocks(self, O, delta, drop_zero=True):
        """Cut a full-space operator with particle change ``delta`` into sector blocks."""
        O = sp.csr_matrix(O)
        idx = {q: i for i, q in enumerate(self.qn_list)}
        blocks = {}
        for si, (a, b) in enumerate(self.qn_list):
            so = idx.get((a + delta[0], b + delta[1]))
            if so is None:
                continue
            blk = O[self.sector_states[so], :][:, self.sector_states[si]].toarray()
            if drop_zero and not np.any(blk):
                continue
            blocks[(so, si)] = blk
        return blocks


def _delta(creators, annihilators):
    """Particle-number change (d_alpha, d_beta) of a product of spin-orbital operators."""
    d = [0, 0]
    for P in creators:
        d[P % 2] += 1
    for P in annihilators:
        d[P % 2] -= 1
    return tuple(d)


def exact_block(orbitals, side, t, w, outside):
    """Exact operator set of a block (see ``dmrg_inputs.blocks`` for the definitions).

    orbitals : contiguous spatial orbitals of the block
    side     : "left" (normal set: H, C, A, B, S) or "right" (complementary set: H, C, U, P, Q)
    t, w     : spin-orbital integrals (``oracle.hamiltonian``)
    outside  : spin-orbital ids outside the block for the one/two-index complementary operators
               (right of the block for S; left of it for U, P, Q)
    """
    k = len(orbitals)
    F = FockSpace(k)
    base = 2 * orbitals[0] if k else 0    # a block with no orbitals (edge bond): the vacuum only
    modes = list(range(2 * k))            # local mode m <-> global spin-orbital base + m
    g = [base + m for m in modes]
    C = [F.c(m) for m in modes]
    D = [F.cd(m) for m in modes]
    ops = []
    zero = sp.csr_matrix((F.size, F.size))

    # Block Hamiltonian: sum t c+c + 1/2 sum w c+c+cc over block indices.
    H = zero.copy()
    for i in modes:
        for j in modes:
            if t[g[i], g[j]] != 0.0:
                H = H + t[g[i], g[j]] * (C[i] @ D[j])
    for i in modes:
        for j in modes:
            inner = zero.copy()
            for m in modes:
                for n in modes:
                    v = w[g[i], g[j], g[m], g[n]]
                    if v != 0.0:
                        inner = inner + v * (D[m] @ D[n])
            if inner.nnz:
                H = H + 0.5 * (C[i] @ C[j] @ inner)
    ops.append(Op("H", -1, -1, F.sector_blocks(H, (0, 0))))
    for i in modes:
        ops.append(Op("C", g[i], -1, F.sector_blocks(C[i], _delta([g[i]], []))))

    if side == "left":
        for i, j in itertools.combinations(modes, 2):
            ops.append(Op("A", g[i], g[j], F.sector_blocks(C[i] @ C[j], _delta([g[i], g[j]], []))))
        for i in modes:
            for j in modes:
                ops.append(Op("B", g[i], g[j], F.sector_blocks(C[i] @ D[j], _delta([g[i]], [g[j]]))))
        for W in outside:
            S = zero.copy()
            for i in modes:
                for j in modes:
                    for m in modes:
                        v = w[g[i], g[j], g[m], W]
                        if v != 0.0:
                            S = S + v * (C[i] @ C[j] @ D[m])
            ops.append(Op("S", W, -1, F.sector_blocks(S, _delta([W], []))))
    else:
        # pair intermediates c_Z c_W and c+_Z c_W inside the block
        DD = {(m, n): D[m] @ D[n] for m in modes for n in modes}
        CD = {(m, n): C[m] @ D[n] for m in modes for n in modes}
        for P in outside:
            U = zero.copy()
            for q in modes:
                inner = zero.copy()
                for m in modes:
                    for n in modes:
                        v = w[P, g[q], g[m], g[n]]
                        if v != 0.0:
                            inner = inner + v * DD[m, n]
                if inner.nnz:
                    U = U + C[q] @ inner
            ops.append(Op("U", P, -1, F.sector_blocks(U, _delta([], [P]))))
        for P, Q in itertools.combinations(sorted(outside), 2):
            Pm = zero.copy()
            for m in modes:
                for n in modes:
                    v = w[P, Q, g[m], g[n]]
                    if v != 0.0:
                        Pm = Pm + v * DD[m, n]
            ops.append(Op("P", P, Q, F.sector_blocks(Pm, _delta([], [P, Q]))))
        for X in outside:
            for Y in outside:
                Qm = zero.copy()
                for m in modes:
                    for n in modes:
                        v = w[X, g[m], g[n], Y] - w[X, g[m], Y, g[n]]
                        if v != 0.0:
                            Qm = Qm + v * CD[m, n]
                ops.append(Op("Q", X, Y, F.sector_blocks(Qm, _delta([Y], [X]))))
    blk = Block(side=side, orbitals=tuple(orbitals), qn=F.qn, dim=F.dim, ops=ops)
    blk.fock = F
    return blk


def truncate(block, bases):
    """Project every operator onto per-sector orthonormal bases: O' = V_out^T O V_in.

    ``bases[i]`` is a (dim_i, m_i) matrix with orthonormal columns (m_i may be 0: sector dropped).
    """
    keep = [i for i, V in enumerate(bases) if V.shape[1] > 0]
    new_index = {old: new for new, old in enumerate(keep)}
    ops = []
    for op in block.ops:
        nb = {}
        for (so, si), m in op.blocks.items():
            if so in new_index and si in new_index:
                nb[(new_index[so], new_index[si])] = bases[so].T @ m @ bases[si]
        ops.append(Op(op.kind, op.i0, op.i1, nb))
    out = Block(side=block.side, orbitals=block.orbitals, qn=block.qn[keep],
                dim=np.array([bases[i].shape[1] for i in keep], dtype=np.int32), ops=ops)
    out.bases = [bases[i] for i in keep]
    out.parent = block
    return out


def random_bases(block, m_max, seed):
    """Seeded random per-sector orthonormal bases with total size <= m_max (largest sectors keep more)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = block.dim.astype(np.int64)
    total = int(dims.sum())
    keep = np.minimum(dims, np.floor(dims * min(1.0, m_max / total) + 0.5).astype(np.int64))
    keep = np.maximum(keep, np.minimum(dims, 1))
    bases = []
    for d, m in zip(dims, keep):
        q, _ = np.linalg.qr(rng.normal(size=(d, d)))
        bases.append(q[:, :m])
    return bases


def _block_state_bits(block, sec, pos):
    """Global determinant bits of basis state ``pos`` of sector ``sec`` of an untruncated block."""
    F = block.fock
    local = int(F.sector_states[sec][pos])
    return local << (2 * block.orbitals[0]) if len(block.orbitals) else local


_SITE_BITS = (0, 1, 2, 3)   # site basis (0, up, down, updown) -> bit pattern (alpha = bit 0, beta = bit 1)


def embed(layout, psi, left, right, s1, s2, dets):
    """Map a superblock vector (in ``layout``) into the determinant basis ``dets``.

    Blocks may be truncated (then their ``bases`` map block states to Fock determinants).
    """
    out = np.zeros(dets.size)
    Lroot = getattr(left, "parent", left)
    Rroot = getattr(right, "parent", right)
    for (a, b, c, d, off, ma, md) in layout.blocks:
        X = psi[off:off + ma * md].reshape(ma, md)
        if hasattr(left, "bases"):
            qa = tuple(left.qn[a])
            ra = Lroot.sector_index()[qa]
            X = left.bases[a] @ X
        else:
            ra = a
        if hasattr(right, "bases"):
            qd = tuple(right.qn[d])
            rd = Rroot.sector_index()[qd]
            X = X @ right.bases[d].T
        else:
            rd = d
        site = (_SITE_BITS[b] << (2 * s1)) | (_SITE_BITS[c] << (2 * s2))
        lbits = np.array([_block_state_bits(Lroot, ra, i) for i in range(X.shape[0])], dtype=np.int64)
        rbits = np.array([_block_state_bits(Rroot, rd, j) for j in range(X.shape[1])], dtype=np.int64)
        full = (lbits[:, None] | rbits[None, :]) | site
        out[np.searchsorted(dets, full.ravel())] += X.ravel()
    return out


def project(layout, vec, left, right, s1, s2, dets):
    """Adjoint of ``embed``: determinant vector -> superblock vector."""
    psi = np.zeros(layout.size)
    Lroot = getattr(left, "parent", left)
    Rroot = getattr(right, "parent", right)
    for (a, b, c, d, off, ma, md) in layout.blocks:
        ra = Lroot.sector_index()[tuple(left.qn[a])]
        rd = Rroot.sector_index()[tuple(right.qn[d])]
        nl = Lroot.dim[ra]
        nr = Rroot.dim[rd]
        site = (_SITE_BITS[b] << (2 * s1)) | (_SITE_BITS[c] << (2 * s2))
        lbits = np.array([_block_state_bits(Lroot, ra, i) for i in range(nl)], dtype=np.int64)
        rbits = np.array([_block_state_bits(Rroot, rd, j) for j in range(nr)], dtype=np.int64)
        full = (lbits[:, None] | rbits[None, :]) | site
        idx = np.searchsorted(dets, full.ravel())
        ok = (idx < dets.size)
        ok[ok] = dets[idx[ok]] == full.ravel()[ok]
        Xf = np.where(ok, vec[np.minimum(idx, dets.size - 1)], 0.0).reshape(nl, nr)
        if hasattr(left, "bases"):
            Xf = left.bases[a].T @ Xf
        if hasattr(right, "bases"):
            Xf = Xf @ right.bases[d]
        psi[off:off + ma * md] = Xf.ravel()
    return psi
