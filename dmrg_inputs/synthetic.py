"""Seeded synthetic block operators with the shapes of a middle-bond QC-DMRG problem.

The paper's block operators come from sweeps over molecular integrals that are not available here.
For throughput and parity work at large bond dimension the operator *values* are drawn at random
while their *structure* is the real one: the operator list of ``dmrg_inputs.blocks`` for the given
bond, each operator's sector change, and sector dimensions from a smooth model (below). The H.psi
of such blocks is a well-defined symmetric operator as long as the adjoint relations hold, so
``B_QP = B_PQ^T`` and ``Q_YX = Q_XY^T`` are not stored (only P <= Q / X <= Y) and H is symmetric.

Sector-dimension model (no arithmetic of the method, just a shape recipe): for a block of k orbitals
at filling (Na, Nb) of L orbitals, the weight of sector (na, nb) is
    exp(-[(na - Na k / L)^2 + (nb - Nb k / L)^2] / (2 sigma^2)),
capped by the number of determinants C(k, na) C(k, nb); dimensions are the weights scaled to a total
of M (largest remainders first), sectors rounding to zero are dropped.

Values: block Hamiltonian sector blocks diag(e) + eps * sym(noise) with e sorted uniform in
[0, h_spread); every other operator block N(0, g^2 / m_in). One PCG64 stream per block, drawn in
operator order, then sector order.
"""
from math import comb

import numpy as np

from .blocks import Block, Op


def sector_dims(k, n_alpha, n_beta, L, M, sigma):
    qn, w, cap = [], [], []
    ca, cb = n_alpha * k / L, n_beta * k / L
    for na in range(k + 1):
        for nb in range(k + 1):
            qn.append((na, nb))
            w.append(np.exp(-((na - ca) ** 2 + (nb - cb) ** 2) / (2.0 * sigma ** 2)))
            cap.append(min(comb(k, na) * comb(k, nb), M))   # a sector never exceeds M states
    w = np.array(w)
    cap = np.array(cap, dtype=np.int64)
    total = min(M, int(cap.sum()))
    dims = np.zeros(len(qn), dtype=np.int64)
    for _ in range(64):                       # water-filling under the caps
        free = dims < cap
        if not free.any():
            break
        left = total - dims.sum()
        if left <= 0:
            break
        share = w * free
        raw = left * share / share.sum()
        add = np.minimum(np.floor(raw).astype(np.int64), cap - dims)
        if add.sum() == 0:
            order = np.argsort(-(raw - np.floor(raw)) - 1e-9 * np.arange(len(qn)))
            for i in order[:left]:
                if dims[i] < cap[i]:
                    dims[i] += 1
            break
        dims += add
    keep = dims > 0
    return [q for q, kk in zip(qn, keep) if kk], dims[keep].astype(np.int32)


def _delta(kind, i0, i1):
    d = [0, 0]
    if kind == "C":
        d[i0 % 2] += 1
    elif kind == "A":
        d[i0 % 2] += 1; d[i1 % 2] += 1
    elif kind == "B":
        d[i0 % 2] += 1; d[i1 % 2] -= 1
    elif kind == "S":
        d[i0 % 2] += 1
    elif kind == "U":
        d[i0 % 2] -= 1
    elif kind == "P":
        d[i0 % 2] -= 1; d[i1 % 2] -= 1
    elif kind == "Q":
        d[i1 % 2] += 1; d[i0 % 2] -= 1
    return tuple(d)


def op_list(side, orbitals, L, site):
    """(kind, i0, i1) of the stored operators of a block at the bond (site, site+1)."""
    mine = [2 * p + s for p in orbitals for s in (0, 1)]
    ops = [("H", -1, -1)] + [("C", P, -1) for P in mine]
    if side == "left":
        ops += [("A", P, Q, ) for i, P in enumerate(mine) for Q in mine[i + 1:]]
        ops += [("B", P, Q) for i, P in enumerate(mine) for Q in mine[i:]]
        ops += [("S", W, -1) for W in range(2 * site, 2 * L)]
    else:
        out = list(range(0, 2 * (site + 2)))
        ops += [("U", P, -1) for P in out]
        ops += [("P", P, Q) for i, P in enumerate(out) for Q in out[i + 1:]]
        ops += [("Q", X, Y) for i, X in enumerate(out) for Y in out[i:]]
    return ops


def synthetic_block(side, L, n_alpha, n_beta, site, M, sigma, seed, g=0.2, h_spread=6.0, eps=0.05,
                    ops=None, dim_of=None):
    """Random-valued block with the operator structure of ``side`` at the bond (site, site+1).
    ``dim_of``: optional function (n_alpha, n_beta) -> sector dimension replacing the model's sizes."""
    orbitals = tuple(range(0, site)) if side == "left" else tuple(range(site + 2, L))
    k = len(orbitals)
    if k == 0:
        qn, dims = [(0, 0)], np.array([1], dtype=np.int32)
    else:
        qn, dims = sector_dims(k, n_alpha, n_beta, L, M, sigma)
    if dim_of is not None:
        dims = np.array([int(dim_of(*q)) for q in qn], dtype=np.int32)
    index = {q: i for i, q in enumerate(qn)}
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for kind, i0, i1 in (ops if ops is not None else op_list(side, orbitals, L, site)):
        d = _delta(kind, i0, i1)
        blocks = {}
        for si, (na, nb) in enumerate(qn):
            so = index.get((na + d[0], nb + d[1]))
            if so is None:
                continue
            mo, mi = int(dims[so]), int(dims[si])
            if kind == "H":
                e = np.sort(rng.uniform(0.0, h_spread, size=mi))
                n = rng.normal(0.0, 1.0, size=(mi, mi))
                blocks[(so, si)] = np.diag(e) + eps * (n + n.T) / np.sqrt(2.0 * mi)
            else:
                m = rng.normal(0.0, g / np.sqrt(mi), size=(mo, mi))
                if kind in ("B", "Q") and i0 == i1:
                    m = 0.5 * (m + m.T)
                blocks[(so, si)] = m
        out.append(Op(kind, i0, i1, blocks))
    return Block(side=side, orbitals=orbitals, qn=np.array(qn, dtype=np.int32).reshape(-1, 2), dim=dims, ops=out)


def share_ops(side, L, site, n_pairs):
    """Operator list of one device's share of the operator combinations: the block Hamiltonian and
    the first ``n_pairs`` (X <= Y) normal/complementary pairs B_XY / Q_XY and (P < Q) A_PQ / P_PQ over
    the left-block spin-orbitals, in index order (the largest families of the sum)."""
    left = [2 * p + s for p in range(site) for s in (0, 1)]
    bq = [(X, Y) for i, X in enumerate(left) for Y in left[i:]][:n_pairs]
    ap = [(P, Q) for i, P in enumerate(left) for Q in left[i + 1:]][:n_pairs]
    if side == "left":
        return [("H", -1, -1)] + [("B", X, Y) for X, Y in bq] + [("A", P, Q) for P, Q in ap]
    return [("H", -1, -1)] + [("Q", X, Y) for X, Y in bq] + [("P", P, Q) for P, Q in ap]


def synthetic_problem(L, n_alpha, n_beta, M, sigma, seed, site=None, **kw):
    """Integrals (``random_integrals``) plus synthetic left/right blocks at the middle bond."""
    from .integrals import random_integrals
    if site is None:
        site = L // 2 - 1
    h, eri = random_integrals(L, seed)
    left = synthetic_block("left", L, n_alpha, n_beta, site, M, sigma, seed + 1000, **kw)
    right = synthetic_block("right", L, n_alpha, n_beta, site, M, sigma, seed + 2000, **kw)
    return h, eri, left, right, site
