"""Reduced density matrices, their truncation and the renormalization of Eq. renorm_mat (Section 2.1)
-- TEST INFRASTRUCTURE ONLY (plain FP64 NumPy; see the package header for who may import it).

What is computed, in the paper's order and notation:

1. The two-site coefficients psi_{l s_l s_r r} (Eq. wf) are read as one matrix psi_{(l s_l), (s_r r)}:
   rows are the enlarged left block (left-block state l with left-site state s_l = b), columns the
   enlarged right block (right-site state s_r = c with right-block state r).
2. rho^L = psi psi^T and rho^R = psi^T psi (real coefficients, so the adjoint is the transpose).
3. O^L (Eq. renorm) holds the M eigenvectors of rho^L with the largest eigenvalues, as columns; the
   truncated basis is |l_p> = sum_{l s} O_{(l s), l_p} |l>|s>.
4. An enlarged-block operator A becomes A' = O^T A O (Eq. renorm_mat).
5. The truncated state O^T psi is carried to the next bond's basis (``next_bond_psi``).

U(1) x U(1) symmetry makes every step block diagonal. The enlarged-left quantum number
q = qn(a) + qn(b) fixes the enlarged-right one, (N_alpha, N_beta) - q, so psi splits into one dense
matrix Psi_q per q. Enlarged-left basis of sector q: the pairs (a, b) with qn(a) + qn(b) = q in (a, b)
lexicographic order, each contributing its m_a states l consecutively. Enlarged-right basis of sector
q': the pairs (c, d) in (c, d) lexicographic order, each contributing m_d states r. Pairs with no psi
block still belong to the basis (their rows or columns of psi are zero), so the enlarged left block
has the full dimension 4 M of Eq. renorm. Enlarged sectors are listed in ascending (n_alpha, n_beta).

Readings (where the paper is silent):
* The M largest eigenvalues are chosen over all sectors together (one global cut, so the kept
  dimension is M overall, as for the 4M x M matrix of Eq. renorm). Equal eigenvalues at the cut are
  taken in (sector order, ascending eigenvalue index) order.
* Eigenvectors are defined up to sign; kept vectors are stored in descending eigenvalue order with
  their largest-magnitude component positive. Only the projector O O^T is unique (when the cut falls
  between distinct eigenvalues), and that is what comparisons of two implementations should use.
* Sectors that keep no state are dropped from the truncated block.
"""
import numpy as np

from oracle.layout import SITE_QN


def _qadd(q, s):
    return (int(q[0]) + SITE_QN[s][0], int(q[1]) + SITE_QN[s][1])


def enlarged_left_basis(left):
    """q -> list of (a, b, start, m_a) and q -> dimension, for the enlarged left block (block, site)."""
    parts, dims = {}, {}
    for a in range(left.n_sec):
        m = int(left.dim[a])
        if m == 0:
            continue
        for b in range(4):
            q = _qadd(left.qn[a], b)
            parts.setdefault(q, [])
            parts[q].append((a, b, dims.get(q, 0), m))
            dims[q] = dims.get(q, 0) + m
    order = sorted(parts)
    return {q: parts[q] for q in order}, {q: dims[q] for q in order}


def enlarged_right_basis(right):
    """q -> list of (c, d, start, m_d) and q -> dimension, for the enlarged right block (site, block)."""
    parts, dims = {}, {}
    for c in range(4):
        for d in range(right.n_sec):
            m = int(right.dim[d])
            if m == 0:
                continue
            q = _qadd(right.qn[d], c)
            parts.setdefault(q, [])
            parts[q].append((c, d, dims.get(q, 0), m))
            dims[q] = dims.get(q, 0) + m
    # (c, d) lexicographic within each sector: the loop above already visits c outermost
    order = sorted(parts)
    return {q: parts[q] for q in order}, {q: dims[q] for q in order}


def psi_matrices(layout, left, right, n_alpha, n_beta, psi):
    """q -> Psi_q, the matrix psi_{(l s_l), (s_r r)} restricted to enlarged-left sector q (step 1)."""
    lparts, ldims = enlarged_left_basis(left)
    rparts, rdims = enlarged_right_basis(right)
    lstart = {(a, b): st for q in lparts for (a, b, st, m) in lparts[q]}
    rstart = {(c, d): st for q in rparts for (c, d, st, m) in rparts[q]}
    out = {}
    for q in ldims:
        qr = (n_alpha - q[0], n_beta - q[1])
        out[q] = np.zeros((ldims[q], rdims.get(qr, 0)))
    for i, (a, b, c, d, off, ma, md) in enumerate(layout.blocks):
        q = _qadd(left.qn[a], b)
        r0, c0 = lstart[(a, b)], rstart[(c, d)]
        out[q][r0:r0 + ma, c0:c0 + md] = layout.view(psi, i)
    return out


def rdm_left(psi_q):
    """rho^L_q = Psi_q Psi_q^T for every enlarged-left sector q (step 2)."""
    return {q: P @ P.T for q, P in psi_q.items()}


def rdm_right(psi_q, n_alpha, n_beta):
    """rho^R_{q'} = Psi^T Psi for every enlarged-right sector q' = N - q that psi reaches (step 2)."""
    return {(n_alpha - q[0], n_beta - q[1]): P.T @ P for q, P in psi_q.items() if P.shape[1] > 0}


def select(rho, M):
    """Keep the M eigenvectors of the block-diagonal rho with the largest eigenvalues (step 3).

    Returns (O, kept, discarded): O maps each sector that keeps states to its (dim_q, k_q) matrix of
    orthonormal columns (descending eigenvalues, largest-magnitude component positive); kept lists
    (eigenvalue, q) in selection order; discarded = trace(rho) - sum of kept eigenvalues.
    """
    eig = {}
    cand = []
    for si, q in enumerate(rho):
        w, V = np.linalg.eigh(rho[q])          # ascending
        eig[q] = (w, V)
        for j in range(w.size):
            cand.append((-w[j], si, j, q))
    cand.sort(key=lambda t: (t[0], t[1], t[2]))
    chosen = cand[:max(0, int(M))]
    cols = {}
    for _, _, j, q in chosen:
        cols.setdefault(q, []).append(j)
    O = {}
    for q in rho:                              # sector order
        if q not in cols:
            continue
        w, V = eig[q]
        js = sorted(cols[q], key=lambda j: (-w[j], j))
        B = V[:, js].copy()
        for k in range(B.shape[1]):
            if B[np.argmax(np.abs(B[:, k])), k] < 0:
                B[:, k] = -B[:, k]
        O[q] = B
    kept = [(-t[0], t[3]) for t in chosen]
    total = sum(float(np.trace(r)) for r in rho.values())
    return O, kept, total - sum(k for k, _ in kept)


def transform_psi(psi_q, O):
    """psi in the truncated left basis: Psi'_q = O_q^T Psi_q for the sectors that keep states."""
    return {q: O[q].T @ psi_q[q] for q in O}


def renormalize(A, O_out, O_in):
    """Eq. renorm_mat per sector block: A'_{(q_out, q_in)} = O_{q_out}^T A_{(q_out, q_in)} O_{q_in}.

    A maps (q_out, q_in) to a dense matrix in the enlarged (4M-dimensional) basis; blocks whose
    sectors keep no state are dropped.
    """
    return {(qo, qi): O_out[qo].T @ m @ O_in[qi] for (qo, qi), m in A.items() if qo in O_out and qi in O_in}


def site_number_left(left, spin):
    """Number operator of the left site's spin-orbital (spin 0: alpha, 1: beta) in the enlarged-left
    basis: diagonal, n = occupation of that spin in site state b, repeated over the m_a states."""
    parts, dims = enlarged_left_basis(left)
    A = {}
    for q in parts:
        d = np.zeros(dims[q])
        for a, b, st, m in parts[q]:
            d[st:st + m] = SITE_QN[b][spin]
        A[(q, q)] = np.diag(d)
    return A


def block_number_left(left, spin):
    """Electron number of the left block for one spin in the enlarged-left basis: diagonal, qn(a)."""
    parts, dims = enlarged_left_basis(left)
    A = {}
    for q in parts:
        d = np.zeros(dims[q])
        for a, b, st, m in parts[q]:
            d[st:st + m] = left.qn[a][spin]
        A[(q, q)] = np.diag(d)
    return A


def next_bond_psi(layout_next, psi_t, right_old, n_alpha, n_beta, split_right):
    """psi of the truncated state in the next bond's basis (the left block grown and renormalized,
    the old right site now the left site, the old right block split into a site and a smaller block).

    psi_t: q -> O_q^T Psi_q (rows: kept states of sector q in O's column order; columns: the old
    enlarged-right basis of sector N - q). The new left block's sectors are the q of psi_t in
    ascending order. split_right(d, r) -> (s, d_new, r_new, coef) writes old right-block state r of
    sector d as coef |s>|r_new> (site state s of the new right site, state r_new of sector d_new).
    """
    rparts, _ = enlarged_right_basis(right_old)
    sidx = {q: i for i, q in enumerate(sorted(psi_t))}
    out = np.zeros(layout_next.size)
    for q, T in psi_t.items():
        qr = (n_alpha - q[0], n_beta - q[1])
        for c, d, st, m in rparts.get(qr, []):
            for r in range(m):
                s, d_new, r_new, coef = split_right(d, r)
                i = layout_next.index[(sidx[q], c, s, d_new)]
                X = layout_next.view(out, i)
                X[:, r_new] += coef * T[:, st + r]
    return out
