"""Sector-decomposed two-site wave function (Eq. wf_sec and the constraints below it, Section 2.1).

psi is a list of dense blocks psi^{abcd}_{lr} (l in left sector a, r in right sector d, site states
b, c); a block exists iff n_alpha(a)+n_alpha(b)+n_alpha(c)+n_alpha(d) = N_alpha and likewise for
beta. Canonical order: (a, b, c) lexicographic, a over the left block's sector list, b and c over the
site basis (0, up, down, updown); d is then fixed. Each block is row-major (m_a x m_d), contiguous.
"""
import numpy as np

SITE_QN = ((0, 0), (1, 0), (0, 1), (1, 1))   # (n_alpha, n_beta) of site states 0, up, down, updown


class Layout:
    def __init__(self, left, right, n_alpha, n_beta):
        ridx = right.sector_index()
        self.blocks = []          # (a, b, c, d, offset, m_a, m_d)
        self.index = {}           # (a, b, c, d) -> position in self.blocks
        off = 0
        for a in range(left.n_sec):
            na, nb = (int(v) for v in left.qn[a])
            for b in range(4):
                for c in range(4):
                    qd = (n_alpha - na - SITE_QN[b][0] - SITE_QN[c][0],
                          n_beta - nb - SITE_QN[b][1] - SITE_QN[c][1])
                    d = ridx.get(qd)
                    if d is None:
                        continue
                    ma, md = int(left.dim[a]), int(right.dim[d])
                    if ma == 0 or md == 0:
                        continue
                    self.index[(a, b, c, d)] = len(self.blocks)
                    self.blocks.append((a, b, c, d, off, ma, md))
                    off += ma * md
        self.size = off

    def view(self, psi, i):
        a, b, c, d, off, ma, md = self.blocks[i]
        return psi[off:off + ma * md].reshape(ma, md)
