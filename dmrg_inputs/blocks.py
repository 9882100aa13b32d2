"""Container for the renormalized operators of one DMRG block (no arithmetic).

A block holds symmetry sectors labelled by ``(n_alpha, n_beta)`` (U(1)xU(1), Section 2.1) with
their dimensions, and a list of operators. Each operator stores only its non-zero sector blocks as
dense row-major matrices ``<l'|O|l>`` of shape ``(dim[sec_out], dim[sec_in])`` -- the operator
class of Section 2.2 (a sector table plus a vector of dense sector tensors).

Operator kinds (spin-orbital ids are global, ``2*p + sigma``, sigma 0 = alpha, 1 = beta):

left ("normal") block X -- orbitals to the left of the two sites:
  ``H``            block Hamiltonian (all integrals inside X)
  ``C  (P)``       creation operator c+_P, P in X
  ``A  (P, Q)``    c+_P c+_Q, P < Q in X
  ``B  (P, Q)``    c+_P c_Q, all ordered pairs P, Q in X
  ``S  (W)``       sum_{P,Q,R in X} w_PQRW c+_P c+_Q c_R for every W right of X (three-index part only)

right ("complementary") block Y -- orbitals to the right of the two sites; outside indices are all
spin-orbitals to the left of Y (left block and both sites):
  ``H``            block Hamiltonian
  ``C  (Z)``       c+_Z, Z in Y
  ``U  (P)``       sum_{Q,Z,W in Y} w_PQZW c+_Q c_Z c_W
  ``P  (P, Q)``    sum_{Z,W in Y} w_PQZW c_Z c_W, P < Q outside
  ``Q  (X, Y')``   sum_{Z,W in Y} (w_XZWY' - w_XZY'W) c+_Z c_W, all ordered outside pairs

with ``w_PQRS = (ps|qr) delta(sigma_P, sigma_S) delta(sigma_Q, sigma_R)`` so that
``H = sum t_PQ c+_P c_Q + 1/2 sum w_PQRS c+_P c+_Q c_R c_S`` (the reading of Eq. H2q with
``v_pqrs = (ps|qr)/2``).
"""
from dataclasses import dataclass, field

import numpy as np

OP_KINDS = ("H", "C", "A", "B", "S", "U", "P", "Q")


@dataclass
class Op:
    kind: str
    i0: int = -1
    i1: int = -1
    blocks: dict = field(default_factory=dict)  # {(sec_out, sec_in): ndarray}

    @property
    def key(self):
        return (self.kind, self.i0, self.i1)


@dataclass
class Block:
    side: str                 # "left" (normal set) or "right" (complementary set)
    orbitals: tuple           # spatial orbitals of the block, ascending and contiguous
    qn: np.ndarray            # (n_sec, 2) int32: (n_alpha, n_beta)
    dim: np.ndarray           # (n_sec,) int32
    ops: list                 # list[Op]

    def __post_init__(self):
        self.qn = np.asarray(self.qn, dtype=np.int32).reshape(-1, 2)
        self.dim = np.asarray(self.dim, dtype=np.int32).reshape(-1)
        self._index = None

    @property
    def n_sec(self):
        return int(self.dim.size)

    def sector_index(self):
        """Map (n_alpha, n_beta) -> sector index."""
        return {(int(a), int(b)): i for i, (a, b) in enumerate(self.qn)}

    def op_map(self):
        if self._index is None or len(self._index) != len(self.ops):
            self._index = {op.key: op for op in self.ops}
        return self._index

    def get(self, kind, i0=-1, i1=-1):
        return self.op_map().get((kind, i0, i1))

    def nbytes(self):
        return sum(b.nbytes for op in self.ops for b in op.blocks.values())

    def flatten(self):
        """Concatenate all sector blocks (in op order, block-key order) into one float64 array.

        Returns ``(data, table)`` where ``table`` is a list per op of ``(sec_out, sec_in, offset)``.
        """
        chunks, table, off = [], [], 0
        for op in self.ops:
            rows = []
            for (so, si), m in sorted(op.blocks.items()):
                m = np.ascontiguousarray(m, dtype=np.float64)
                assert m.shape == (self.dim[so], self.dim[si]), (op.key, so, si, m.shape)
                rows.append((so, si, off))
                chunks.append(m.ravel())
                off += m.size
            table.append(rows)
        data = np.concatenate(chunks) if chunks else np.zeros(0)
        return data, table
