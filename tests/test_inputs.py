"""CPU checks of the seeded input generators that both the oracle and the library read.

* The benchmark's H.psi workload (L = 24, N = (12, 12), M = 1024 at the middle bond, sigma = 1.5,
  seed 1) has the shape the benchmark reports: 1024 states and 60 sectors per block, 844 psi blocks,
  586,140 coefficients, bond (11, 12).
* The same seed gives the same integrals and operators; another seed does not.
* Sector dimensions follow the recipe: at most M in total, each within its determinant count, and
  the largest sector at the filling point N k / L of a k-orbital block.
* Every synthetic operator maps each sector to the one shifted by the operator's particle-number
  change (the structure the oracle's and the library's term lists rely on).
"""
from math import comb

import numpy as np

from dmrg_inputs.synthetic import sector_dims, synthetic_problem
from oracle.layout import Layout


def test_benchmark_workload_shape():
    h, eri, left, right, site = synthetic_problem(24, 12, 12, 1024, 1.5, 1)
    assert site == 11 and h.shape == (24, 24) and eri.shape == (24,) * 4
    assert int(left.dim.sum()) == int(right.dim.sum()) == 1024
    assert left.n_sec == right.n_sec == 60
    lay = Layout(left, right, 12, 12)
    assert len(lay.blocks) == 844 and lay.size == 586140


def test_generators_are_seeded():
    a = synthetic_problem(10, 5, 5, 60, 1.2, 4)
    b = synthetic_problem(10, 5, 5, 60, 1.2, 4)
    c = synthetic_problem(10, 5, 5, 60, 1.2, 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for x, y in zip(a[2].ops + a[3].ops, b[2].ops + b[3].ops):
        assert x.key == y.key and x.blocks.keys() == y.blocks.keys()
        assert all(np.array_equal(x.blocks[k], y.blocks[k]) for k in x.blocks)
    assert not np.array_equal(a[0], c[0])


def test_sector_dimension_recipe():
    for k, na, nb, L, M, sigma in ((11, 12, 12, 24, 1024, 1.5), (5, 5, 4, 10, 40, 1.0), (37, 57, 56, 76, 6000, 2.5)):
        qn, dims = sector_dims(k, na, nb, L, M, sigma)
        qn, dims = np.asarray(qn), np.asarray(dims)
        assert dims.sum() <= M and np.all(dims >= 0)
        for (a, b), d in zip(qn, dims):
            assert d <= comb(k, int(a)) * comb(k, int(b))
        top = qn[int(np.argmax(dims))]
        assert abs(top[0] - na * k / L) <= 1.0 and abs(top[1] - nb * k / L) <= 1.0


def _shift(kind, i0, i1):
    def d(P):
        return np.array([1, 0]) if P % 2 == 0 else np.array([0, 1])
    if kind == "H":
        return np.zeros(2, dtype=int)
    if kind == "C":
        return d(i0)
    if kind == "A":
        return d(i0) + d(i1)
    if kind == "B":
        return d(i0) - d(i1)
    if kind == "S":                               # c+_P c+_Q c_R with spins (W, Q, Q): one W-spin electron in
        return d(i0)
    if kind == "U":                               # c+_Q c_Z c_W with spins (Q, Q, P): one P-spin electron out
        return -d(i0)
    if kind == "P":                               # c_Z c_W with spins (Q, P)
        return -d(i0) - d(i1)
    if kind == "Q":                               # c+_Z c_W: zero when X, Y share a spin, else exchange (Y, X)
        return d(i1) - d(i0)
    raise KeyError(kind)


def test_operators_shift_sectors_by_their_particle_number_change():
    h, eri, left, right, site = synthetic_problem(10, 5, 4, 80, 1.2, 2)
    for blk in (left, right):
        for op in blk.ops:
            for (so, si) in op.blocks:
                diff = blk.qn[so].astype(int) - blk.qn[si].astype(int)
                assert np.array_equal(diff, _shift(op.kind, op.i0, op.i1)), (op.key, so, si)
