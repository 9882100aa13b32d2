"""CPU tests of libdmrg: exported symbols, host-side logic (term generator + task list) and errors.

The host-only build (device = -1) runs the psi layout, the operator-combination generator and the
task-list builder without touching a GPU; the exported task list is executed here by a few lines of
numpy and compared with the oracle. This checks the library's term derivation (an independent,
hand-derived family list) against the oracle's mechanical expansion on the CPU.
"""
import re
import os

import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle.hpsi import OracleHop
from helpers import exact_problem, rel_err, synth

lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, DmrgError = lib_mod.Hop, lib_mod.DmrgError

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "dmrg.h")


def test_library_exports_every_declared_symbol():
    decl = open(HEADER).read()
    names = set(re.findall(r"\b(dmrg_[a-z_]+)\s*\(", decl))
    names -= {"dmrg_status"}
    assert {"dmrg_build_blocks", "dmrg_hpsi", "dmrg_davidson", "dmrg_hop_layout"} <= names
    for n in sorted(names):
        assert hasattr(lib_mod.lib, n), n
    assert "gfx950" in lib_mod.version()


def _exec_tasks(hop, left, right, x):
    quads, f, ti, tc = hop.export_tasks()
    mats = {}
    for (m, side, op, tr), c in zip(ti, tc):
        mats.setdefault(int(m), []).append((side, op, tr, c))

    def block_of(m, si):
        out = None
        for side, op, tr, c in mats[m]:
            B = left if side == 0 else right
            for (so_, si_), M in B.ops[op].blocks.items():
                if (not tr and si_ == si) or (tr and so_ == si):
                    v = c * (M.T if tr else M)
                    out = v if out is None else out + v
        return out

    y = np.zeros_like(x)
    for (i, j, lm, rm), ff in zip(quads, f):
        a, b, c, d = hop.abcd[i]
        ma, md = hop.dims[i]
        mj, nj = hop.dims[j]
        X = x[hop.offsets[i]:hop.offsets[i] + ma * md].reshape(ma, md)
        T = X if lm < 0 else block_of(lm, a) @ X
        if rm >= 0:
            T = T @ block_of(rm, d).T
        y[hop.offsets[j]:hop.offsets[j] + mj * nj] += ff * T.ravel()
    return y


@pytest.mark.parametrize("case", ["exact8", "trunc10_odd", "synth12", "edge4_left_empty", "edge6_right_empty",
                                  "edge2_both_empty", "spin_polarized8", "off_center9", "near_full6", "one_electron6"])
def test_host_task_list_matches_oracle(case):
    if case == "exact8":
        h, eri, left, right, na, nb, site = exact_problem(8, 0)
    elif case == "spin_polarized8":        # N_alpha - N_beta = 4: many (a, b, c, d) combinations vanish
        h, eri, left, right, na, nb, site = exact_problem(8, 4, n_alpha=6, n_beta=2)
    elif case == "off_center9":            # bond (2, 3) of L = 9: 2-orbital left block, 5-orbital right block
        h, eri, left, right, na, nb, site = exact_problem(9, 5, n_alpha=5, n_beta=3, site=2)
    elif case == "near_full6":             # two holes: the particle-hole mirror of a 2-electron problem
        h, eri, left, right, na, nb, site = exact_problem(6, 6, n_alpha=5, n_beta=5)
    elif case == "one_electron6":          # one electron: no two-body term has a nonzero matrix element
        h, eri, left, right, na, nb, site = exact_problem(6, 7, n_alpha=1, n_beta=0)
    elif case == "edge4_left_empty":
        h, eri, left, right, na, nb, site = exact_problem(4, 3, site=0)
    elif case == "edge6_right_empty":
        h, eri, left, right, na, nb, site = exact_problem(6, 3, site=4)
    elif case == "edge2_both_empty":
        h, eri, left, right, na, nb, site = exact_problem(2, 3, n_alpha=1, n_beta=1, site=0)
    elif case == "trunc10_odd":
        h, eri, left, right, na, nb, site = exact_problem(10, 1, n_alpha=5, n_beta=4, trunc=40)
    else:
        h, eri, left, right, na, nb, site = synth(12, 60, 1.2, 5)
    hop = Hop(h, eri, left, right, na, nb, site, device=-1)
    oh = OracleHop(h, eri, left, right, na, nb, site)
    assert [tuple(b[:4]) for b in oh.layout.blocks] == [tuple(r) for r in hop.abcd]
    x = random_vector(hop.n_coeff, 3)
    assert rel_err(_exec_tasks(hop, left, right, x), oh.apply(x)) < 1e-12
    st = hop.stats()
    assert st["n_alpha"] > 0 and st["n_tasks"] > 0
    # with both blocks empty every task is a site-only scaling (identity on both sides): no GEMM flops
    assert (st["flops"] == 0) if case == "edge2_both_empty" else (st["flops"] > 0)


def test_host_only_handle_refuses_compute():
    h, eri, left, right, na, nb, site = exact_problem(6, 0)
    hop = Hop(h, eri, left, right, na, nb, site, device=-1)

    class Fake:
        def dim(self):
            return 1

        def numel(self):
            return hop.n_coeff

        dtype = None

        def is_contiguous(self):
            return True

        def data_ptr(self):
            return 16

    with pytest.raises(DmrgError) as e:
        hop.hpsi(Fake(), Fake())
    assert e.value.status == -7


def test_missing_operator_is_an_argument_error():
    h, eri, left, right, na, nb, site = exact_problem(6, 0)
    right.ops = [op for op in right.ops if not (op.kind == "P" and op.i0 == 0 and op.i1 == 1)]
    with pytest.raises(DmrgError) as e:
        Hop(h, eri, left, right, na, nb, site, device=-1)
    assert e.value.status == -1 and "P(0,1)" in str(e.value)


def test_bad_bond_and_nan_inputs():
    h, eri, left, right, na, nb, site = exact_problem(6, 0)
    with pytest.raises(DmrgError) as e:
        Hop(h, eri, left, right, na, nb, 5, device=-1)
    assert e.value.status == -1
    bad = h.copy()
    bad[0, 0] = np.nan
    with pytest.raises(DmrgError) as e:
        Hop(bad, eri, left, right, na, nb, site, device=-1)
    assert e.value.status == -5


def test_electron_number_out_of_range_and_empty_sector():
    h, eri, left, right, na, nb, site = exact_problem(6, 0)
    with pytest.raises(DmrgError) as e:
        Hop(h, eri, left, right, 7, 3, site, device=-1)      # 7 alpha electrons in 6 orbitals
    assert e.value.status == -1
    hop = Hop(h, eri, left, right, 6, 6, site, device=-1)   # completely filled: one determinant
    assert hop.n_coeff == 1
    left.qn = left.qn[:1]                                    # keep only the empty left sector
    left.dim = left.dim[:1]
    left.ops = [type(op)(op.kind, op.i0, op.i1, {k: v for k, v in op.blocks.items() if k == (0, 0)})
                for op in left.ops]
    with pytest.raises(DmrgError) as e:
        Hop(h, eri, left, right, 6, 6, site, device=-1)
    assert e.value.status == -2


@pytest.mark.parametrize("case", ["exact8", "synth12", "edge4_left_empty"])
def test_flop_count_follows_its_definition(case):
    """The algorithmic flop count behind every TFLOP/s figure: per exported task, 2 MACs of the cheaper
    association of A.X.B^T (one product when a side is the identity, none when both are), summed."""
    if case == "exact8":
        p = exact_problem(8, 0)
    elif case == "synth12":
        p = synth(12, 60, 1.2, 5)
    else:
        p = exact_problem(4, 3, site=0)
    hop = Hop(*p, device=-1)
    quads, f, ti, tc = hop.export_tasks()
    ma, md = hop.dims[:, 0].astype(np.float64), hop.dims[:, 1].astype(np.float64)
    i, j, lm, rm = quads[:, 0], quads[:, 1], quads[:, 2], quads[:, 3]
    a, d, mj, nj = ma[i], md[i], ma[j], md[j]
    both = 2.0 * np.minimum(mj * a * d + mj * d * nj, a * d * nj + mj * a * nj)
    fl = np.where((lm < 0) & (rm < 0), 0.0,
                  np.where(lm < 0, 2.0 * a * d * nj, np.where(rm < 0, 2.0 * mj * a * d, both)))
    assert hop.stats()["n_tasks"] == len(quads)
    assert abs(hop.stats()["flops"] - fl.sum()) <= 1e-12 * fl.sum()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU only: --gpus 2 (or a multi-rank launch) exits with status 2 and a
    message, before any GPU work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py")] + args, capture_output=True, text=True,
                           env={**os.environ, **env}, timeout=120)
        assert r.returncode == 2 and "one GPU only" in r.stderr


@pytest.mark.parametrize("case", ["exact8", "trunc10_odd", "synth12", "edge4_left_empty"])
def test_rdm_left_layout_matches_oracle(case):
    """dmrg_rdm_left_layout / dmrg_rdm_right_layout list the enlarged-left / -right sectors (ascending q)
    with the oracle's dimensions."""
    from oracle import renorm
    if case == "exact8":
        p = exact_problem(8, 0)
    elif case == "trunc10_odd":
        p = exact_problem(10, 1, n_alpha=5, n_beta=4, trunc=40)
    elif case == "edge4_left_empty":
        p = exact_problem(4, 3, site=0)
    else:
        p = synth(12, 60, 1.2, 5)
    hop = Hop(*p, device=-1)
    for layout, basis, blk in ((hop.rdm_left_layout, renorm.enlarged_left_basis, p[2]),
                               (hop.rdm_right_layout, renorm.enlarged_right_basis, p[3])):
        qn, dims, off = layout()
        _, odims = basis(blk)
        assert [tuple(int(v) for v in q) for q in qn] == list(odims)
        assert dims.tolist() == list(odims.values())
        assert off[0] == 0 and np.array_equal(np.diff(off), dims.astype(np.int64) ** 2)

    class Fake:
        def numel(self):
            return hop.n_coeff

        def is_contiguous(self):
            return True

        def data_ptr(self):
            return 16

    for fn in (hop.rdm_left, hop.rdm_right):
        with pytest.raises(DmrgError) as e:
            fn(Fake(), Fake())
        assert e.value.status == -7


@pytest.fixture(scope="module")
def rho_case():
    """Oracle rho^L of a random psi over synthetic blocks (L = 12, M = 60), in the sector order of
    dmrg_rdm_left_layout."""
    from oracle import renorm
    from oracle.layout import Layout
    h, eri, left, right, na, nb, site = synth(12, 60, 1.2, 5)
    x = random_vector(Layout(left, right, na, nb).size, 13)
    x /= np.linalg.norm(x)
    rho = renorm.rdm_left(renorm.psi_matrices(Layout(left, right, na, nb), left, right, na, nb, x))
    dims = np.array([r.shape[0] for r in rho.values()], dtype=np.int32)
    flat = np.concatenate([r.ravel() for r in rho.values()])
    return rho, dims, flat


def test_truncate_eigenpairs_match_dense_eigh(rho_case):
    rho, dims, flat = rho_case
    kept, evals, vecs, disc = lib_mod.truncate(flat, dims, 10 ** 6)
    assert np.array_equal(kept, dims) and abs(disc) < 1e-13
    scale = max(float(np.abs(r).max()) for r in rho.values())
    for (q, r), w, V in zip(rho.items(), evals, vecs):
        assert np.all(np.diff(w) <= 0)
        assert np.abs(w - np.sort(np.linalg.eigvalsh(r))[::-1]).max(initial=0) < 1e-13 * scale
        assert np.abs(V.T @ V - np.eye(len(w))).max(initial=0) < 1e-12
        assert np.abs(r @ V - V * w).max(initial=0) < 1e-12 * scale
        for k in range(len(w)):
            assert V[np.argmax(np.abs(V[:, k])), k] > 0


@pytest.mark.parametrize("M", [0, 1, 5, 17, 40, 60])
def test_truncate_matches_oracle_cut(rho_case, M):
    """Kept counts, discarded weight and the kept projector of each sector equal the oracle's global
    M-cut (M up to the rank, where the cut falls in a gap)."""
    from oracle import renorm
    rho, dims, flat = rho_case
    kept, evals, vecs, disc = lib_mod.truncate(flat, dims, M)
    O, okept, odisc = renorm.select(rho, M)
    assert int(kept.sum()) == M and abs(disc - odisc) < 1e-13
    for i, q in enumerate(rho):
        k = int(kept[i])
        assert k == (O[q].shape[1] if q in O else 0), q
        if k:
            P = vecs[i][:, :k] @ vecs[i][:, :k].T
            assert np.abs(P - O[q] @ O[q].T).max() < 1e-9


def test_truncate_rejects_bad_arguments(rho_case):
    rho, dims, flat = rho_case
    with pytest.raises(DmrgError) as e:
        lib_mod.truncate(flat, dims, -1)
    assert e.value.status == -1
    bad = flat.copy()
    bad[0] = np.nan
    with pytest.raises(DmrgError) as e:
        lib_mod.truncate(bad, dims, 3)
    assert e.value.status == -5


def test_truncate_at_benchmark_size():
    """L = 24, M = 1024 (77 sectors, up to 284 states): the same kept counts and discarded weight as
    the oracle's cut to M = 1024."""
    from oracle import renorm
    from oracle.layout import Layout
    from dmrg_inputs.synthetic import synthetic_problem
    h, eri, left, right, site = synthetic_problem(24, 12, 12, 1024, 1.5, 1)
    lay = Layout(left, right, 12, 12)
    x = random_vector(lay.size, 1)
    x /= np.linalg.norm(x)
    rho = renorm.rdm_left(renorm.psi_matrices(lay, left, right, 12, 12, x))
    dims = np.array([r.shape[0] for r in rho.values()], dtype=np.int32)
    kept, evals, vecs, disc = lib_mod.truncate(np.concatenate([r.ravel() for r in rho.values()]), dims, 1024)
    O, _, odisc = renorm.select(rho, 1024)
    assert len(dims) == 77 and int(dims.max()) == 284
    assert abs(disc - odisc) < 1e-12
    assert [int(k) for k in kept] == [O[q].shape[1] if q in O else 0 for q in rho]


def test_truncate_large_rank_deficient_sector_is_fast():
    """One graded, rank-deficient 1000-state sector (rank 300): the eigenpairs satisfy the
    eigen-equation and orthonormality, the spectrum equals numpy's, and the solve stays within a time
    bound (a cyclic Jacobi took minutes on this shape)."""
    import time
    rng = np.random.default_rng(21)
    n, rank = 1000, 300
    X = rng.normal(size=(n, rank)) * np.exp(-0.05 * np.arange(rank))
    r = X @ X.T
    t0 = time.perf_counter()
    kept, evals, vecs, disc = lib_mod.truncate(r.ravel(), [n], 150)
    dt = time.perf_counter() - t0
    w, V = evals[0], vecs[0]
    scale = float(np.abs(r).max())
    assert dt < 20.0, dt
    assert int(kept[0]) == 150
    assert np.abs(w - np.sort(np.linalg.eigvalsh(r))[::-1]).max() < 1e-12 * scale
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-12
    assert np.abs(r @ V - V * w).max() < 1e-12 * scale
    assert abs(disc - float(w[150:].sum())) < 1e-10 * scale


def test_renormalize_blocks_checks_arguments_before_any_device_work():
    class Fake:
        def __init__(self, n):
            self.n = n

        def is_contiguous(self):
            return True

        def data_ptr(self):
            return 16

        def numel(self):
            return self.n

    dims, kept, o_off = [3, 4], [2, 4], [0, 6]
    ok = dict(dims=dims, kept=kept, o_off=o_off, O=Fake(22), sec_out=[0, 1], sec_in=[1, 0], a_off=[0, 12],
              A=Fake(24), out_off=[0, 8], out=Fake(16))
    for noalloc in (False, True):      # the allocation-free variant checks the same way
        for change, status in (({"sec_out": [0, 2]}, -1), ({"kept": [4, 4]}, -1), ({"A": Fake(23)}, -2),
                               ({"out": Fake(15)}, -2), ({"O": Fake(21)}, -2), ({"a_off": [-1, 12]}, -2)):
            with pytest.raises(DmrgError) as e:
                lib_mod.renormalize_blocks(**{**ok, **change}, noalloc=noalloc)
            assert e.value.status == status, change
        lib_mod.renormalize_blocks(**{**ok, "sec_out": [], "sec_in": [], "a_off": [], "out_off": []},
                                   noalloc=noalloc)   # no blocks: no-op
    # a request beyond the fixed 64 MiB scratch is refused before any device work
    big = dict(dims=[3000], kept=[3000], o_off=[0], O=Fake(9_000_000), sec_out=[0], sec_in=[0], a_off=[0],
               A=Fake(9_000_000), out_off=[0], out=Fake(9_000_000))
    with pytest.raises(DmrgError) as e:
        lib_mod.renormalize_blocks(**big, noalloc=True)
    assert e.value.status == -3 and "scratch" in str(e.value)


def test_header_is_plain_c():
    """include/dmrg.h compiles as C99 (the boundary is a C ABI) and as C++17, without warnings."""
    import shutil
    import subprocess
    for cc, args in (("gcc", ["-std=c99", "-x", "c"]), ("g++", ["-std=c++17", "-x", "c++"])):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        r = subprocess.run([cc, *args, "-Wall", "-Wextra", "-Werror", "-fsyntax-only", HEADER],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
