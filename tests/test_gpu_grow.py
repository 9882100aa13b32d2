"""GPU parity of block growth and renormalization (Section 2.1: the enlarged block's operators, the
M-state cut, Eq. renorm and Eq. renorm_mat; Section 2.2.2) through the C-ABI, against the oracle.

* dmrg_block_grow with a given O: every operator of the grown block (left: H, C, A, B, S; right: H,
  C, U, P, Q) equals the oracle's grown_block -- the exact operators of the grown orbital set in its
  own Fock space, projected onto the kept basis -- within 1e-12 of the operator's largest element;
  exact and randomly truncated old blocks, both sides, L = 6 and L = 8, several sectors keeping no
  state. kept = O = NULL keeps every state.
* dmrg_renormalize (rho from psi on the GPU, the host cut, growth): from the FCI ground state at the
  bond (2, 3) of L = 6, the kept dimensions and the discarded weight equal the oracle's cut; the
  next bond (left growth) and the previous bond (right growth) built from the returned block have,
  under Davidson, the FCI energy when nothing is discarded and the oracle's energy when truncated.
* Failure paths of Davidson and of the build: DMRG_NOT_CONVERGED (max_iter = 1, best pair returned)
  and DMRG_ERR_NOMEM (a device-memory budget below what the operator needs).
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals, random_vector
from oracle import renorm
from oracle.blocking import grown_block
from oracle.fci import FCI
from oracle.fock import exact_block, project, random_bases, truncate
from oracle.hamiltonian import spin_orbital_integrals
from oracle.hpsi import OracleHop

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop = lib_mod.Hop

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def dense(block, op):
    off = np.concatenate([[0], np.cumsum(block.dim)]).astype(np.int64)
    D = np.zeros((off[-1], off[-1]))
    if op is not None:
        for (so, si), m in op.blocks.items():
            D[off[so]:off[so + 1], off[si]:off[si + 1]] = m
    return D


def expected_ops(side, L, site):
    """(kind, i0, i1) of the grown block's stored operators, in the library's order."""
    if side == 0:
        mine = list(range(0, 2 * site + 2))
        ops = [("H", -1, -1)] + [("C", P, -1) for P in mine]
        ops += [("A", P, Q) for P in mine for Q in mine if P < Q]
        ops += [("B", P, Q) for P in mine for Q in mine if P <= Q]
        ops += [("S", W, -1) for W in range(2 * site + 2, 2 * L)]
    else:
        mine = list(range(2 * (site + 1), 2 * L))
        out = list(range(0, 2 * (site + 1)))
        ops = [("H", -1, -1)] + [("C", Z, -1) for Z in mine]
        ops += [("U", P, -1) for P in out]
        ops += [("P", P, Q) for P in out for Q in out if P < Q]
        ops += [("Q", X, Y) for X in out for Y in out if X <= Y]
    return ops


def compare_blocks(got, want, side, L, site):
    assert got.qn.tolist() == want.qn.tolist() and got.dim.tolist() == want.dim.tolist()
    assert [op.key for op in got.ops] == expected_ops(side, L, site)
    worst = 0.0
    for op in got.ops:
        D = dense(got, op)
        W = dense(want, want.get(*op.key))
        scale = max(1.0, float(np.abs(W).max(initial=0.0)))
        worst = max(worst, float(np.abs(D - W).max(initial=0.0)) / scale)
    return worst


CASES = {
    # name: (L, s1, seed, side, truncate old block to, M kept fraction)
    "L6_left_exact": (6, 2, 5, 0, None),
    "L6_right_exact": (6, 2, 5, 1, None),
    "L8_left_trunc": (8, 3, 6, 0, 20),
    "L8_right_trunc": (8, 3, 6, 1, 20),
    "L8_left_edge": (8, 0, 7, 0, None),          # the vacuum grows into one orbital
    "L8_right_edge": (8, 6, 7, 1, None),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_block_grow_matches_oracle(name):
    L, s1, seed, side, trunc = CASES[name]
    print(f"[grow] {name}", flush=True)
    h, eri = random_integrals(L, seed)
    t, w = spin_orbital_integrals(h, eri)
    if side == 0:
        old = exact_block(list(range(s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
        site = s1
    else:
        old = exact_block(list(range(s1 + 2, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s1 + 1])
        site = s1 + 1
    if trunc is not None:
        old = truncate(old, random_bases(old, trunc, seed + 50))
    qn, dims = lib_mod.block_grow_layout(old, side)
    _, odims = (renorm.enlarged_left_basis if side == 0 else renorm.enlarged_right_basis)(old)
    assert [tuple(int(v) for v in q) for q in qn] == list(odims) and dims.tolist() == list(odims.values())
    rng = np.random.default_rng(seed)
    O = []
    for k, d in enumerate(dims):
        keep = 0 if k % 5 == 3 else max(1, (2 * int(d)) // 3)
        O.append(np.linalg.qr(rng.normal(size=(d, d)))[0][:, :keep])
    got = lib_mod.block_grow(h, eri, (L + 1) // 2, L // 2, s1, old, side, O=O)
    want = grown_block("left" if side == 0 else "right", old, site,
                       {tuple(int(v) for v in q): o for q, o in zip(qn, O)}, t, w)
    err = compare_blocks(got, want, side, L, s1)
    print(f"[grow] {name}: {len(got.ops)} operators, max err {err:.2e}", flush=True)
    assert err < 1e-12


def test_block_grow_keep_all_is_exact():
    L, s1 = 6, 2
    h, eri = random_integrals(L, 8)
    t, w = spin_orbital_integrals(h, eri)
    old = exact_block(list(range(s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    got = lib_mod.block_grow(h, eri, 3, 3, s1, old, 0)
    _, odims = renorm.enlarged_left_basis(old)
    want = grown_block("left", old, s1, {q: np.eye(d) for q, d in odims.items()}, t, w)
    assert compare_blocks(got, want, 0, L, s1) < 1e-12


# ---------------------------------------------------------------- dmrg_renormalize: one sweep step
@pytest.fixture(scope="module")
def step():
    L, s1, na, nb = 6, 2, 3, 3
    h, eri = random_integrals(L, 5)
    t, w = spin_orbital_integrals(h, eri)
    left = exact_block(list(range(s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    right = exact_block(list(range(s1 + 2, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s1 + 1])
    oh = OracleHop(h, eri, left, right, na, nb, s1)
    fci = FCI(h, eri, na, nb)
    e_fci, c = fci.ground_state()
    psi = project(oh.layout, c, left, right, s1, s1 + 1, fci.dets)
    P = renorm.psi_matrices(oh.layout, left, right, na, nb, psi)
    hop = Hop(h, eri, left, right, na, nb, s1, device=0)
    return dict(h=h, eri=eri, t=t, w=w, left=left, right=right, na=na, nb=nb, s1=s1, e_fci=e_fci, P=P,
                psi=torch.as_tensor(psi, device=DEV), hop=hop, L=L)


def davidson_energy(hop, seed=0):
    psi = torch.as_tensor(random_vector(hop.n_coeff, seed), device=DEV)
    r = hop.davidson(psi, tol=1e-9, max_iter=400)
    assert r["converged"]
    return r["energy"]


@pytest.mark.parametrize("direction,M", [(0, 1000), (0, 12), (0, 6), (1, 1000), (1, 8)])
def test_renormalize_step(step, direction, M):
    s = step
    L, s1 = s["L"], s["s1"]
    block, disc = s["hop"].renormalize(s["psi"], direction, M)
    if direction == 0:
        rho = renorm.rdm_left(s["P"])
        O, kept, odisc = renorm.select(rho, M)
        want = grown_block("left", s["left"], s1, O, s["t"], s["w"])
        other = exact_block(list(range(s1 + 3, L)), "right", s["t"], s["w"], [P for P in range(2 * L) if P // 2 <= s1 + 2])
        args = (block, other, s["na"], s["nb"], s1 + 1)
        oargs = (want, other, s["na"], s["nb"], s1 + 1)
    else:
        rho = renorm.rdm_right(s["P"], s["na"], s["nb"])
        O, kept, odisc = renorm.select(rho, M)
        want = grown_block("right", s["right"], s1 + 1, O, s["t"], s["w"])
        other = exact_block(list(range(s1 - 1)), "left", s["t"], s["w"], [P for P in range(2 * L) if P // 2 >= s1 - 1])
        args = (other, block, s["na"], s["nb"], s1 - 1)
        oargs = (other, want, s["na"], s["nb"], s1 - 1)
    assert block.qn.tolist() == want.qn.tolist() and block.dim.tolist() == want.dim.tolist()
    assert abs(disc - odisc) < 1e-12
    e = davidson_energy(Hop(s["h"], s["eri"], *args, device=0))
    Hm = OracleHop(s["h"], s["eri"], *oargs).apply(np.eye(OracleHop(s["h"], s["eri"], *oargs).layout.size))
    e_oracle = float(np.linalg.eigvalsh(0.5 * (Hm + Hm.T))[0])
    print(f"[renormalize] dir {direction} M {M}: kept {int(block.dim.sum())}, discarded {disc:.3e}, "
          f"E {e:.12f} oracle {e_oracle:.12f} FCI {s['e_fci']:.12f}", flush=True)
    assert abs(e - e_oracle) < 1e-9
    if odisc < 1e-14:
        assert abs(e - s["e_fci"]) < 1e-9
    else:
        assert e > s["e_fci"] - 1e-10


# ---------------------------------------------------------------- failure paths
def test_davidson_not_converged_returns_best_pair(step):
    hop = step["hop"]
    psi = torch.as_tensor(random_vector(hop.n_coeff, 4), device=DEV)
    r = hop.davidson(psi, tol=1e-12, max_iter=1)
    assert not r["converged"] and r["iters"] == 1
    assert np.isfinite(r["energy"]) and r["energy"] >= step["e_fci"] - 1e-10
    assert abs(float(torch.linalg.norm(psi)) - 1.0) < 1e-12        # the Ritz vector, normalized


def test_build_over_memory_budget_is_nomem(step):
    s = step
    with pytest.raises(lib_mod.DmrgError) as e:
        Hop(s["h"], s["eri"], s["left"], s["right"], s["na"], s["nb"], s["s1"], device=0, mem_budget_bytes=1024)
    assert e.value.status == -3
