"""GPU parity of Eq. renorm_mat (dmrg_renormalize_blocks, out = O_out^T A O_in per sector block)
through the C-ABI.

* Oracle case: one renormalization step at the bond (2, 3) of L = 6 with exact blocks (the oracle's
  step keeps the FCI energy, pinned on the CPU): the grown block's H, C, B and S operators in the
  enlarged basis, O from the oracle's cut to M = 12; GPU = oracle.renorm.renormalize.
* Random case: sectors of 1, 17, 64, 130 and 200 states keeping 0, 5, 64, 33 and 97, every sector
  pair, random orthonormal O; GPU = O_out^T A O_in in numpy.
Bars: within 1e-13 (oracle case) and 1e-12 (random case) of the largest element; two calls bitwise
equal; untouched output padding stays NaN (no write outside the blocks).
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals
from oracle import renorm
from oracle.blocking import GrownLeft
from oracle.fci import FCI
from oracle.fock import exact_block, project
from oracle.hamiltonian import spin_orbital_integrals
from oracle.hpsi import OracleHop

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def run(dims, kept, Os, blocks):
    """Os: per sector (d, k) arrays; blocks: list of (so, si, A). Returns the list of GPU outputs."""
    o_off = np.concatenate([[0], np.cumsum([d * k for d, k in zip(dims, kept)])]).astype(np.int64)
    O = np.concatenate([o.ravel() for o in Os] + [np.zeros(1)])
    a_off = np.concatenate([[0], np.cumsum([A.size for _, _, A in blocks])]).astype(np.int64)
    A = np.concatenate([A.ravel() for _, _, A in blocks])
    sizes = [kept[so] * kept[si] for so, si, _ in blocks]
    out_off = np.concatenate([[0], np.cumsum([s + 3 for s in sizes])]).astype(np.int64)   # 3 NaN guards each
    res = []
    for _ in range(2):
        out = torch.full((int(out_off[-1]),), float("nan"), dtype=torch.float64, device=DEV)
        lib_mod.renormalize_blocks(dims, kept, o_off[:-1], torch.as_tensor(O, device=DEV),
                                   [b[0] for b in blocks], [b[1] for b in blocks], a_off[:-1],
                                   torch.as_tensor(A, device=DEV), out_off[:-1], out)
        torch.cuda.synchronize()
        res.append(out.cpu().numpy())
    assert np.array_equal(res[0], res[1], equal_nan=True)
    r = res[0]
    outs = []
    for b, (so, si, _) in enumerate(blocks):
        seg = r[out_off[b]:out_off[b + 1]]
        if sizes[b]:
            outs.append(seg[:sizes[b]].reshape(kept[so], kept[si]))
            assert not np.any(np.isnan(outs[-1]))
        else:
            outs.append(np.zeros((kept[so], kept[si])))
        assert np.all(np.isnan(seg[sizes[b]:]))
    return outs


def test_renorm_mat_matches_oracle_step():
    L, s1, na, nb = 6, 2, 3, 3
    h, eri = random_integrals(L, 5)
    t, w = spin_orbital_integrals(h, eri)
    left = exact_block(list(range(s1)), "left", t, w, [P for P in range(2 * L) if P // 2 >= s1])
    right = exact_block(list(range(s1 + 2, L)), "right", t, w, [P for P in range(2 * L) if P // 2 <= s1 + 1])
    hop = OracleHop(h, eri, left, right, na, nb, s1)
    fci = FCI(h, eri, na, nb)
    _, c = fci.ground_state()
    psi = project(hop.layout, c, left, right, s1, s1 + 1, fci.dets)
    O, _, _ = renorm.select(renorm.rdm_left(renorm.psi_matrices(hop.layout, left, right, na, nb, psi)), 12)
    g = GrownLeft(left, t, w, s1)
    _, edims = renorm.enlarged_left_basis(left)
    qs = list(edims)
    dims = [edims[q] for q in qs]
    kept = [O[q].shape[1] if q in O else 0 for q in qs]
    Os = [O[q] if q in O else np.zeros((edims[q], 0)) for q in qs]
    worst = 0.0
    for name, M in (("H", g.H()), ("C", g.C(g.smodes[1])), ("B", g.B(1, g.smodes[0])), ("S", g.S(2 * s1 + 2))):
        A = g.to_sectors(M)
        blocks = [(qs.index(qo), qs.index(qi), blk) for (qo, qi), blk in A.items()]
        ref = renorm.renormalize(A, O, O)
        got = run(dims, kept, Os, blocks)
        scale = max(float(np.abs(m).max()) for m in A.values())
        for (so, si, _), gb in zip(blocks, got):
            key = (qs[so], qs[si])
            want = ref.get(key, np.zeros((kept[so], kept[si])))
            worst = max(worst, float(np.abs(gb - want).max(initial=0.0)) / scale)
        print(f"[renorm] oracle step {name}: {len(blocks)} blocks", flush=True)
    print(f"[renorm] oracle step: max err {worst:.2e} of max|A|", flush=True)
    assert worst < 1e-13


def test_renorm_mat_random_sectors():
    rng = np.random.default_rng(8)
    dims, kept = [1, 17, 64, 130, 200], [0, 5, 64, 33, 97]
    Os = [np.linalg.qr(rng.normal(size=(d, d)))[0][:, :k] if d else np.zeros((0, 0)) for d, k in zip(dims, kept)]
    blocks = [(so, si, rng.normal(size=(dims[so], dims[si]))) for so in range(5) for si in range(5)]
    got = run(dims, kept, Os, blocks)
    worst = 0.0
    for (so, si, A), gb in zip(blocks, got):
        want = Os[so].T @ A @ Os[si]
        worst = max(worst, float(np.abs(gb - want).max(initial=0.0)))
    print(f"[renorm] random sectors: max err {worst:.2e}", flush=True)
    assert worst < 1e-12 * max(float(np.abs(A).max()) for _, _, A in blocks) * 10
