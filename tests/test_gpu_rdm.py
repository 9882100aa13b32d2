"""GPU parity of the reduced density matrices rho^L = psi psi^T and rho^R = psi^T psi (Section 2.1)
through the C-ABI (dmrg_rdm_left, dmrg_rdm_right) against the oracle (oracle.renorm, pinned on the
CPU against FCI Schmidt values). Sectors that psi does not reach are zero.

Cases: exact blocks at L = 8 (config 0 shape) with the FCI ground state and with a random vector;
truncated blocks with odd N; synthetic blocks at L = 14, M = 300 (sectors up to 139 states); an edge
bond. Bars: every sector block within 1e-13 of the largest element (FP64, summation order only);
rho symmetric, trace = |psi|^2; two calls bitwise equal.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle import renorm
from oracle.layout import Layout
from helpers import exact_problem, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop = lib_mod.Hop

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
CASES = {"exact8": lambda: exact_problem(8, 0), "trunc10_odd": lambda: exact_problem(10, 1, n_alpha=5, n_beta=4, trunc=40),
         "synth14_M300": lambda: synth(14, 300, 0.6, 5), "edge6_right_empty": lambda: exact_problem(6, 3, site=4)}


@pytest.mark.parametrize("side", ["left", "right"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_rdm_matches_oracle(name, side):
    print(f"[rdm] {name} {side}", flush=True)
    p = CASES[name]()
    h, eri, left, right, na, nb, site = p
    hop = Hop(*p, device=0)
    layout, call = (hop.rdm_left_layout, hop.rdm_left) if side == "left" else (hop.rdm_right_layout, hop.rdm_right)
    qn, dims, off = layout()
    x = random_vector(hop.n_coeff, 21)
    P = renorm.psi_matrices(Layout(left, right, na, nb), left, right, na, nb, x)
    ref = renorm.rdm_left(P) if side == "left" else renorm.rdm_right(P, na, nb)
    xd = torch.as_tensor(x, device=DEV)
    rho = torch.full((int(off[-1]),), float("nan"), dtype=torch.float64, device=DEV)
    call(xd, rho)
    torch.cuda.synchronize()
    r = rho.cpu().numpy()
    assert not np.any(np.isnan(r))
    scale = max(float(np.abs(m).max()) for m in ref.values() if m.size)
    err = 0.0
    for i, q in enumerate(qn):
        got = r[off[i]:off[i + 1]].reshape(dims[i], dims[i])
        want = ref.get((int(q[0]), int(q[1])), np.zeros((dims[i], dims[i])))
        err = max(err, float(np.abs(got - want).max(initial=0.0)))
        assert np.array_equal(got, got.T)
    print(f"[rdm] {name} {side}: {len(dims)} sectors, {int(off[-1])} elements, max err {err:.2e} of {scale:.2e}", flush=True)
    assert err < 1e-13 * scale
    tr = sum(float(np.trace(r[off[i]:off[i + 1]].reshape(dims[i], dims[i]))) for i in range(len(dims)))
    assert abs(tr - float(x @ x)) < 1e-12 * float(x @ x)
    rho2 = torch.empty_like(rho)
    call(xd, rho2)
    torch.cuda.synchronize()
    assert torch.equal(rho, rho2)
