"""GPU parity at uneven shapes through the C-ABI, with exact blocks (the oracle is the FCI matvec,
pinned on the CPU): strong spin imbalance N = (6, 2) at L = 8, the off-centre bond (2, 3) of L = 9
with N = (5, 3), two holes (5, 5) at L = 6, and a single electron at L = 6.

Bars: H.psi FP64 within 1e-12 of max|y|, split within its error bound (helpers.assert_split_bound); Davidson (FP64) reaches the FCI
ground-state energy within 1e-10.
"""
import pytest

from dmrg_inputs import random_vector
from oracle.fci import FCI
from oracle.hpsi import OracleHop
from helpers import assert_split_bound, exact_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
CASES = {"spin_polarized8": (8, 4, 6, 2, None), "off_center9": (9, 5, 5, 3, 2), "near_full6": (6, 6, 5, 5, None),
         "one_electron6": (6, 7, 1, 0, None)}


def run(hop, x, prec):
    xd = torch.as_tensor(x, device=DEV).contiguous()
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("name", sorted(CASES))
def test_uneven_shape_matches_oracle_and_fci(name):
    L, seed, na, nb, site = CASES[name]
    print(f"[uneven] {name}", flush=True)
    p = exact_problem(L, seed, n_alpha=na, n_beta=nb, site=site)
    h, eri = p[0], p[1]
    hop = Hop(*p, device=0, want_split=True)
    oh = OracleHop(*p)
    x = random_vector(hop.n_coeff, 8)
    ref = oh.apply(x)
    ysp = run(hop, x, PREC_SPLIT2)
    e64, esp = rel_err(run(hop, x, PREC_FP64), ref), rel_err(ysp, ref)
    print(f"[uneven] {name}: n={hop.n_coeff} fp64 {e64:.2e} split {esp:.2e}", flush=True)
    assert e64 < 1e-12
    assert_split_bound(ysp, ref, oh.magnitude(x), name)
    e_fci, _ = FCI(h, eri, na, nb).ground_state()
    psi = torch.as_tensor(random_vector(hop.n_coeff, 0), device=DEV)
    r = hop.davidson(psi, tol=1e-10, max_iter=300, max_sub=min(24, max(2, hop.n_coeff)))
    print(f"[uneven] {name}: E={r['energy']:.12f} FCI={e_fci:.12f} iters={r['iters']}", flush=True)
    assert r["converged"] and abs(r["energy"] - e_fci) < 1e-10
