"""GPU tests of share mode (one device's share of the operator combinations, dmrg_build_opts.share).

With every operator supplied, share mode builds the same combinations as the default mode, so
H.psi must be identical bit for bit. With a subset of operators (the block Hamiltonians and some
B/Q, A/P pairs) H.psi is the sum of the Hamiltonian terms whose block operators are supplied: it
equals the oracle's share (FP64 within 1e-12 of max|y|, split within its error bound), is symmetric
(<x|Hy> = <Hx|y>, FP64, relative 1e-12) since the share keeps each term together with its Hermitian
partner, and is deterministic.
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals, random_vector
from dmrg_inputs.synthetic import share_ops, synthetic_block
from helpers import assert_split_bound, rel_err, synth
from oracle.hpsi import OracleHop

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def _run(hop, x, prec):
    xd = torch.as_tensor(x, device=DEV)
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def test_share_with_all_operators_equals_default():
    h, eri, left, right, na, nb, site = synth(12, 70, 0.9, 3)
    a = Hop(h, eri, left, right, na, nb, site, device=0, want_split=True)
    b = Hop(h, eri, left, right, na, nb, site, device=0, want_split=True, share=True)
    assert a.stats()["n_alpha"] == b.stats()["n_alpha"]
    x = random_vector(a.n_coeff, 9)
    for prec in (PREC_FP64, PREC_SPLIT2):
        assert np.array_equal(_run(a, x, prec), _run(b, x, prec))


@pytest.fixture(scope="module")
def share_hop():
    L, na, nb, M, sigma, seed = 16, 8, 8, 300, 0.8, 11
    site = L // 2 - 1
    h, eri = random_integrals(L, seed)
    left = synthetic_block("left", L, na, nb, site, M, sigma, seed + 1000, ops=share_ops("left", L, site, 12))
    right = synthetic_block("right", L, na, nb, site, M, sigma, seed + 2000, ops=share_ops("right", L, site, 12))
    print(f"[share] L={L} M={M}: max sector {int(left.dim.max())}", flush=True)
    return (Hop(h, eri, left, right, na, nb, site, device=0, want_split=True, share=True),
            OracleHop(h, eri, left, right, na, nb, site, share=True))


def test_share_subset_symmetric_and_split(share_hop):
    hop, oh = share_hop
    x, z = random_vector(hop.n_coeff, 1), random_vector(hop.n_coeff, 2)
    hx, hz = _run(hop, x, PREC_FP64), _run(hop, z, PREC_FP64)
    assert abs(x @ hz - hx @ z) <= 1e-12 * np.linalg.norm(hx) * np.linalg.norm(z)
    ysp = _run(hop, x, PREC_SPLIT2)
    assert np.array_equal(_run(hop, x, PREC_FP64), hx)
    # the oracle's share (the same Hamiltonian terms, from its own term-by-term expansion)
    ref = oh.apply(x)
    err = rel_err(hx, ref)
    print(f"[share] L=16 M=300 subset: {hop.stats()['n_alpha']} combinations, fp64 {err:.2e}", flush=True)
    assert err < 1e-12
    assert_split_bound(ysp, ref, oh.magnitude(x), "share")
