"""GPU tests of the hipGraph form of H.psi (dmrg_hpsi_graph) and of Davidson with use_graph = 1.

The graph replays exactly the launch sequence of dmrg_hpsi on the same plan, so every replay must
equal the eager result bit for bit; replays are interleaved with eager work and synchronizations,
and a rebuilt plan (autotune) must drop the old graphs and capture new ones.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle.hpsi import OracleHop
from helpers import assert_split_bound, rel_err, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def prob():
    p = synth(12, 70, 0.9, 3)
    h, eri, left, right, na, nb, site = p
    print("[graph] building L=12 M=70", flush=True)
    return p, Hop(h, eri, left, right, na, nb, site, device=0, want_split=True)


@pytest.mark.parametrize("prec", [PREC_FP64, PREC_SPLIT2])
def test_graph_replays_equal_eager(prob, prec):
    p, hop = prob
    x = torch.as_tensor(random_vector(hop.n_coeff, 31), device=DEV)
    x2 = torch.as_tensor(random_vector(hop.n_coeff, 32), device=DEV)
    y_eager = torch.empty_like(x)
    hop.hpsi(x, y_eager, prec)
    torch.cuda.synchronize()
    ref = y_eager.clone()
    y = torch.empty_like(x)
    for rep in range(4):
        y.fill_(float("nan"))
        hop.hpsi_graph(x, y, prec)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), rep
        # eager work on other buffers between replays (shares the plan's packing buffers)
        hop.hpsi(x2, y_eager, prec)
        torch.cuda.synchronize()
    h, eri, left, right, na, nb, site = p
    oh = OracleHop(h, eri, left, right, na, nb, site)
    xh = x.cpu().numpy()
    if prec == PREC_FP64:
        assert rel_err(y.cpu().numpy(), oh.apply(xh)) < 1e-12
    else:
        assert_split_bound(y.cpu().numpy(), oh.apply(xh), oh.magnitude(xh), "graph replay")


def test_graph_after_autotune(prob):
    p, hop = prob
    x = torch.as_tensor(random_vector(hop.n_coeff, 33), device=DEV)
    y = torch.empty_like(x)
    hop.hpsi_graph(x, y, PREC_SPLIT2)
    torch.cuda.synchronize()
    before = y.clone()
    hop.autotune(PREC_SPLIT2, reps=1)
    y2 = torch.empty_like(x)
    hop.hpsi(x, y2, PREC_SPLIT2)
    hop.hpsi_graph(x, y, PREC_SPLIT2)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    assert rel_err(y.cpu().numpy(), before.cpu().numpy()) < 2e-6   # new plan: FP32 run boundaries move


@pytest.mark.parametrize("prec", [PREC_FP64, PREC_SPLIT2])
def test_davidson_graph_equals_eager(prob, prec):
    p, hop = prob
    res = {}
    for g in (False, True):
        psi = torch.as_tensor(random_vector(hop.n_coeff, 5), device=DEV)
        r = hop.davidson(psi, tol=1e-8, max_iter=300, max_sub=16, precision=prec, fp64_polish=prec == PREC_SPLIT2,
                         split_tol=3e-5, use_graph=g)
        res[g] = (r, psi.cpu().numpy())
        print(f"[graph] davidson prec={prec} graph={g}: E={r['energy']:.12f} iters={r['iters']}", flush=True)
    (r0, v0), (r1, v1) = res[False], res[True]
    assert r0["converged"] and r1["converged"]
    assert r0["iters"] == r1["iters"] and r0["energy"] == r1["energy"]
    assert np.array_equal(v0, v1)
