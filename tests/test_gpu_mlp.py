"""GPU tests of the learned Davidson preconditioner (dmrg_mlp_*) through the C-ABI.

Bars. Features: FP32 storage of FP64 values, 2e-6 relative (plus 1e-6 absolute). Network output
and gradients against the FP64 oracle (oracle/mlp.py) in the same precision: FP32 debug mode
against the FP64 network within 1e-5 relative (norm-wise per parameter group); BF16 matrix-core
mode against the oracle's BF16 mode (same rounding points, so the relu masks agree) within 1e-4
(output) and 1e-3 (gradients), and its output within 2e-2 of the FP64 network (BF16 keeps 8
significant bits of weights, inputs and first-layer activations). Adam: the
update of one step from the GPU's own gradient within 1e-6 absolute. A fresh network (zero output
layer) reproduces the diagonal-preconditioned Davidson exactly. Training pairs recorded during a
solve match the oracle's pairs for the first iteration (subspace V = [u]) within 1e-5.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle import mlp as omlp
from oracle.davidson import davidson
from oracle.hpsi import OracleHop
from helpers import exact_problem, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, Mlp = lib_mod.Hop, lib_mod.Mlp

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
GROUPS = {"W1": (0, omlp.OFF_B1), "b1": (omlp.OFF_B1, omlp.OFF_W2), "W2": (omlp.OFF_W2, omlp.OFF_B2),
          "b2": (omlp.OFF_B2, omlp.OFF_W3), "w3": (omlp.OFF_W3, omlp.OFF_B3), "b3": (omlp.OFF_B3, omlp.N_PARAMS)}


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _random_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(omlp.N_PARAMS)
    p[:omlp.OFF_B1] = rng.uniform(-1, 1, omlp.OFF_B1) * np.sqrt(6 / 16)
    p[omlp.OFF_B1:omlp.OFF_W2] = rng.normal(0, 0.1, 256)
    p[omlp.OFF_W2:omlp.OFF_B2] = rng.uniform(-1, 1, 256 * 256) * np.sqrt(6 / 256)
    p[omlp.OFF_B2:omlp.OFF_W3] = rng.normal(0, 0.1, 256)
    p[omlp.OFF_W3:omlp.OFF_B3] = rng.normal(0, 0.05, 256)
    p[omlp.OFF_B3] = 0.02
    return p.astype(np.float32)


def _batch(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, 16)).astype(np.float32)
    A = np.stack([rng.normal(0, 1, n), rng.normal(0, 1, n), rng.uniform(0.5, 1.5, n)], axis=1).astype(np.float32)
    return X, A


@pytest.fixture(scope="module")
def problem():
    # psi blocks up to 172 x 172 = 29584 coefficients: several feature chunks (16384) per block
    h, eri, left, right, na, nb, site = synth(14, 200, 0.4, 21)
    print("[mlp] building synth L=14 M=200", flush=True)
    hop = Hop(h, eri, left, right, na, nb, site, device=0)
    oh = OracleHop(h, eri, left, right, na, nb, site)
    return hop, oh


def test_features_match_oracle(problem):
    hop, oh = problem
    n = hop.n_coeff
    assert max(int(b[5]) * int(b[6]) for b in oh.layout.blocks) > 16384
    d = oh.diagonal()
    theta = float(d.min()) - 0.37
    r = random_vector(n, 1)
    u = random_vector(n, 2)
    u /= np.linalg.norm(u)
    feat = torch.empty((n, 16), dtype=torch.float32, device=DEV)
    t = torch.empty(n, dtype=torch.float64, device=DEV)
    Mlp.features(hop, _dev(r, torch.float64), _dev(u, torch.float64), theta, feat, t)
    torch.cuda.synchronize()
    blocks = [(b[4], b[5], b[6], b[1], b[2]) for b in oh.layout.blocks]
    F = omlp.features(blocks, r, u, d, theta)
    got = feat.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - F) <= 2e-6 * np.abs(F) + 1e-6)
    tref = omlp.diag_correction(r, d, theta)
    assert np.abs(t.cpu().numpy() - tref).max() <= 1e-12 * np.abs(tref).max()


@pytest.mark.parametrize("fp32,tol", [(True, 1e-5), (False, 1e-4)])
def test_forward_matches_oracle(fp32, tol):
    net = Mlp(device=0, seed=1)
    p = _random_params(3)
    net.set_params(p)
    net.set_fp32(fp32)
    X, _ = _batch(4, 1000)               # ragged: 1000 = 15 * 64 + 40
    out = torch.empty(1000, dtype=torch.float32, device=DEV)
    net.forward(_dev(X, torch.float32), out)
    torch.cuda.synchronize()
    m = out.cpu().numpy()
    m_ref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64), bf16=not fp32)
    err = np.abs(m - m_ref).max() / np.abs(m_ref).max()
    m_exact, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    dev_exact = np.abs(m - m_exact).max() / np.abs(m_exact).max()
    print(f"[mlp forward fp32={fp32}] rel err vs same-precision oracle {err:.2e}, vs FP64 network {dev_exact:.2e}")
    assert err < tol and dev_exact < 2e-2


@pytest.mark.parametrize("fp32,tol", [(True, 1e-5), (False, 1e-3)])
def test_gradient_matches_oracle(fp32, tol):
    net = Mlp(device=0, seed=1)
    p = _random_params(5)
    net.set_params(p)
    net.set_fp32(fp32)
    X, A = _batch(6, 300)
    grad = torch.empty(omlp.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    net.grad(_dev(X, torch.float32), _dev(A, torch.float32), grad, loss)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    p64, X64, A64 = p.astype(np.float64), X.astype(np.float64), A.astype(np.float64)
    gref = omlp.grad(p64, X64, A64, bf16=not fp32)
    gexact = omlp.grad(p64, X64, A64)
    lref = omlp.loss(p64, X64, A64, bf16=not fp32)
    assert abs(float(loss.cpu()[0]) - lref) <= tol * lref
    for name, (a, b) in GROUPS.items():
        e = np.linalg.norm(g[a:b] - gref[a:b]) / np.linalg.norm(gref[a:b])
        ex = np.linalg.norm(g[a:b] - gexact[a:b]) / np.linalg.norm(gexact[a:b])
        print(f"[mlp grad fp32={fp32}] {name}: rel err vs same-precision oracle {e:.2e}, vs FP64 network {ex:.2e}")
        assert e < tol, name


def test_adam_step_matches_oracle():
    net = Mlp(device=0, seed=1)
    p = _random_params(7)
    net.set_params(p)
    net.set_fp32(True)
    X, A = _batch(8, 256)
    grad = torch.empty(omlp.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    net.grad(_dev(X, torch.float32), _dev(A, torch.float32), grad, loss, lr=1e-3)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    z = np.zeros(omlp.N_PARAMS)
    pref, _, _ = omlp.adam(p.astype(np.float64), g, z, z, 1, 1e-3)
    assert np.abs(net.get_params() - pref).max() < 1e-6


def test_fresh_network_equals_diagonal_davidson(problem):
    hop, _ = problem
    net = Mlp(device=0, seed=9)
    runs = []
    for use in (None, net):
        psi = _dev(random_vector(hop.n_coeff, 11), torch.float64)
        runs.append(hop.davidson(psi, tol=1e-8, max_iter=200, mlp=use))
        runs[-1]["psi"] = psi.cpu().numpy()
    a, b = runs
    assert a["converged"] and b["converged"]
    assert a["iters"] == b["iters"] and a["energy"] == b["energy"]
    assert np.array_equal(a["psi"], b["psi"])


def test_collected_pairs_match_oracle():
    h, eri, left, right, na, nb, site = exact_problem(8, 0)
    hop = Hop(h, eri, left, right, na, nb, site, device=0)
    oh = OracleHop(h, eri, left, right, na, nb, site)
    n = hop.n_coeff
    x0 = random_vector(n, 13)
    net = Mlp(device=0, seed=2)
    res = net.collect(hop, _dev(x0, torch.float64), slot=0, rows_per_iter=n, tol=1e-10)
    assert res["converged"] and res["rows"] % n == 0 and res["rows"] >= n
    # first recorded iteration: u = x0 / |x0|, theta = <u, H u>, r = H u - theta u
    d = oh.diagonal()
    ref = davidson(oh.apply, d, x0, tol=1e-11, max_iter=300)
    u = x0 / np.linalg.norm(x0)
    hu = oh.apply(u)
    theta = float(u @ hu)
    r = hu - theta * u
    blocks = [(b[4], b[5], b[6], b[1], b[2]) for b in oh.layout.blocks]
    F = omlp.features(blocks, r, u, d, theta)
    P = omlp.pairs(omlp.diag_correction(r, d, theta), u, ref["vector"], np.arange(n))   # V = [u]
    feat, pairs = net.dataset(0, 0, n)
    assert np.all(np.abs(feat - F) <= 2e-6 * np.abs(F) + 1e-6)
    assert np.abs(pairs - P).max() <= 1e-5 * np.abs(P).max()


def test_training_lowers_validation_loss_and_ab():
    """Train on pairs from converged solves of four problems; the network must fit held-out pairs of
    a fifth problem better than the diagonal preconditioner (m = 0). A/B on the held-out problem:
    Davidson with each preconditioner from the same start at the same tolerance (1e-8) must reach
    the same energy, and the learned one must not need more iterations (training and solves are
    deterministic: fixed seeds, fixed-order reductions)."""
    net = Mlp(device=0, seed=5)
    train = [synth(10, 64, 0.8, 3000), synth(12, 64, 0.8, 3001), synth(12, 80, 1.0, 3002), synth(14, 96, 1.0, 3003)]
    for k, (h, eri, left, right, na, nb, site) in enumerate(train):
        hop = Hop(h, eri, left, right, na, nb, site, device=0)
        res = net.collect(hop, _dev(random_vector(hop.n_coeff, 40 + k), torch.float64), slot=0,
                          rows_per_iter=4096, seed=k, tol=1e-10)
        print(f"[mlp collect] train {k}: iters {res['iters']} rows {res['rows']}", flush=True)
        assert res["converged"]
    h, eri, left, right, na, nb, site = synth(12, 72, 0.9, 3100)
    hop = Hop(h, eri, left, right, na, nb, site, device=0)
    res = net.collect(hop, _dev(random_vector(hop.n_coeff, 50), torch.float64), slot=1, rows_per_iter=4096,
                      seed=9, tol=1e-10)
    assert res["converged"]
    before, diag = net.eval(1)
    assert before == pytest.approx(diag, rel=1e-12)          # fresh network == diagonal
    losses = net.train(3000, batch=2048, lr=1e-3, seed=1)
    after, _ = net.eval(1)
    print(f"[mlp train] minibatch loss {losses[:50].mean():.4f} -> {losses[-50:].mean():.4f}; "
          f"held-out loss diag {diag:.4f} mlp {after:.4f}", flush=True)
    assert np.all(np.isfinite(losses)) and after < 0.8 * diag
    ab = {}
    for name, use in (("diag", None), ("mlp", net)):
        psi = _dev(random_vector(hop.n_coeff, 77), torch.float64)
        ab[name] = hop.davidson(psi, tol=1e-8, max_iter=400, mlp=use)
        print(f"[mlp A/B] {name}: iters {ab[name]['iters']} E {ab[name]['energy']:.12f} "
              f"resid {ab[name]['resid']:.2e}", flush=True)
    assert ab["diag"]["converged"] and ab["mlp"]["converged"]
    assert abs(ab["diag"]["energy"] - ab["mlp"]["energy"]) < 1e-9
    assert ab["mlp"]["iters"] <= ab["diag"]["iters"]
