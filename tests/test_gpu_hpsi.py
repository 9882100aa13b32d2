"""GPU parity of the HIP H.psi path (through the C-ABI) against the FP64 oracle.

Bars: FP64 path element-wise within 1e-12 relative to max|y| (only the summation order differs);
split-BF16 path element by element within 2^-12 of the size of that element's summands (the error
model of the 2-term BF16 split, ``helpers.assert_split_bound``); Davidson energies with
exact blocks equal the FCI energy within 1e-10 (FP64) and within 1e-6 Eh for split + FP64 polish.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle.davidson import davidson
from oracle.fci import FCI
from oracle.hpsi import OracleHop
from helpers import assert_split_bound, exact_problem, rel_err, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
FP64_TOL = 1e-12


def gpu_hpsi(hop, x, precision=PREC_FP64):
    xd = torch.as_tensor(x, dtype=torch.float64, device=DEV).contiguous()
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, precision)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


CASES = {
    # name: (builder, args) -- sizes span several 32x32 tiles and ragged edges
    "cfg0_exact_L8": (exact_problem, (8, 0)),
    "exact_L10_odd": (exact_problem, (10, 1, 5, 4)),
    "trunc_L10_M50": (exact_problem, (10, 2, 5, 5, 50)),
    "synth_L12_M70": (synth, (12, 70, 0.9, 3)),
    "synth_L14_M160_big_sectors": (synth, (14, 160, 0.7, 4)),
    # sectors up to 139 states: targets above the 96-wide LDS stages take the one-wavefront kernel
    "synth_L14_M300_sectors_above_96": (synth, (14, 300, 0.6, 5)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    fn, args = CASES[request.param]
    h, eri, left, right, na, nb, site = fn(*args)
    print(f"[case {request.param}] building", flush=True)
    hop = Hop(h, eri, left, right, na, nb, site, device=0, want_split=True)
    oh = OracleHop(h, eri, left, right, na, nb, site)
    return request.param, hop, oh


def test_layout_matches_oracle(case):
    name, hop, oh = case
    assert [tuple(b[:4]) for b in oh.layout.blocks] == [tuple(r) for r in hop.abcd]
    assert hop.n_coeff == oh.layout.size


def test_fp64_matches_oracle(case):
    name, hop, oh = case
    x = random_vector(hop.n_coeff, 11)
    y = gpu_hpsi(hop, x)
    assert rel_err(y, oh.apply(x)) < FP64_TOL, name


def test_split_matches_oracle(case):
    name, hop, oh = case
    x = random_vector(hop.n_coeff, 12)
    y = gpu_hpsi(hop, x, PREC_SPLIT2)
    ref = oh.apply(x)
    print(f"[{name}] split rel err {rel_err(y, ref):.2e}", flush=True)
    assert_split_bound(y, ref, oh.magnitude(x), name)


def test_diag_matches_oracle(case):
    name, hop, oh = case
    d = torch.empty(hop.n_coeff, dtype=torch.float64, device=DEV)
    hop.diagonal(d)
    torch.cuda.synchronize()
    assert rel_err(d.cpu().numpy(), oh.diagonal()) < FP64_TOL


def test_deterministic_and_multivector(case):
    name, hop, oh = case
    X = np.stack([random_vector(hop.n_coeff, 20 + k) for k in range(3)])
    xd = torch.as_tensor(X, device=DEV).contiguous()
    y1 = torch.empty_like(xd)
    y2 = torch.empty_like(xd)
    hop.hpsi(xd, y1)
    hop.hpsi(xd, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    for k in range(3):
        assert np.array_equal(y1[k].cpu().numpy(), gpu_hpsi(hop, X[k]))


def test_hermiticity_gpu(case):
    name, hop, oh = case
    x, z = random_vector(hop.n_coeff, 1), random_vector(hop.n_coeff, 2)
    hx, hz = gpu_hpsi(hop, x), gpu_hpsi(hop, z)
    assert abs(x @ hz - hx @ z) < 1e-12 * np.linalg.norm(hx) * np.linalg.norm(z)


def test_alias_rejected():
    h, eri, left, right, na, nb, site = exact_problem(6, 0)
    hop = Hop(h, eri, left, right, na, nb, site, device=0)
    x = torch.zeros(hop.n_coeff, dtype=torch.float64, device=DEV)
    with pytest.raises(lib_mod.DmrgError) as e:
        hop.hpsi(x, x)
    assert e.value.status == -6


def test_davidson_cfg0_equals_fci():
    """Config 0: L=8, (4,4), M=64 exact blocks, Davidson to 1e-10 on the GPU equals FCI."""
    h, eri, left, right, na, nb, site = exact_problem(8, 0)
    hop = Hop(h, eri, left, right, na, nb, site, device=0, want_split=True)
    e_fci, _ = FCI(h, eri, na, nb).ground_state()
    psi = torch.as_tensor(random_vector(hop.n_coeff, 0), device=DEV)
    r = hop.davidson(psi, tol=1e-10, max_iter=300)
    print(f"[cfg0] fp64 E={r['energy']:.12f} FCI={e_fci:.12f} iters={r['iters']}")
    assert r["converged"] and abs(r["energy"] - e_fci) < 1e-10
    psi2 = torch.as_tensor(random_vector(hop.n_coeff, 0), device=DEV)
    r2 = hop.davidson(psi2, tol=1e-8, max_iter=300, precision=PREC_SPLIT2, fp64_polish=True, split_tol=1e-4)
    print(f"[cfg0] split+polish E={r2['energy']:.12f} matvecs={r2['matvecs']} split={r2['matvecs_split']}")
    assert r2["converged"] and abs(r2["energy"] - e_fci) < 1e-6
    # the eigenvector: residual of the oracle operator
    oh = OracleHop(h, eri, left, right, na, nb, site)
    v = psi.cpu().numpy()
    assert np.linalg.norm(oh.apply(v) - r["energy"] * v) < 1e-9


def test_davidson_matches_oracle_truncated():
    h, eri, left, right, na, nb, site = exact_problem(10, 3, 5, 5, 60)
    hop = Hop(h, eri, left, right, na, nb, site, device=0)
    oh = OracleHop(h, eri, left, right, na, nb, site)
    ref = davidson(oh.apply, oh.diagonal(), random_vector(hop.n_coeff, 4), tol=1e-9)
    psi = torch.as_tensor(random_vector(hop.n_coeff, 4), device=DEV)
    r = hop.davidson(psi, tol=1e-9, max_iter=400, max_sub=16)
    assert r["converged"] and abs(r["energy"] - ref["energy"]) < 1e-9
