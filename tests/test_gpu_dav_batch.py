"""GPU tests of the batched, device-resident Davidson (dmrg_davidson_batch) through the C-ABI.

* Exact problems: four parts with exact blocks from the oracle's Fock space (L = 6, 8, 8 with other
  integrals, 7 with N = (4, 3)), merged into one handle; every part's energy equals its FCI ground
  state within 1e-9, and its Ritz vector has a residual under the oracle's H.psi below 1e-8.
* Agreement with the single-problem Davidson: six uneven synthetic parts (L 10..14, M 30..120);
  every part's energy equals dmrg_davidson on its own handle within 1e-10 (same tolerance, 1e-10).
* Restarts (max_sub = 4: the subspace is collapsed to {u, u_prev} every second iteration) give the
  same energies; the graph-captured launch sequence gives the eager one's results bit for bit.
* Split precision with an FP64 polish: energies within 1e-8 of the FP64 ones.
* Errors: max_sub < 3 is rejected; a part with a zero start vector is an argument error.
* Part mask: the merged H.psi skips the work of parts that have left the active set; parts whose
  sectors take every H.psi route (up to 139 states: the two-pass large-block kernels and the
  LDS-staged ones, next to one-wavefront problems), in plans with cut items (partial tiles and their
  reductions) and with the large-block and FP64 LDS-staged paths off, give the same energies and Ritz
  vectors bit for bit with the mask as without it (DMRG_BATCH_PART_MASK=0).
"""
import os

import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle.fci import FCI
from oracle.hpsi import OracleHop
from helpers import exact_problem, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def start(hop, seed):
    return torch.as_tensor(random_vector(hop.n_coeff, seed), device=DEV)


@pytest.fixture(scope="module")
def exact():
    specs = [(6, 1, None, None), (8, 0, None, None), (8, 5, None, None), (7, 2, 4, 3)]
    probs, hops = [], []
    for L, seed, na, nb in specs:
        p = exact_problem(L, seed, na, nb)
        probs.append(p)
        h, eri, left, right, na_, nb_, site = p
        hops.append(Hop(h, eri, left, right, na_, nb_, site, device=0, want_split=True))
    return probs, hops, Hop.combine(hops)


@pytest.fixture(scope="module")
def synthetic():
    rng = np.random.default_rng(7)
    hops = []
    for k in range(6):
        L = int(rng.integers(10, 15))
        M = int(rng.integers(30, 120))
        h, eri, left, right, na, nb, site = synth(L, M, 1.0 + 0.2 * k, 300 + k)
        hops.append(Hop(h, eri, left, right, na, nb, site, device=0, want_split=True))
    return hops, Hop.combine(hops)


def test_exact_parts_equal_fci(exact):
    probs, hops, comb = exact
    psi = start(comb, 11)
    r = comb.davidson_batch(psi, tol=1e-10, max_iter=400, max_sub=24)
    print(f"[dav batch] exact: energies {r['energy']}, iters {r['iters']}, graphs {r['graphs']}", flush=True)
    assert r["converged"] and list(r["status"]) == [0] * len(probs)
    v = psi.cpu().numpy()
    for p, (h, eri, left, right, na, nb, site) in enumerate(probs):
        e_fci = FCI(h, eri, na, nb).ground_state()[0]
        assert abs(r["energy"][p] - e_fci) < 1e-9, (p, r["energy"][p], e_fci)
        seg = v[comb.part_coeff[p]:comb.part_coeff[p + 1]]
        oh = OracleHop(h, eri, left, right, na, nb, site)
        assert abs(np.linalg.norm(seg) - 1.0) < 1e-10
        assert np.linalg.norm(oh.apply(seg) - r["energy"][p] * seg) < 1e-8


def test_parts_equal_single_davidson(synthetic):
    hops, comb = synthetic
    psi = start(comb, 21)
    r = comb.davidson_batch(psi, tol=1e-10, max_iter=600, max_sub=24)
    assert r["converged"]
    for p, hop in enumerate(hops):
        x = start(hop, 31 + p)
        s = hop.davidson(x, tol=1e-10, max_iter=600, max_sub=24)
        print(f"[dav batch] part {p}: batched {r['energy'][p]:.12f} ({r['iters'][p]} it), "
              f"single {s['energy']:.12f} ({s['iters']} it)", flush=True)
        assert s["converged"]
        assert abs(r["energy"][p] - s["energy"]) < 1e-10 * max(1.0, abs(s["energy"]))


def test_restarts_graph_and_eager_agree(synthetic):
    hops, comb = synthetic
    ref = comb.davidson_batch(start(comb, 21), tol=1e-10, max_iter=600, max_sub=24)
    out = {}
    for use_graph in (True, False):
        psi = start(comb, 21)
        r = comb.davidson_batch(psi, tol=1e-10, max_iter=2000, max_sub=4, use_graph=use_graph)
        out[use_graph] = (r, psi.cpu().numpy())
        print(f"[dav batch] max_sub 4, graph {use_graph}: iters {r['iters']}, graphs {r['graphs']}", flush=True)
        assert r["converged"]
        assert np.allclose(r["energy"], ref["energy"], rtol=0, atol=1e-9 * np.abs(ref["energy"]).max())
    (rg, vg), (re, ve) = out[True], out[False]
    assert rg["graphs"] > 0 and re["graphs"] == 0
    assert np.array_equal(rg["energy"], re["energy"]) and np.array_equal(vg, ve)


def test_split_polish_matches_fp64(synthetic):
    hops, comb = synthetic
    ref = comb.davidson_batch(start(comb, 21), tol=1e-10, max_iter=600, max_sub=24)
    r = comb.davidson_batch(start(comb, 21), tol=1e-9, max_iter=600, max_sub=24, precision=PREC_SPLIT2,
                            fp64_polish=True, split_tol=1e-4)
    print(f"[dav batch] split + polish: max |dE| {np.abs(r['energy'] - ref['energy']).max():.2e}", flush=True)
    assert r["converged"]
    assert np.abs(r["energy"] - ref["energy"]).max() < 1e-8 * np.abs(ref["energy"]).max()


def test_argument_errors(exact):
    probs, hops, comb = exact
    with pytest.raises(lib_mod.DmrgError):
        comb.davidson_batch(start(comb, 1), max_sub=2)
    psi = start(comb, 1)
    psi[comb.part_coeff[1]:comb.part_coeff[2]] = 0.0
    with pytest.raises(lib_mod.DmrgError):
        comb.davidson_batch(psi)


MASK_PLANS = {
    "default": {},
    "cut": {"DMRG_BIG64": "2", "DMRG_BIG_STAGES": "4", "DMRG_BIG_STAGES1": "4", "DMRG_BIG_TBUDGET_MB": "16",
            "DMRG_LDS_ITEMS": "64", "DMRG_LDS64_ITEMS": "64", "DMRG_ITEMS": "256"},
    "off": {"DMRG_BIG": "0", "DMRG_BIG64": "0", "DMRG_LDS64": "0"},
}


def with_env(env, fn):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.fixture(scope="module")
def mixed_problems():
    # (L, M, sigma, seed): sectors up to 139 states (L = 14, M = 300), up to about 110, and small ones
    return [synth(L, M, sg, sd) for L, M, sg, sd in ((14, 300, 0.6, 5), (12, 50, 1.0, 311), (14, 200, 0.8, 9),
                                                     (10, 40, 1.2, 312))]


@pytest.mark.parametrize("plan", sorted(MASK_PLANS))
def test_part_mask_bitwise(mixed_problems, plan):
    def build():
        hops = [Hop(*p, device=0, want_split=True) for p in mixed_problems]
        return Hop.combine(hops)
    comb = with_env(MASK_PLANS[plan], build)
    out = {}
    for mask in ("1", "0"):
        psi = start(comb, 51)
        r = with_env({"DMRG_BATCH_PART_MASK": mask},
                     lambda: comb.davidson_batch(psi, tol=1e-8, max_iter=600, max_sub=16, precision=PREC_SPLIT2,
                                                 fp64_polish=True, split_tol=1e-4))
        print(f"[dav batch] mask {mask}, plan {plan}: iters {r['iters']}, energies {r['energy']}", flush=True)
        assert r["converged"]
        out[mask] = (r, psi.cpu().numpy())
    (r1, v1), (r0, v0) = out["1"], out["0"]
    assert len(set(r1["iters"].tolist())) > 1          # parts leave the active set at different iterations
    assert np.array_equal(r1["energy"], r0["energy"]) and np.array_equal(r1["iters"], r0["iters"])
    assert np.array_equal(v1, v0)
    # every plan converges to the same energies (FP64 polish to 1e-8)
    for other, e in _MASK_ENERGIES.items():
        assert np.allclose(r1["energy"], e, rtol=0, atol=1e-9 * np.abs(e).max()), (plan, other)
    _MASK_ENERGIES[plan] = r1["energy"]


_MASK_ENERGIES = {}
