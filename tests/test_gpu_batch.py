"""GPU tests of batching (one launch sequence for many H.psi problems) and of the plan autotuner.

A merged handle must give, for every part, the H.psi of that part's own handle: identical up to the
order in which task contributions are summed (the work items are cut differently). FP64: bar 1e-12
relative to max|y|. Split precision: the per-task BF16 rounding is identical, but task results are
summed in FP32 over runs of at most 8 tasks before the FP64 update, and the runs start at item
boundaries, which differ between the two plans; each FP32 addition rounds at 2^-24 relative to the
running sum, so the bar is 2e-6 (measured 2.3e-7). One part is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle.hpsi import OracleHop
from helpers import rel_err, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(42)
    probs, hops = [], []
    for k in range(6):
        L = int(rng.integers(10, 15))
        M = int(rng.integers(30, 120))
        p = synth(L, M, 1.0 + 0.2 * k, 100 + k)
        print(f"[batch] part {k}: L={L} M={M}", flush=True)
        probs.append(p)
        h, eri, left, right, na, nb, site = p
        hops.append(Hop(h, eri, left, right, na, nb, site, device=0, want_split=True))
    comb = Hop.combine(hops)
    return probs, hops, comb


def _run(hop, x, prec):
    xd = torch.as_tensor(x, device=DEV)
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def test_combined_layout(batch):
    probs, hops, comb = batch
    assert comb.n_coeff == sum(h.n_coeff for h in hops)
    assert list(comb.part_coeff) == list(np.cumsum([0] + [h.n_coeff for h in hops]))
    assert comb.stats()["n_tasks"] == sum(h.stats()["n_tasks"] for h in hops)


BAR = {PREC_FP64: 1e-12, PREC_SPLIT2: 2e-6}


@pytest.mark.parametrize("prec", [PREC_FP64, PREC_SPLIT2])
def test_combined_equals_parts(batch, prec):
    probs, hops, comb = batch
    xs = [random_vector(h.n_coeff, 7 + k) for k, h in enumerate(hops)]
    ycomb = _run(comb, np.concatenate(xs), prec)
    for k, h in enumerate(hops):
        a, b = comb.part_coeff[k], comb.part_coeff[k + 1]
        assert rel_err(ycomb[a:b], _run(h, xs[k], prec)) < BAR[prec], k


def test_combined_part_matches_oracle(batch):
    probs, hops, comb = batch
    k = 3
    h, eri, left, right, na, nb, site = probs[k]
    xs = [random_vector(hh.n_coeff, 50 + i) for i, hh in enumerate(hops)]
    y = _run(comb, np.concatenate(xs), PREC_FP64)
    ref = OracleHop(h, eri, left, right, na, nb, site).apply(xs[k])
    assert rel_err(y[comb.part_coeff[k]:comb.part_coeff[k + 1]], ref) < 1e-12


def test_autotune_keeps_results(batch):
    probs, hops, comb = batch
    x = random_vector(comb.n_coeff, 3)
    allowed = {PREC_SPLIT2: {"lds_items": (4096, 8192, 16384, 32768, 65536), "lds_order": (0, 1, 2),
                             "small_shape": (0, 1, 2), "split64": (0, 1), "six_wave": (0, 0x8, 0xA),
                             "copy_wave": (0, 0xF), "prefetch": (0, 0x4)},
               PREC_FP64: {"lds64_items": (8192, 16384, 32768, 65536), "lds64_copy_wave": (0, 1),
                           "lds64_small": (0, 1), "lds64_w7_cap": (0, 1), "big64": (1, 2), "max_tq": (2, 4, 8),
                           "items": (8192, 32768, 65536), "order": (0, 2)}}
    for prec in (PREC_SPLIT2, PREC_FP64):
        before = _run(comb, x, prec)
        t = comb.autotune(prec, reps=2)
        print(f"[autotune] precision {prec}: {t}", flush=True)
        assert t["ms"] > 0
        for k, vals in allowed[prec].items():
            assert t[k] in vals, (prec, k, t[k])
        # a new plan moves the FP32 run boundaries of the split path and the FP64 summation order
        assert rel_err(_run(comb, x, prec), before) < (BAR[prec] if prec == PREC_SPLIT2 else 1e-13)


def test_trimmed_handles_combine_to_the_same_result():
    """dmrg_hop_trim keeps what merging needs: a merge of trimmed handles equals the merge of the
    untrimmed ones bit for bit, and a trimmed handle refuses H.psi (DMRG_ERR_UNSUPPORTED)."""
    ps = [synth(12, 60, 1.1, 300), synth(11, 40, 0.9, 301), synth(13, 90, 1.3, 302)]
    full = [Hop(*p, device=0, want_split=True) for p in ps]
    ref = Hop.combine(full)
    parts = [Hop(*p, device=0, want_split=True) for p in ps]
    xs = [random_vector(h.n_coeff, 70 + k) for k, h in enumerate(parts)]
    for h in parts:
        h.trim()
        h.trim()                                   # trimming twice does nothing
    with pytest.raises(lib_mod.DmrgError) as e:
        _run(parts[0], xs[0], PREC_FP64)
    assert e.value.status == -7
    comb = Hop.combine(parts)
    x = np.concatenate(xs)
    for prec in (PREC_FP64, PREC_SPLIT2):
        assert np.array_equal(_run(comb, x, prec), _run(ref, x, prec))
    d = torch.empty(parts[1].n_coeff, dtype=torch.float64, device=DEV)
    parts[1].diagonal(d)                           # diag(H) survives the trim
    torch.cuda.synchronize()
    d_ref = torch.empty_like(d)
    full[1].diagonal(d_ref)
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref)


def test_hpsi_batched_equals_each_handle(batch):
    """dmrg_hpsi_batched: every output equals its handle's own dmrg_hpsi bit for bit (same launch
    sequences), in both precisions; an output that overlaps another problem's input is refused."""
    probs, hops, comb = batch
    xs = [torch.as_tensor(random_vector(h.n_coeff, 80 + k), device=DEV) for k, h in enumerate(hops)]
    for prec in (PREC_FP64, PREC_SPLIT2):
        ys = [torch.empty_like(x) for x in xs]
        Hop.hpsi_batched(hops, xs, ys, prec)
        for h, x, y in zip(hops, xs, ys):
            ref = torch.empty_like(x)
            h.hpsi(x, ref, prec)
            torch.cuda.synchronize()
            assert torch.equal(y, ref)
    i = int(np.argmin([h.n_coeff for h in hops]))    # the smallest problem's output inside another's input
    j = (i + 1) % len(hops)
    bad = [torch.empty_like(x) for x in xs]
    bad[i] = xs[j][: hops[i].n_coeff]
    with pytest.raises(lib_mod.DmrgError):
        Hop.hpsi_batched(hops, xs, bad, PREC_FP64)
