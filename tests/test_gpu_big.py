"""GPU parity of the two-pass large-block path (targets whose own or source blocks exceed the 96-wide
LDS stages) against the FP64 oracle, through the C-ABI, in both precisions.

Case C has the large shape's sector sizes: 420-state sectors (four 128-row tiles, the last ragged)
next to 97-, 33-, 5- and 1-state ones (L = 12, |psi| = 9.3 M), checked on sampled targets.

Plan variants: every target above the LDS stages on the two-pass path in both precisions ("forced";
by default the FP64 path takes it only where its cost model says it is cheaper); a cut plan of the
same (16 MB T budget: several chunks; 4-step pass-1 workgroups: many groups per workgroup; 4-step
pass-2 items: task lists cut into partial tiles that ordered reductions add); the default choice
("auto"); the large-block path switched off (one-wavefront kernels); and "target_route": a target
with any source above the stages sends all its tasks to the large-block path (by default only those
tasks do, the rest of the target stays in the LDS-staged kernel), with the FP64 LDS kernel off; and
"copy_wave": the split row-mode classes with a copy wavefront (four and two row tiles per compute
wavefront); "lds64_route": FP64 targets within the 112-wide LDS-staged tiles keep the tasks whose
source fits them there and send only the larger-source tasks to the two-pass (or one-wavefront)
path, with the two-pass path chosen by cost or forced. Bars as for
every H.psi: FP64 within 1e-12 of max|y|, split element by element within its error bound
(helpers.assert_split_bound); split plans that move FP32 run boundaries agree within 2e-6; every
plan is deterministic bit for bit.
"""
import os

import numpy as np
import pytest

from dmrg_inputs import random_integrals, random_vector
from dmrg_inputs.synthetic import synthetic_block
from oracle.hpsi import OracleHop
from helpers import assert_split_bound, rel_err, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
FP64_TOL = 1e-12
VARIANTS = {
    "forced": {"DMRG_BIG64": "2"},
    "cut": {"DMRG_BIG64": "2", "DMRG_BIG_STAGES": "4", "DMRG_BIG_STAGES1": "4", "DMRG_BIG_TBUDGET_MB": "16"},
    "auto": {},
    "off": {"DMRG_BIG": "0", "DMRG_BIG64": "0"},
    "target_route": {"DMRG_SPLIT_TASK_ROUTE": "0", "DMRG_LDS64": "0"},
    "copy_wave": {"DMRG_LDS_CW": "15", "DMRG_LDS_W6": "0"},
    "lds64_route": {"DMRG_LDS64_TASK_ROUTE": "1"},
    "lds64_route_forced": {"DMRG_LDS64_TASK_ROUTE": "1", "DMRG_BIG64": "2"},
}


def build(p, variant):
    h, eri, left, right, na, nb, site = p
    env = VARIANTS[variant]
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return Hop(h, eri, left, right, na, nb, site, device=0, want_split=True)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def run(hop, x, prec):
    xd = torch.as_tensor(x, device=DEV).contiguous()
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def block_slices(oh, targets):
    return [slice(oh.layout.blocks[j][4], oh.layout.blocks[j][4] + oh.layout.blocks[j][5] * oh.layout.blocks[j][6])
            for j in targets]


def check_sampled(hop, oh, x, ref, mag, targets, what):
    """Both precisions of the GPU H.psi on the sampled target blocks against the oracle."""
    sl = block_slices(oh, targets)
    r = np.concatenate([ref[s] for s in sl])
    m = np.concatenate([mag[s] for s in sl])
    for prec in (PREC_FP64, PREC_SPLIT2):
        y = run(hop, x, prec)
        got = np.concatenate([y[s] for s in sl])
        print(f"[{what}] prec {prec}: rel err {rel_err(got, r):.2e}", flush=True)
        if prec == PREC_FP64:
            assert rel_err(got, r) < FP64_TOL, (what, prec)
        else:
            assert_split_bound(got, r, m, what)


# ---------------------------------------------------------------- case A: every target, full oracle
@pytest.fixture(scope="module")
def case_a():
    # L = 14, M = 300: sectors up to 139 states (two 128-row tiles, the second ragged)
    p = synth(14, 300, 0.6, 5)
    print("[big A] L=14 M=300: oracle", flush=True)
    oh = OracleHop(*p)
    x = random_vector(oh.layout.size, 41)
    return p, oh, x, oh.apply(x), oh.magnitude(x)


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_case_a_matches_oracle(case_a, variant):
    p, oh, x, ref, mag = case_a
    print(f"[big A] variant {variant}", flush=True)
    hop = build(p, variant)
    y64 = run(hop, x, PREC_FP64)
    assert rel_err(y64, ref) < FP64_TOL, variant
    ysp = run(hop, x, PREC_SPLIT2)
    print(f"[big A] {variant}: fp64 {rel_err(y64, ref):.2e} split {rel_err(ysp, ref):.2e}", flush=True)
    assert_split_bound(ysp, ref, mag, f"big A {variant}")
    assert np.array_equal(run(hop, x, PREC_FP64), y64)
    assert np.array_equal(run(hop, x, PREC_SPLIT2), ysp)


def test_case_a_plans_agree(case_a):
    p, oh, x, ref, mag = case_a
    a, b = build(p, "forced"), build(p, "cut")
    assert rel_err(run(b, x, PREC_FP64), run(a, x, PREC_FP64)) < 1e-13
    assert rel_err(run(b, x, PREC_SPLIT2), run(a, x, PREC_SPLIT2)) < 2e-6


# ---------------------------------------------------------------- case B: sampled large targets
@pytest.fixture(scope="module")
def case_b():
    # L = 16, M = 1000, sigma = 0.35: 36 blocks, the largest 250 x 250 (rows 250 = 128 + 122)
    p = synth(16, 1000, 0.35, 7)
    print("[big B] L=16 M=1000: oracle", flush=True)
    oh = OracleHop(*p)
    bl = oh.layout.blocks
    big = [j for j in range(len(bl)) if max(bl[j][5], bl[j][6]) > 96]
    rng = np.random.default_rng(3)
    targets = sorted(set(sorted(big, key=lambda j: -bl[j][5] * bl[j][6])[:4]) |
                     set(rng.choice(big, size=min(3, len(big)), replace=False).tolist()))
    x = random_vector(oh.layout.size, 43)
    tasks = oh.target_tasks(targets)
    return p, oh, x, oh.apply(x, tasks=tasks), targets, oh.magnitude(x, tasks=tasks)


@pytest.mark.parametrize("variant", ["forced", "cut", "auto"])
def test_case_b_sampled_targets(case_b, variant):
    p, oh, x, ref, targets, mag = case_b
    print(f"[big B] variant {variant}, targets {targets}", flush=True)
    check_sampled(build(p, variant), oh, x, ref, mag, targets, f"big B {variant}")


def test_case_b_multivector_deterministic(case_b):
    p, oh, x, ref, targets, mag = case_b
    hop = build(p, "forced")
    X = np.stack([random_vector(hop.n_coeff, 50 + k) for k in range(5)])   # more vectors than one launch holds
    xd = torch.as_tensor(X, device=DEV).contiguous()
    for prec in (PREC_FP64, PREC_SPLIT2):
        y1, y2 = torch.empty_like(xd), torch.empty_like(xd)
        hop.hpsi(xd, y1, prec)
        hop.hpsi(xd, y2, prec)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2)
        for k in (0, 4):
            assert np.array_equal(y1[k].cpu().numpy(), run(hop, X[k], prec))


# ---------------------------------------------------------------- case C: the large shape's sector sizes
C_DIMS = {1: 420, 2: 97, 3: 33, 4: 5, 5: 1}     # by distance |n_alpha - 2.5| + |n_beta - 2.5| of the sector


@pytest.fixture(scope="module")
def case_c():
    L, na, nb, site = 12, 6, 6, 5
    h, eri = random_integrals(L, 44)
    dim_of = lambda a, b: C_DIMS[int(abs(a - 2.5) + abs(b - 2.5))]
    left = synthetic_block("left", L, na, nb, site, 4000, 3.0, 1044, dim_of=dim_of)
    right = synthetic_block("right", L, na, nb, site, 4000, 3.0, 2044, dim_of=dim_of)
    p = (h, eri, left, right, na, nb, site)
    print("[big C] L=12, 420-state sectors: oracle set-up", flush=True)
    oh = OracleHop(*p)
    bl = oh.layout.blocks
    order = sorted(range(len(bl)), key=lambda j: -bl[j][5] * bl[j][6])
    rng = np.random.default_rng(5)
    ragged = [j for j in range(len(bl)) if {bl[j][5], bl[j][6]} == {420, 97}]
    targets = sorted({order[0]} | set(rng.choice(ragged, size=1).tolist()) | {order[-1]})
    x = random_vector(oh.layout.size, 45)
    tasks = oh.target_tasks(targets)
    print(f"[big C] |psi| = {oh.layout.size}, targets {[(bl[j][5], bl[j][6]) for j in targets]}", flush=True)
    return p, oh, x, oh.apply(x, tasks=tasks), targets, oh.magnitude(x, tasks=tasks)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("variant", ["auto", "forced"])
def test_case_c_sampled_targets(case_c, variant):
    p, oh, x, ref, targets, mag = case_c
    check_sampled(build(p, variant), oh, x, ref, mag, targets, f"big C {variant}")
