"""GPU parity of the FP64 LDS-staged H.psi kernel (hpsi_lds64.hip: targets whose own and source blocks
fit the 96-wide stages) against the FP64 oracle, through the C-ABI.

Problem 1: L = 14, M = 200, sigma = 0.6 (100 blocks, sectors of 1 .. 95 states): every target fits
the 96 x 96 workgroup tile, targets of up to 3 and of 4 .. 6 column tiles, and most targets have
sources of both k-tile bounds (at most 32 rows, and more), so their task lists run in two launch
classes. Plan variants: the default; "cut" (cost bound at its floor: every long task list cut into
many items whose partial tiles a reduction adds, including targets with items in both classes,
which share one reduction record); "whole" (few, long items); by
default tasks whose source is a single 32 x 32 tile run in the one-wavefront kernel next to the
LDS-staged ones of the same target, "small" (and "cut", "whole") put them in the LDS kernel too;
the kernel switched off (every target on the one-wavefront kernel); and without the copy wavefront
(every wavefront issues a share of the LDS copies), cut to its floor; the classes of sources with
at most 32 rows stage their copies one step ahead in two LDS slots by default ("two_slots"), two
steps ahead in three with DMRG_LDS64_NS3=1 ("three_slots_cut": with many short items). The plan
trace names the
launch classes and reductions each variant produced, so the test checks that the paths it means to
cover were taken. Bars: FP64 within 1e-12 of max|y| against the oracle on every element, plans
within 1e-13 of each other, every plan deterministic bit for bit.

Problem 2: L = 14, M = 240, sigma = 0.6 (sectors up to 111 states: seven row and column tiles, the
last one ragged) for the 7-wavefront class, which takes every target with a dimension above 96 (and
the tasks of other targets whose source has more than 96 rows); held to 128 VGPRs (two workgroups per
CU, the default), without that cap, and cut into many items.
"""
import os
import re

import numpy as np
import pytest

from dmrg_inputs import random_vector
from oracle.hpsi import OracleHop
from helpers import rel_err, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64 = lib_mod.Hop, lib_mod.PREC_FP64

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
FP64_TOL = 1e-12
VARIANTS = {
    "default": {},
    "small": {"DMRG_LDS64_SMALL": "1"},
    "cut": {"DMRG_LDS64_ITEMS": "100000000", "DMRG_LDS64_SMALL": "1"},
    "whole": {"DMRG_LDS64_ITEMS": "64", "DMRG_LDS64_SMALL": "1"},
    "off": {"DMRG_LDS64": "0"},
    "no_copy_wave": {"DMRG_LDS64_CW": "0", "DMRG_LDS64_ITEMS": "100000000"},
    "two_slots": {"DMRG_LDS64_NS3": "0", "DMRG_LDS64_SMALL": "1"},
    "three_slots_cut": {"DMRG_LDS64_NS3": "1", "DMRG_LDS64_ITEMS": "100000000", "DMRG_LDS64_SMALL": "1"},
}
TRACE = re.compile(r"\[dmrg lds64 plan\] items (\d+) classes (\d+) (\d+) (\d+) (\d+) (\d+) reduces (\d+)")


@pytest.fixture(scope="module")
def problem():
    p = synth(14, 200, 0.6, 5)
    print("[lds64] L=14 M=200: oracle", flush=True)
    oh = OracleHop(*p)
    x = random_vector(oh.layout.size, 61)
    return p, x, oh.apply(x)


def build(p, variant, capfd, variants=VARIANTS):
    h, eri, left, right, na, nb, site = p
    env = dict(variants[variant], DMRG_PLAN_TRACE="1")
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        capfd.readouterr()
        hop = Hop(h, eri, left, right, na, nb, site, device=0)
        err = capfd.readouterr().err
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    m = TRACE.findall(err)
    plan = [int(v) for v in m[-1]] if m else None
    print(f"[lds64] {variant}: plan {plan}", flush=True)
    return hop, plan


def run(hop, x):
    xd = torch.as_tensor(x, device=DEV).contiguous()
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, PREC_FP64)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_lds64_matches_oracle(problem, variant, capfd):
    p, x, ref = problem
    hop, plan = build(p, variant, capfd)
    if variant == "off":
        assert plan is None
    else:
        items, k2q3, k2q6, k6q3, k6q6, k7, reduces = plan
        assert k7 == 0
        assert items > 0
        if variant != "default":
            assert k2q3 + k2q6 > 0 and k6q3 + k6q6 > 0, "sources of both k-tile bounds"
            assert k2q3 + k6q3 > 0 and k2q6 + k6q6 > 0, "narrow and wide targets"
        if variant == "cut":
            assert reduces > 0 and items > 4 * reduces
    y = run(hop, x)
    err = rel_err(y, ref)
    print(f"[lds64] {variant}: rel err {err:.2e}", flush=True)
    assert err < FP64_TOL, variant
    assert np.array_equal(run(hop, x), y), "deterministic"


def test_lds64_plans_agree(problem, capfd):
    p, x, ref = problem
    ys = {v: run(build(p, v, capfd)[0], x) for v in ("cut", "whole", "off")}
    assert rel_err(ys["cut"], ys["whole"]) < 1e-13
    assert rel_err(ys["cut"], ys["off"]) < 1e-13


VARIANTS7 = {
    "default": {},
    "w7_uncapped": {"DMRG_LDS64_W7": "0"},
    "cut": {"DMRG_LDS64_ITEMS": "100000000"},
    "no_copy_wave": {"DMRG_LDS64_CW": "0"},
}


@pytest.fixture(scope="module")
def problem112():
    p = synth(14, 240, 0.6, 5)
    print("[lds64] L=14 M=240: oracle", flush=True)
    oh = OracleHop(*p)
    x = random_vector(oh.layout.size, 62)
    return p, x, oh.apply(x)


@pytest.mark.parametrize("variant", sorted(VARIANTS7))
def test_lds64_seven_tile_class_matches_oracle(problem112, variant, capfd):
    p, x, ref = problem112
    hop, plan = build(p, variant, capfd, VARIANTS7)
    items, k2q3, k2q6, k6q3, k6q6, k7, reduces = plan
    assert k7 > 0, "7-wavefront class"
    if variant == "cut":
        assert reduces > 0
    y = run(hop, x)
    err = rel_err(y, ref)
    print(f"[lds64] 112 {variant}: rel err {err:.2e}", flush=True)
    assert err < FP64_TOL, variant
    assert np.array_equal(run(hop, x), y), "deterministic"
