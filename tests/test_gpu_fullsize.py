"""Full-size GPU parity: the benchmark's H.psi workloads at L = 24, N = 24 (12, 12), M = 1024, middle
bond, built and launched exactly as bench.py times them (eager dmrg_hpsi on the caller's stream, and
the captured graph), checked on sampled output blocks that the oracle computes target by target:

* swept (the default workload): the blocks that two sweeps over random integrals (seed 1, M 256 then
  1024, split precision with an FP64 polish, tolerance 1e-5) leave at the bond (11, 12); sectors up
  to 107 states, so the FP64 LDS kernel's 7-wavefront class and the split two-pass path run;
* synthetic: sector sizes from the sigma = 1.5 model, random operator values (844 psi blocks).

Sample: the three largest blocks, the smallest, and four seeded random blocks. Bars: FP64 within
1e-12 of the sample's max|y|, split element by element within its error bound
(helpers.assert_split_bound); graph replays equal the eager launch bit for bit.
"""
import numpy as np
import pytest

from dmrg_inputs import random_vector
from dmrg_inputs.synthetic import synthetic_problem
from oracle.hpsi import OracleHop
from helpers import assert_split_bound, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")
Hop, PREC_FP64, PREC_SPLIT2 = lib_mod.Hop, lib_mod.PREC_FP64, lib_mod.PREC_SPLIT2

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
L, NA, NB, M, SIGMA, SEED = 24, 12, 12, 1024, 1.5, 1


def swept_problem():
    """The bench's default operators (bench.py swept_problem with its default options)."""
    from dmrg_inputs import random_integrals
    h, eri = random_integrals(L, SEED)
    site = L // 2 - 1
    r = lib_mod.sweep(h, eri, NA, NB, [256, 1024], m_warmup=256, tol=1e-5, max_iter=400, max_sub=24,
                      precision=PREC_SPLIT2, fp64_polish=True, split_tol=3e-4, seed=SEED, keep_site=site)
    print(f"[full] swept: {r['seconds']:.1f}s, E {r['energy']:.10f}, kept {r['left'].dim.sum()} x "
          f"{r['right'].dim.sum()}, largest sectors {r['left'].dim.max()} / {r['right'].dim.max()}", flush=True)
    return h, eri, r["left"], r["right"], site


@pytest.fixture(scope="module", params=["swept", "synthetic"])
def full(request):
    if request.param == "swept":
        print(f"[full] L={L} M={M}: sweeping", flush=True)
        h, eri, left, right, site = swept_problem()
    else:
        h, eri, left, right, site = synthetic_problem(L, NA, NB, M, SIGMA, SEED)
    print(f"[full] L={L} M={M} {request.param}: building the GPU operator", flush=True)
    stream = torch.cuda.current_stream()
    hop = Hop(h, eri, left, right, NA, NB, site, device=0, want_split=True, stream=stream)
    x = random_vector(hop.n_coeff, 7)
    print("[full] oracle set-up (pre-summed operators of every combination)", flush=True)
    oh = OracleHop(h, eri, left, right, NA, NB, site)
    bl = oh.layout.blocks
    order = sorted(range(len(bl)), key=lambda j: -bl[j][5] * bl[j][6])
    rng = np.random.default_rng(11)
    targets = sorted(set(order[:3]) | {order[-1]} | set(rng.choice(len(bl), size=4, replace=False).tolist()))
    print(f"[full] oracle on targets {targets}", flush=True)
    tasks = oh.target_tasks(targets)
    ref = oh.apply(x, tasks=tasks)
    mag = oh.magnitude(x, tasks=tasks)
    sl = [slice(bl[j][4], bl[j][4] + bl[j][5] * bl[j][6]) for j in targets]
    return hop, stream, x, np.concatenate([ref[s] for s in sl]), sl, np.concatenate([mag[s] for s in sl])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [PREC_FP64, PREC_SPLIT2])
def test_full_size_sampled_blocks(full, prec):
    hop, stream, x, ref, sl, mag = full
    xd = torch.as_tensor(x, device=DEV)
    y = torch.empty_like(xd)
    hop.hpsi(xd, y, prec, stream=stream)
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    got = np.concatenate([yh[s] for s in sl])
    err = rel_err(got, ref)
    print(f"[full] prec {prec}: sampled rel err {err:.2e}", flush=True)
    if prec == PREC_FP64:
        assert err < 1e-12
    else:
        assert_split_bound(got, ref, mag, "full size")
    yg = torch.empty_like(xd)
    for _ in range(2):
        yg.fill_(float("nan"))
        hop.hpsi_graph(xd, yg, prec, stream=stream)
        torch.cuda.synchronize()
        assert torch.equal(yg, y)
