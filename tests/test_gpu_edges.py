"""GPU edge cases of H.psi and Davidson through the C-ABI, against the oracle.

* Edge bonds: the bond (0, 1) leaves the left block without orbitals (vacuum only, one sector of
  dimension 1), the bond (L-2, L-1) the right block, and L = 2 both; every psi block is then as thin
  as a site pair. Exact blocks, so the oracle is the FCI matvec (pinned on the CPU) and Davidson must
  reach the FCI ground-state energy.
* Sector sizes on every kernel boundary: synthetic blocks whose sector dimensions cycle through
  1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 95, 96, 97, 128, 129 (one-tile sources for the task-mode
  kernel, 64- and 96-wide LDS classes and their edges, the large-block path with ragged 128-row tiles).
* Degenerate inputs: x = 0 gives y = 0 exactly; unit vectors give columns of H; nvec = 0 is an
  argument error.
Bars: FP64 within 1e-12 of max|y|, split within its error bound (helpers.assert_split_bound); energies within 1e-10 (FP64).
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals, random_vector
from dmrg_inputs.synthetic import synthetic_block
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
BOUNDARY = (1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 95, 96, 97, 128, 129)


def run(hop, x, prec=PREC_FP64):
    xd = torch.as_tensor(x, device=DEV).contiguous()
    yd = torch.empty_like(xd)
    hop.hpsi(xd, yd, prec)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


EDGE = {"L4_left_empty": (4, 0, 2, 2), "L6_right_empty": (6, 4, 3, 3), "L5_left_empty_odd": (5, 0, 3, 2),
        "L2_both_empty": (2, 0, 1, 1)}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_bond_matches_oracle_and_fci(name):
    L, site, na, nb = EDGE[name]
    print(f"[edges] {name}", flush=True)
    p = exact_problem(L, 3, n_alpha=na, n_beta=nb, site=site)
    h, eri, left, right, na, nb, site = p
    hop = Hop(*p, device=0, want_split=True)
    oh = OracleHop(*p)
    x = random_vector(hop.n_coeff, 8)
    ref = oh.apply(x)
    assert rel_err(run(hop, x), ref) < 1e-12
    assert_split_bound(run(hop, x, PREC_SPLIT2), ref, oh.magnitude(x), name)
    e_fci, _ = FCI(h, eri, na, nb).ground_state()
    psi = torch.as_tensor(random_vector(hop.n_coeff, 0), device=DEV)
    r = hop.davidson(psi, tol=1e-10, max_iter=200, max_sub=min(24, max(2, hop.n_coeff)))
    print(f"[edges] {name}: E={r['energy']:.12f} FCI={e_fci:.12f} iters={r['iters']}", flush=True)
    assert r["converged"] and abs(r["energy"] - e_fci) < 1e-10


@pytest.fixture(scope="module")
def boundary():
    L, na, nb, site = 10, 5, 5, 4
    h, eri = random_integrals(L, 21)

    def dim_of(a, b):
        return BOUNDARY[(3 * a + 7 * b) % len(BOUNDARY)]

    left = synthetic_block("left", L, na, nb, site, 1000, 1.0, 1021, dim_of=dim_of)
    right = synthetic_block("right", L, na, nb, site, 1000, 1.0, 2021, dim_of=lambda a, b: dim_of(b, a))
    p = (h, eri, left, right, na, nb, site)
    print(f"[edges] boundary dims: left {sorted(set(left.dim.tolist()))}", flush=True)
    hop = Hop(*p, device=0, want_split=True)
    oh = OracleHop(*p)
    return p, hop, oh


def test_boundary_dims_match_oracle(boundary):
    p, hop, oh = boundary
    x = random_vector(hop.n_coeff, 9)
    ref = oh.apply(x)
    y64 = run(hop, x)
    ysp = run(hop, x, PREC_SPLIT2)
    print(f"[edges] boundary: n={hop.n_coeff} fp64 {rel_err(y64, ref):.2e} split {rel_err(ysp, ref):.2e}", flush=True)
    assert rel_err(y64, ref) < 1e-12
    assert_split_bound(ysp, ref, oh.magnitude(x), "boundary dims")
    assert np.array_equal(run(hop, x), y64) and np.array_equal(run(hop, x, PREC_SPLIT2), ysp)
    d = torch.empty(hop.n_coeff, dtype=torch.float64, device=DEV)
    hop.diagonal(d)
    torch.cuda.synchronize()
    assert rel_err(d.cpu().numpy(), oh.diagonal()) < 1e-12


def test_zero_and_unit_vectors(boundary):
    p, hop, oh = boundary
    z = np.zeros(hop.n_coeff)
    for prec in (PREC_FP64, PREC_SPLIT2):
        assert not np.any(run(hop, z, prec))
    rng = np.random.default_rng(4)
    offs = np.array([b[4] for b in oh.layout.blocks])
    for i in [0, hop.n_coeff - 1] + rng.choice(hop.n_coeff, size=3, replace=False).tolist():
        e = np.zeros(hop.n_coeff)
        e[i] = 1.0
        src = int(np.searchsorted(offs, i, side="right") - 1)          # block holding coefficient i
        ref = oh.apply(e, tasks=[tk for tk in oh.tasks() if tk[0] == src])
        assert rel_err(run(hop, e), ref) < 1e-12, i


def test_nvec_zero_is_an_argument_error(boundary):
    p, hop, oh = boundary
    x = torch.zeros((0, hop.n_coeff), dtype=torch.float64, device=DEV)
    y = torch.zeros((0, hop.n_coeff), dtype=torch.float64, device=DEV)
    with pytest.raises(lib_mod.DmrgError) as e:
        hop.hpsi(x, y)
    assert e.value.status == -1
