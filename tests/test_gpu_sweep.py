"""GPU two-site DMRG sweeps (dmrg_sweep: warm-up, forward and backward sweeps; Section 2.1) against
brute-force FCI (the oracle's determinant CI from the same integrals).

* Full M (no nonzero weight can be discarded: M exceeds the Schmidt rank at every cut), L = 8 and
  L = 10: every solve of the last sweep equals E_FCI within 1e-8 (Davidson tolerance 1e-9).
* Truncated M at L = 8 (M = 6, 12, 24): the final energy is variational (>= E_FCI), decreases with M,
  and the last sweep does not end above the first one.
"""
import numpy as np
import pytest

from dmrg_inputs import random_integrals
from oracle.fci import FCI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(scope="module")
def l8():
    h, eri = random_integrals(8, 0)
    return h, eri, FCI(h, eri, 4, 4).ground_state()[0]


@pytest.mark.parametrize("L,M", [(8, 256), (10, 1024)])
def test_full_m_sweeps_reach_fci(L, M):
    h, eri = random_integrals(L, 0)
    e_fci = FCI(h, eri, L // 2, L // 2).ground_state()[0]
    print(f"[sweep] L={L} M={M}: FCI {e_fci:.12f}", flush=True)
    r = lib_mod.sweep(h, eri, L // 2, L // 2, [M, M], m_warmup=M, tol=1e-9, max_iter=500, seed=1)
    last = r["energies"][-(2 * L - 4):]
    print(f"[sweep] L={L}: {len(r['energies'])} solves in {r['seconds']:.1f}s, last sweep "
          f"max |E - E_FCI| {np.abs(last - e_fci).max():.2e}", flush=True)
    assert r["converged"]
    assert np.abs(last - e_fci).max() < 1e-8
    assert np.all(r["discarded"][-(2 * L - 4):] < 1e-12)


def test_truncated_sweeps_are_variational_and_monotone_in_m(l8):
    h, eri, e_fci = l8
    finals = []
    for M in (6, 12, 24):
        r = lib_mod.sweep(h, eri, 4, 4, [M, M, M], m_warmup=M, tol=1e-9, max_iter=500, seed=2)
        e = r["energies"]
        per = len(e) // 3
        print(f"[sweep] L=8 M={M}: final {r['energy']:.10f} best {r['best_energy']:.10f} FCI {e_fci:.10f}, "
              f"max discarded {r['discarded'].max():.2e}", flush=True)
        assert np.all(e >= e_fci - 1e-10)
        assert r["best_energy"] <= e[:per].min() + 1e-10
        finals.append(r["best_energy"])
    assert finals[0] >= finals[1] - 1e-9 >= finals[2] - 2e-9
    assert finals[0] > e_fci + 1e-6
