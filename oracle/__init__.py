"""FP64 CPU oracle for the two-site QC-DMRG H.psi path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
anything from this package. The GPU library (``paper_2001_04890_amd``) never imports it and shares
no code with it; both read their inputs from the seeded generators in ``dmrg_inputs``.

Everything here is plain, slow and written for checkability against the paper
(Brabec et al., "Massively parallel quantum chemical DMRG", Section 2):

* :mod:`oracle.hamiltonian` -- spin-orbital integrals from Eq. H2q (reading: ``v_pqrs = (ps|qr)/2``).
* :mod:`oracle.fci`         -- brute-force determinant FCI (matvec and lowest eigenvalue).
* :mod:`oracle.fock`        -- exact block operators built in a block's full Fock space, and the
  embedding of a superblock vector into the determinant basis.
* :mod:`oracle.layout`      -- sector-decomposed wave-function layout (Eq. wf_sec and its constraints).
* :mod:`oracle.terms`       -- expansion of H into left-block x site x site x right-block operator
  combinations (the sum over alpha in the H.Phi equation of Section 2.2.1), with pre-summed
  left-block operators (Section 2.1 / 2.2.3).
* :mod:`oracle.hpsi`        -- the sector GEMMs of Eq. dgemm, and diag(H).
* :mod:`oracle.davidson`    -- Davidson's method for the lowest eigenpair.
* :mod:`oracle.renorm`      -- reduced density matrices, the M-state truncation and Eq. renorm_mat
  (the renormalization step that follows the Davidson solve; no GPU counterpart yet).
* :mod:`oracle.blocking`    -- operators of the grown left block (block + site) from the block's
  stored operators and the site matrices, and their renormalized block (no GPU counterpart yet).

Parity pins (see ``tests/test_oracle_*.py``): closed forms of tiny Hamiltonians, CAR relations,
brute-force FCI matvecs and energies with exact blocks, Hermiticity, particle-number/Sz
conservation, and dense diagonalisation of the explicit operator.
"""
