"""Seeded synthetic inputs shared by the FP64 oracle and the HIP library's tests/benchmarks.

This package only draws random numbers and holds plain data containers. It carries none of
the DMRG arithmetic (no operator algebra, no Hamiltonian terms, no contractions), so that the
oracle (``oracle/``) and the GPU path (``paper_2001_04890_amd``) stay independent of each other.

* :mod:`dmrg_inputs.integrals` -- random-integral Hamiltonians (one- and two-electron integrals).
* :mod:`dmrg_inputs.blocks`    -- the block-operator container (sector table + dense sector blocks).
* :mod:`dmrg_inputs.synthetic` -- seeded synthetic block operators with prescribed sector sizes.
"""
from .integrals import random_integrals, random_vector
from .blocks import Block, Op, OP_KINDS

__all__ = ["random_integrals", "random_vector", "Block", "Op", "OP_KINDS"]
