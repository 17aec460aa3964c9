"""CPU FP64 oracle of the phase-field lattice Boltzmann step (test infrastructure).

This package is test infrastructure.  It is imported only by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product library never calls it, and it shares no code with the GPU path:
no kernels, tables, constant generators, or pre/post-processing.

It is a plain, slow, vectorised-over-the-grid rendering of the discrete
algorithm in float64 with ordinary PyTorch CPU tensor operations: one tensor
operation per term of each formula, no blocking or fusion, the MRT collision
done with explicit transformation matrices M, S, M^-1.

Modules
-------
lattice      velocity sets, weights, orthogonal moment bases (Appendix B)
asymptotics  thin-interface constants I, J, F, H, K, a1, a2 (Appendix A)
model        parameters, initial state, one time step, macros, diagnostics

Parity status of each function is stated in its docstring; a function whose
result no independent pin checks says "parity unpinned".
"""
from .lattice import Lattice, lattice  # noqa: F401
from .model import OracleParams, OracleSim  # noqa: F401
