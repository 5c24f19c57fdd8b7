"""CPU oracle for circuit amplitudes <x|C|0^n> in complex128.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the plan builder) imports, calls or links anything here; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
The oracle shares no code with the GPU path: it builds its own tensor network
from the circuit's gate list, with its own labelling, and contracts it with
plain numpy operations in float64/complex128.

Contents
  statevector  dense state-vector simulation (explicit time evolution, the
               naive scheme whose cost the paper bounds by T N 2^{2+N})
  pairwise     naive pairwise tensor-network contraction (each step costs
               the product of the dimensions of the union of both operands'
               indices, Eq. (3)), with its own greedy order or with an order
               and index slicing imported as data
  iqp          closed form for H-diagonal-H (IQP) circuits
  doubled      the paper's expectation value <0|U^dag (x) P_i U|0> as a
               doubled network of U and U^dag

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: agreement of the two independent definitions, unitarity, closed forms,
order and slicing invariance, mirror circuits and stabilizer magnitudes.
"""
from .statevector import statevector, statevector_amplitudes
from .pairwise import (OracleNetwork, pairwise_amplitudes, pairwise_amplitude,
                       contract_pair)
from .iqp import iqp_amplitudes_bruteforce, iqp_amplitudes_transfer
from .doubled import doubled_expectation

__all__ = ["statevector", "statevector_amplitudes", "OracleNetwork",
           "pairwise_amplitudes", "pairwise_amplitude",
           "contract_pair", "iqp_amplitudes_bruteforce",
           "iqp_amplitudes_transfer", "doubled_expectation"]
