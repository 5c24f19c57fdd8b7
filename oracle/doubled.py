"""The paper's quantity c = <0|U^dag (x)_i P_i U|0> (test infrastructure only).

The paper states its simulation problem as the expectation value of a product
of single-qubit projectors, written as one tensor network of U, the P_i and
U^dag.  Read as a circuit, that network is U, then every P_i, then U^dag,
closed by <0| on the output, so it is an amplitude of a (non-unitary) gate
list and the pairwise evaluator computes it directly.  With P_i = |x_i><x_i|
it equals |<x|U|0>|^2, with P_i = 1 it equals 1.
"""
import numpy as np

from circuits.model import Circuit, Gate
from .pairwise import pairwise_amplitude
from .statevector import statevector


def doubled_circuit(circ, projectors):
    gates = list(circ.gates)
    for q, P in enumerate(projectors):
        gates.append(Gate((q,), np.asarray(P, dtype=np.complex128), "P"))
    gates += [Gate(g.qubits, g.matrix.conj().T.copy(), g.name + "_dg")
              for g in reversed(circ.gates)]
    return Circuit(circ.n, gates, circ.positions.copy(), circ.name + "_doubled")


def doubled_expectation(circ, projectors, method="pairwise"):
    """c for one projector (2x2 array) per qubit."""
    d = doubled_circuit(circ, projectors)
    if method == "pairwise":
        return pairwise_amplitude(d, 0)
    psi = statevector(circ)
    phi = psi
    for q, P in enumerate(projectors):
        phi = np.moveaxis(np.tensordot(np.asarray(P), phi, axes=([1], [q])), 0, q)
    return complex(np.vdot(psi, phi))
