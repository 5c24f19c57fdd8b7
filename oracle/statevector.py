"""Dense state-vector simulation in complex128 (test infrastructure only).

This is explicit time evolution of |0...0> through the gate list: the plain
definition of <x|C|0>, and the naive scheme the paper compares against (its
cost bound T N 2^{2+N}, quoted beside side-wise contraction).  The state is a
(2,)*n array whose axis q is qubit q; gates are applied with tensordot on
their qubit axes, and amplitudes are read by tuple index, never by flat
integer, so no bit-order convention is involved.
"""
import numpy as np


def statevector(circ):
    n = circ.n
    if n > 28:
        raise ValueError("state vector limited to n <= 28 qubits")
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for g in circ.gates:
        if len(g.qubits) == 1:
            (q,) = g.qubits
            psi = np.tensordot(g.matrix, psi, axes=([1], [q]))
            psi = np.moveaxis(psi, 0, q)
        else:
            q1, q2 = g.qubits
            u = g.matrix.reshape(2, 2, 2, 2)        # [o1, o2, i1, i2]
            psi = np.tensordot(u, psi, axes=([2, 3], [q1, q2]))
            psi = np.moveaxis(psi, [0, 1], [q1, q2])
    return psi


def bits_of(word, n):
    return tuple((int(word) >> q) & 1 for q in range(n))


def statevector_amplitudes(circ, words, psi=None):
    """<x|C|0> for each packed bitstring (bit q of the word = x_q)."""
    if psi is None:
        psi = statevector(circ)
    return np.array([psi[bits_of(w, circ.n)] for w in words], dtype=np.complex128)
