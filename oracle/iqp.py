"""Closed form for IQP circuits H^n D H^n (test infrastructure only).

For a circuit that applies H to every qubit, then only diagonal gates, then H
to every qubit, the amplitude is

    a(x) = 2^{-n} sum_z (-1)^{x.z} prod_g d_g(z restricted to g's qubits),

since H^n|0> is the uniform superposition, each diagonal gate multiplies |z>
by its diagonal entry, and <x|H^n|z> = 2^{-n/2} (-1)^{x.z}.  The phase-gate
family of the paper's IQP example is of this kind (diagonal one- and
two-qubit phase gates between Hadamard layers).

Two evaluations of that sum: brute force over all z (n <= 22), and, for a
rows x cols grid whose two-qubit gates span at most two columns, a transfer
matrix over pairs of neighbouring columns (2^{3*rows} entries per column).
"""
import numpy as np

_H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def _split_iqp(circ):
    n = circ.n
    first = {}
    last = {}
    for gi, g in enumerate(circ.gates):
        for q in g.qubits:
            first.setdefault(q, gi)
            last[q] = gi
    if len(first) != n:
        raise ValueError("every qubit needs gates in an IQP circuit")
    diag = []
    for gi, g in enumerate(circ.gates):
        if len(g.qubits) == 1 and (first[g.qubits[0]] == gi or last[g.qubits[0]] == gi):
            if not np.allclose(g.matrix, _H, atol=1e-15, rtol=0):
                raise ValueError("IQP circuit must start and end with H on every qubit")
            continue
        m = g.matrix
        if np.count_nonzero(m - np.diag(np.diag(m))):
            raise ValueError("gate %d between the H layers is not diagonal" % gi)
        diag.append((g.qubits, np.diag(m).copy()))
    return diag


def iqp_amplitudes_bruteforce(circ, words):
    n = circ.n
    if n > 22:
        raise ValueError("brute force limited to n <= 22")
    diag = _split_iqp(circ)
    z = np.arange(1 << n, dtype=np.int64)
    bit = [((z >> q) & 1) for q in range(n)]
    w = np.ones(1 << n, dtype=np.complex128)
    for qs, d in diag:
        if len(qs) == 1:
            w *= d[bit[qs[0]]]
        else:
            w *= d[2 * bit[qs[0]] + bit[qs[1]]]
    out = []
    for x in words:
        par = np.zeros(1 << n, dtype=np.int64)
        for q in range(n):
            if (int(x) >> q) & 1:
                par ^= bit[q]
        sign = 1.0 - 2.0 * par
        out.append(np.sum(sign * w) / float(1 << n))
    return np.array(out, dtype=np.complex128)


def iqp_amplitudes_transfer(circ, words):
    """Transfer matrix over columns of a rows x cols grid, q = r*cols + c."""
    pos = circ.positions
    R = int(pos[:, 0].max()) + 1
    C = int(pos[:, 1].max()) + 1
    n = circ.n
    for q in range(n):
        if int(pos[q, 0]) * C + int(pos[q, 1]) != q:
            raise ValueError("qubits must be numbered row-major")
    diag = _split_iqp(circ)
    S = 1 << R
    # broadcast grids over (s_{c-2}, s_{c-1}, s_c)
    g2 = np.arange(S).reshape(S, 1, 1)
    g1 = np.arange(S).reshape(1, S, 1)
    g0 = np.arange(S).reshape(1, 1, S)
    grids = {2: g2, 1: g1, 0: g0}
    G = [np.ones((S, S, S), dtype=np.complex128) for _ in range(C)]
    for qs, d in diag:
        cols = [q % C for q in qs]
        cmax = max(cols)
        offs = [cmax - c for c in cols]
        if max(offs) > 2:
            raise ValueError("gate spans more than three columns")
        bits = [(grids[o] >> (q // C)) & 1 for q, o in zip(qs, offs)]
        if len(qs) == 1:
            G[cmax] = G[cmax] * d[bits[0]]
        else:
            G[cmax] = G[cmax] * d[2 * bits[0] + bits[1]]
    popc = np.array([bin(s).count("1") & 1 for s in range(S)])
    out = []
    for x in words:
        V = np.zeros((S, S), dtype=np.complex128)
        V[0, 0] = 1.0          # two virtual all-zero columns before column 0
        for c in range(C):
            xc = 0
            for r in range(R):
                xc |= ((int(x) >> (r * C + c)) & 1) << r
            sign = 1.0 - 2.0 * popc[np.arange(S) & xc]
            F = G[c] * sign.reshape(1, 1, S)
            if c == 0:
                F = np.where((g2 == 0) & (g1 == 0), F, 0)
            elif c == 1:
                F = np.where(g2 == 0, F, 0)
            V = np.einsum("ab,abc->bc", V, F)
        out.append(V.sum() / float(1 << n))
    return np.array(out, dtype=np.complex128)
