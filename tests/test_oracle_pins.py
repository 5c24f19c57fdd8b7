"""Pins for the CPU oracle: each check ties it to something other than
itself (closed forms, unitarity, two independent definitions, identities).
"""
import itertools

import numpy as np
import pytest

from circuits import (lattice_circuit, iqp_lattice_circuit, stack3d_circuit,
                      product_circuit, mirror, random_bitstrings, make_config,
                      paper_iqp_circuit, sycamore_type_circuit, Circuit, Gate, haar_su2, haar_su4,
                      SQRT_X, SQRT_Y, SQRT_W, H, CZ, fsim, cphase, z_phase)
from circuits.families import serving_pool
from oracle import (statevector, statevector_amplitudes, pairwise_amplitudes,
                    pairwise_amplitude, iqp_amplitudes_bruteforce,
                    iqp_amplitudes_transfer, doubled_expectation)
from oracle.pairwise import OracleNetwork


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _all_small_circuits():
    return [
        lattice_circuit(3, 3, 4, 11, "sqrt", "cz"),
        lattice_circuit(3, 3, 4, 12, "sqrt", "fsim"),
        lattice_circuit(2, 4, 5, 13, "haar", "cz"),
        lattice_circuit(3, 4, 3, 14, "clifford", "cz"),
        iqp_lattice_circuit(3, 3, 15),
        stack3d_circuit(2, 2, 3, 5, 16),
        paper_iqp_circuit(3, 4, 17),
        sycamore_type_circuit(3, 2, 0.3, 18),
    ]


def test_gate_unitarity_all_generators():
    rng = np.random.Generator(np.random.PCG64(1))
    mats = [SQRT_X, SQRT_Y, SQRT_W, H, CZ, fsim(np.pi / 2, np.pi / 6),
            cphase(1.234), z_phase(0.77)]
    mats += [haar_su2(rng) for _ in range(50)] + [haar_su4(rng) for _ in range(50)]
    for name in ("cfg1", "cfg2", "cfg3", "cfg4"):
        c, _, _ = make_config(name)
        mats += [g.matrix for g in c.gates]
    for _, c, _ in serving_pool():
        mats += [g.matrix for g in c.gates]
    for m in mats:
        assert np.max(np.abs(m.conj().T @ m - np.eye(m.shape[0]))) <= 1e-14
    for m in [haar_su2(rng) for _ in range(10)] + [haar_su4(rng) for _ in range(10)]:
        assert abs(np.linalg.det(m) - 1) < 1e-12


def test_single_qubit_closed_forms_fix_orientation():
    # <1| sqrtY |0> = +1/sqrt2 fixes the row/column orientation of 1q gates
    c = Circuit(1, [Gate((0,), SQRT_Y.copy())], np.zeros((1, 2)))
    assert abs(pairwise_amplitude(c, 1) - 1 / np.sqrt(2)) < 1e-15
    assert abs(statevector_amplitudes(c, [1])[0] - 1 / np.sqrt(2)) < 1e-15
    c = Circuit(1, [Gate((0,), SQRT_W.copy())], np.zeros((1, 2)))
    want = np.exp(-1j * np.pi / 4) / np.sqrt(2)
    assert abs(pairwise_amplitude(c, 1) - want) < 1e-15


def test_two_qubit_index_convention_and_bit_order():
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    pos = np.zeros((4, 2))
    # X on qubit 2, CNOT(control 2, target 0): final |x> has bits 0 and 2 set
    c = Circuit(4, [Gate((2,), X), Gate((2, 0), CNOT)], pos)
    for f in (lambda w: statevector_amplitudes(c, [w])[0],
              lambda w: pairwise_amplitude(c, w),
              lambda w: pairwise_amplitude(c, w, diagonal_hyperedges=False)):
        assert abs(f(0b0101) - 1) < 1e-15
        assert abs(f(0b0100)) < 1e-15
        assert abs(f(0b0001)) < 1e-15
    # GHZ on 3 qubits
    g = Circuit(3, [Gate((0,), H.copy()), Gate((0, 1), CNOT), Gate((1, 2), CNOT)],
                np.zeros((3, 2)))
    amps = pairwise_amplitudes(g, list(range(8)))
    want = np.zeros(8)
    want[0] = want[7] = 1 / np.sqrt(2)
    assert np.max(np.abs(amps - want)) < 1e-15


@pytest.mark.parametrize("idx", range(8))
def test_statevector_equals_pairwise(idx):
    c = _all_small_circuits()[idx]
    words = random_bitstrings(c.n, 6, 100 + idx)
    sv = statevector_amplitudes(c, words)
    for dh in (True, False):
        pw = pairwise_amplitudes(c, words, diagonal_hyperedges=dh)
        assert _rel(pw, sv) <= 1e-12


def test_normalisation_over_all_bitstrings():
    c = lattice_circuit(2, 3, 5, 21, "haar", "cz")
    words = list(range(1 << c.n))
    pw = pairwise_amplitudes(c, words)
    assert abs(np.sum(np.abs(pw) ** 2) - 1) <= 1e-12
    psi = statevector(lattice_circuit(4, 4, 8, 22, "sqrt", "fsim"))
    assert abs(np.sum(np.abs(psi) ** 2) - 1) <= 1e-12


def _random_order(circ, word, rng):
    net = OracleNetwork(circ, word)
    tags = sorted(set(t for _, _, t in net.pieces))
    leaves = [[t] for t in tags]
    lab = {}
    for a, l, t in net.pieces:
        lab.setdefault(t, set()).update(l)
    live = {i: set(lab[t]) for i, t in enumerate(tags)}
    steps = []
    nid = len(leaves)
    while len(live) > 1:
        ids = list(live)
        pairs = [(a, b) for a, b in itertools.combinations(ids, 2) if live[a] & live[b]]
        if not pairs:
            pairs = list(itertools.combinations(ids, 2))
        a, b = pairs[int(rng.integers(len(pairs)))]
        steps.append([a, b])
        live[nid] = live.pop(a) | live.pop(b)
        nid += 1
    return {"leaves": leaves, "steps": steps}


def test_order_invariance():
    rng = np.random.Generator(np.random.PCG64(5))
    for c in (lattice_circuit(3, 3, 4, 31, "haar", "cz"),
              lattice_circuit(3, 3, 3, 32, "sqrt", "fsim")):
        w = int(random_bitstrings(c.n, 1, 33)[0])
        ref = pairwise_amplitude(c, w)
        for _ in range(5):
            order = _random_order(c, w, rng)
            assert abs(pairwise_amplitude(c, w, order=order) - ref) <= 1e-12 * abs(ref)


def test_slicing_invariance():
    c = lattice_circuit(3, 3, 5, 41, "haar", "cz")
    w = int(random_bitstrings(c.n, 1, 42)[0])
    ref = pairwise_amplitude(c, w)
    # wires after the 1q gates of cycle 1 on qubits 0, 4, 8
    specs = []
    for gi, g in enumerate(c.gates):
        if len(g.qubits) == 1 and gi >= c.n and g.qubits[0] in (0, 4, 8) and len(specs) < 3:
            specs.append((g.qubits[0], gi))
    got = pairwise_amplitude(c, w, sliced=specs)
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_product_circuit_64_qubits():
    c = product_circuit(64, 3, 51)
    words = random_bitstrings(64, 4, 52)
    pw = pairwise_amplitudes(c, words)
    for w, a in zip(words, pw):
        want = 1.0 + 0j
        for q in range(64):
            U = np.eye(2, dtype=complex)
            for g in c.gates:
                if g.qubits == (q,):
                    U = g.matrix @ U
            want *= U[(int(w) >> q) & 1, 0]
        assert abs(a - want) <= 1e-13 * abs(want)


def test_iqp_closed_forms():
    c = iqp_lattice_circuit(3, 4, 61)
    words = random_bitstrings(c.n, 8, 62)
    sv = statevector_amplitudes(c, words)
    assert _rel(iqp_amplitudes_bruteforce(c, words), sv) <= 1e-12
    assert _rel(iqp_amplitudes_transfer(c, words), sv) <= 1e-12
    c = iqp_lattice_circuit(4, 5, 63)
    words = random_bitstrings(c.n, 4, 64)
    assert _rel(iqp_amplitudes_transfer(c, words), iqp_amplitudes_bruteforce(c, words)) <= 1e-12


def test_mirror_circuit_identity():
    m = mirror(lattice_circuit(3, 3, 4, 71, "haar", "cz"))
    words = [0, 1, 6, 511]
    for amps in (statevector_amplitudes(m, words), pairwise_amplitudes(m, words)):
        assert abs(amps[0] - 1) <= 1e-12
        assert np.max(np.abs(amps[1:])) <= 1e-12


def test_clifford_magnitudes():
    c = lattice_circuit(3, 4, 5, 81, "clifford", "cz")
    psi = statevector(c)
    p = np.abs(psi.ravel()) ** 2
    nz = p[p > 1e-12]
    k = -np.log2(nz)
    assert np.max(np.abs(k - np.round(k))) <= 1e-9
    assert len(set(np.round(k).astype(int))) == 1
    words = random_bitstrings(c.n, 5, 82)
    pw = np.abs(pairwise_amplitudes(c, words)) ** 2
    for v in pw:
        assert v <= 1e-12 or abs(-np.log2(v) - round(-np.log2(v))) <= 1e-9


def test_doubled_network():
    c = lattice_circuit(2, 3, 4, 91, "haar", "cz")
    I = np.eye(2, dtype=complex)
    assert abs(doubled_expectation(c, [I] * c.n) - 1) <= 1e-12
    for w in random_bitstrings(c.n, 3, 92):
        P = []
        for q in range(c.n):
            e = np.zeros((2, 2), dtype=complex)
            b = (int(w) >> q) & 1
            e[b, b] = 1
            P.append(e)
        a = pairwise_amplitude(c, w)
        assert abs(doubled_expectation(c, P) - abs(a) ** 2) <= 1e-12
        assert abs(doubled_expectation(c, P, method="statevector") - abs(a) ** 2) <= 1e-12


def test_porter_thomas_mean():
    c = lattice_circuit(4, 4, 12, 101, "haar", "cz")
    psi = statevector(c)
    words = random_bitstrings(16, 3000, 102)
    amps = statevector_amplitudes(c, words, psi)
    m = np.mean((1 << 16) * np.abs(amps) ** 2)
    assert abs(m - 1) < 0.1


def test_dense_and_hyperedge_forms_agree_at_25_qubits():
    """The stored 8x8 depth-16 values use the oracle's exact re-labelling of
    diagonal gates (one wire label shared across a CZ); here the plain dense
    form (every gate its own rank-2 or rank-4 tensor, as the oracle's
    definition has it) gives the same amplitude at 25 qubits on the same
    Haar SU(2) + CZ family, in a plan's order imported as data."""
    from paper_2208_01498_amd.planner.plan import make_plan
    circ = lattice_circuit(5, 5, 10, 5100, "haar", "cz")
    spec = make_plan(circ, n_slices=0, B=1, trials=1).order_spec()
    w = random_bitstrings(25, 1, 7)
    a = pairwise_amplitudes(circ, w, order=spec, diagonal_hyperedges=True)
    b = pairwise_amplitudes(circ, w, order=spec, diagonal_hyperedges=False)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
