"""Seeded circuit families and output bitstrings.

Lattice random circuits (the depth-d workloads): each cycle is a layer of
single-qubit gates on every qubit followed by a layer of two-qubit gates on one
of four nearest-neighbour edge patterns, used cyclically:
  P0 horizontal (r,c)-(r,c+1), c even;  P1 vertical (r,c)-(r+1,c), r even;
  P2 horizontal, c odd;                 P3 vertical, r odd;
cycle t uses P_{t mod 4}; there is no final single-qubit layer.  These follow
the Sycamore-type structure the paper's examples use (one single-qubit and at
most one two-qubit gate per qubit per cycle); the patterns themselves are a
reading, since the paper does not list them.

The IQP family of the paper's first example and the (2+1)-dimensional stack
are here too.  Random numbers come from numpy's PCG64 with explicit seeds.
"""
import numpy as np

from .gates import (H, SQRT_X, SQRT_Y, SQRT_W, CZ, z_phase, cphase, fsim,
                    haar_su2, haar_su4)
from .model import Circuit, Gate

SQRT_SET = (("sqrtX", SQRT_X), ("sqrtY", SQRT_Y), ("sqrtW", SQRT_W))
CLIFFORD_SET = (("sqrtX", SQRT_X), ("sqrtY", SQRT_Y))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def lattice_positions(R, C):
    return np.array([[r, c] for r in range(R) for c in range(C)], dtype=np.float64)


def edge_patterns(R, C):
    """The four edge patterns P0..P3 as lists of (q1, q2) with q1 < q2."""
    P = [[], [], [], []]
    for r in range(R):
        for c in range(C):
            q = r * C + c
            if c + 1 < C:
                P[0 if c % 2 == 0 else 2].append((q, q + 1))
            if r + 1 < R:
                P[1 if r % 2 == 0 else 3].append((q, q + C))
    return [sorted(p) for p in P]


def lattice_circuit(R, C, depth, seed, oneq="sqrt", twoq="cz", name=""):
    """Random lattice circuit.

    oneq: "sqrt" (sqrtX/sqrtY/sqrtW, never the same gate twice in a row on a
          qubit), "clifford" (sqrtX/sqrtY alternating the same way) or "haar"
          (Haar SU(2) per gate).
    twoq: "cz" or "fsim" (fSim(pi/2, pi/6)).
    """
    rng = _rng(seed)
    n = R * C
    pats = edge_patterns(R, C)
    gates = []
    prev = [None] * n
    gset = SQRT_SET if oneq == "sqrt" else CLIFFORD_SET
    G2 = CZ if twoq == "cz" else fsim(np.pi / 2, np.pi / 6)
    n2 = "CZ" if twoq == "cz" else "fSim"
    for t in range(depth):
        for q in range(n):
            if oneq == "haar":
                gates.append(Gate((q,), haar_su2(rng), "su2"))
                continue
            if prev[q] is None:
                k = int(rng.integers(len(gset)))
            else:
                choices = [i for i in range(len(gset)) if i != prev[q]]
                k = choices[int(rng.integers(len(choices)))]
            prev[q] = k
            gates.append(Gate((q,), gset[k][1].copy(), gset[k][0]))
        for (a, b) in pats[t % 4]:
            gates.append(Gate((a, b), G2.copy(), n2))
    return Circuit(n, gates, lattice_positions(R, C),
                   name or f"lattice{R}x{C}_d{depth}_{oneq}_{twoq}",
                   {"R": R, "C": C, "depth": depth, "seed": seed,
                    "oneq": oneq, "twoq": twoq})


def iqp_lattice_circuit(R, C, seed, max_dist=2, name=""):
    """H on all qubits; Z(theta_i), theta_i ~ U[0, 2pi); CP(phi_ij),
    phi_ij ~ U[0, 2pi), on every pair at Manhattan distance <= max_dist, in
    lexicographic (i, j) order; H on all qubits."""
    rng = _rng(seed)
    n = R * C
    gates = [Gate((q,), H.copy(), "H") for q in range(n)]
    thetas = rng.uniform(0, 2 * np.pi, size=n)
    for q in range(n):
        gates.append(Gate((q,), z_phase(thetas[q]), "Z"))
    pairs = []
    for i in range(n):
        ri, ci = divmod(i, C)
        for j in range(i + 1, n):
            rj, cj = divmod(j, C)
            if abs(ri - rj) + abs(ci - cj) <= max_dist:
                pairs.append((i, j))
    phis = rng.uniform(0, 2 * np.pi, size=len(pairs))
    for (i, j), ph in zip(pairs, phis):
        gates.append(Gate((i, j), cphase(ph), "CP"))
    gates += [Gate((q,), H.copy(), "H") for q in range(n)]
    return Circuit(n, gates, lattice_positions(R, C),
                   name or f"iqp{R}x{C}_dist{max_dist}",
                   {"R": R, "C": C, "seed": seed, "thetas": thetas.tolist(),
                    "pairs": pairs, "phis": phis.tolist()})


def paper_iqp_circuit(L, T, seed, gamma=3.0):
    """The IQP family of the paper's first example on an L x L lattice: H on
    all qubits; T steps, each putting diag(1, e^{i pi m/4}), m uniform in
    0..7, on every qubit, then diag(1,1,1,i^m), m uniform in 0..3, on each
    nearest-neighbour pair none of whose qubits was already paired in this
    step, with probability gamma ln(N)/N (m = 0 is the identity, which makes
    the paper's 7/8 and 3/4 factors); H on all qubits."""
    rng = _rng(seed)
    n = L * L
    p = gamma * np.log(n) / n
    gates = [Gate((q,), H.copy(), "H") for q in range(n)]
    edges = sorted(e for pat in edge_patterns(L, L) for e in pat)
    for _ in range(T):
        for q in range(n):
            m = int(rng.integers(8))
            if m:
                gates.append(Gate((q,), z_phase(np.pi * m / 4), "P"))
        used = set()
        for (a, b) in [edges[i] for i in rng.permutation(len(edges))]:
            if a in used or b in used:
                continue
            if rng.random() < p:
                m = int(rng.integers(4))
                used.update((a, b))
                if m:
                    gates.append(Gate((a, b), cphase(np.pi * m / 2), "CP"))
    gates += [Gate((q,), H.copy(), "H") for q in range(n)]
    return Circuit(n, gates, lattice_positions(L, L), f"paperiqp{L}x{L}_T{T}",
                   {"L": L, "T": T, "seed": seed, "gamma": gamma})


def sycamore_type_circuit(L, periods, p_inaccessible, seed):
    """The paper's second example on an L x L lattice: cycles of one
    single-qubit gate per qubit (sqrt(X/Y/W), never the same twice in a row)
    followed by fSim(pi/2, pi/6) on one of the four nearest-neighbour edge
    patterns, eight cycles per period in the order A B C D C D A B (each
    coupling applied twice per period), repeated for `periods` periods; in
    each period every qubit is independently inaccessible with probability
    `p_inaccessible`, and no gate acts on it during that period."""
    rng = _rng(seed)
    n = L * L
    pats = edge_patterns(L, L)
    order = [0, 1, 2, 3, 2, 3, 0, 1]
    G2 = fsim(np.pi / 2, np.pi / 6)
    gates = []
    prev = [None] * n
    for _ in range(periods):
        off = rng.random(n) < p_inaccessible
        for c in order:
            for q in range(n):
                if off[q]:
                    continue
                if prev[q] is None:
                    k = int(rng.integers(len(SQRT_SET)))
                else:
                    choices = [i for i in range(len(SQRT_SET)) if i != prev[q]]
                    k = choices[int(rng.integers(len(choices)))]
                prev[q] = k
                gates.append(Gate((q,), SQRT_SET[k][1].copy(), SQRT_SET[k][0]))
            for (a, b) in pats[c]:
                if not off[a] and not off[b]:
                    gates.append(Gate((a, b), G2.copy(), "fSim"))
    return Circuit(n, gates, lattice_positions(L, L), f"sycamoretype{L}x{L}_q{periods}",
                   {"L": L, "periods": periods, "p": p_inaccessible, "seed": seed})


def paper_family_instances(L):
    """One seeded realization per family of the paper's examples at size L:
    (name, circuit, time steps T) for the IQP family (T = L^2, gamma = 3),
    the Sycamore-type family (5 periods of 8 cycles; qubits inaccessible
    with probability 0.88, and 0.5 as a denser variant) and the
    (2+1)-dimensional family with cavities (S = 5, sigma = 10,
    lam = 5e4 (L/200)^3.5) at T = L time steps: the paper's alpha = 0.1
    gives less than one step below L = 10, so these sizes take alpha = 1."""
    return [("iqp_T=L^2_gamma=3", paper_iqp_circuit(L, L * L, 5200 + L), L * L),
            ("sycamore_type_q=5_p=0.88", sycamore_type_circuit(L, 5, 0.88, 5300 + L), 40),
            ("sycamore_type_q=5_p=0.5", sycamore_type_circuit(L, 5, 0.5, 5400 + L), 40),
            ("cavity_T=L_S=5", cavity_circuit(L, 5500 + L, T=L), L)]


def _pattern_counts(free, pat):
    """Two-qubit gates per site of an L x L grid for edge pattern `pat`
    (P0/P2: horizontal pairs from even/odd columns, P1/P3: vertical pairs
    from even/odd rows), a gate on a pair when both sites are free."""
    L = free.shape[-1]
    f = np.zeros(free.shape, dtype=np.int64)
    start = 0 if pat in (0, 1) else 1
    idx = np.arange(start, L - 1, 2)
    if pat in (0, 2):
        g = free[..., :, idx] & free[..., :, idx + 1]
        f[..., :, idx] += g
        f[..., :, idx + 1] += g
    else:
        g = free[..., idx, :] & free[..., idx + 1, :]
        f[..., idx, :] += g
        f[..., idx + 1, :] += g
    return f


def sycamore_type_gate_counts(L, periods, p_inaccessible, seed):
    """Two-qubit gate count per qubit (L x L array) of a Sycamore-type
    circuit under the rule of `sycamore_type_circuit` (each edge pattern
    twice per period, a qubit inaccessible for a whole period with
    probability p), without building the gates: for the bound evaluations
    at sizes whose gate lists would not fit in memory.  One realization per
    seed (its own random stream, not that of `sycamore_type_circuit`)."""
    rng = _rng(seed)
    f = np.zeros((L, L), dtype=np.int64)
    for _ in range(periods):
        free = rng.random((L, L)) >= p_inaccessible
        for pat in range(4):
            f += 2 * _pattern_counts(free, pat)
    return f


def _cavity_layers(L, rng, T, S, sigma, lam):
    """Space-time layout of the paper's third example: v ~ Poisson(lam)
    cavities of S x S x S sites (t, x, y) with uniformly random corners,
    each kept with probability exp(-(x^2/L^2 + y^2/L^2 + t^2/T^2) / sigma^2)
    for its centre measured from the centre of the T x L x L box; one edge
    pattern (orientation and parity uniform, as in `_pattern_counts`) per
    time step.  Returns (free[T, L, L]: site outside every cavity, pats[T])."""
    v = int(rng.poisson(lam))
    corner = np.stack([rng.integers(0, T, v), rng.integers(0, L, v), rng.integers(0, L, v)], axis=1)
    ctr = corner + (S - 1) / 2.0 - np.array([T, L, L]) / 2.0
    keep = rng.random(v) < np.exp(-((ctr[:, 1] / L) ** 2 + (ctr[:, 2] / L) ** 2 +
                                    (ctr[:, 0] / T) ** 2) / sigma ** 2)
    corner = corner[keep]
    # coverage by a 3-D difference array: +1 at a box's low corner, signed
    # corrections at the other seven corners, then prefix sums
    diff = np.zeros((T + 1, L + 1, L + 1), dtype=np.int32)
    hi = np.minimum(corner + S, np.array([T, L, L]))
    for dt in (0, 1):
        for dx in (0, 1):
            for dy in (0, 1):
                sign = (-1) ** (dt + dx + dy)
                pt = np.where(dt, hi[:, 0], corner[:, 0])
                px = np.where(dx, hi[:, 1], corner[:, 1])
                py = np.where(dy, hi[:, 2], corner[:, 2])
                np.add.at(diff, (pt, px, py), sign)
    cover = diff.cumsum(0).cumsum(1).cumsum(2)[:T, :L, :L]
    pats = rng.integers(0, 4, T)
    return cover == 0, pats


def _cavity_steps(L, alpha, T):
    return max(1, int(round(alpha * L))) if T is None else int(T)


def cavity_circuit_gate_counts(L, seed, alpha=0.1, S=5, sigma=10.0, lam=None, T=None):
    """The paper's third example, (2+1)-dimensional random circuits with
    cavities, as two-qubit gate counts per qubit (L x L) and the number of
    time steps T = max(1, round(alpha L)) (or T as given).  Each time step
    applies one edge pattern of uniformly random orientation and parity (a
    dense layer of nearest-neighbour gates) to the pairs whose sites are
    both outside every cavity (`_cavity_layers`).  lam = 5e4 (L/200)^3.5 by
    default.  The same realization as `cavity_circuit(L, seed, ...)`."""
    rng = _rng(seed)
    T = _cavity_steps(L, alpha, T)
    if lam is None:
        lam = 5e4 * (L / 200.0) ** 3.5
    free, pats = _cavity_layers(L, rng, T, S, sigma, lam)
    f = np.zeros((L, L), dtype=np.int64)
    for t in range(T):
        f += _pattern_counts(free[t], int(pats[t]))
    return f, T


def cavity_circuit(L, seed, alpha=0.1, S=5, sigma=10.0, lam=None, T=None):
    """The paper's third example as a circuit on an L x L lattice
    (q = r L + c): T time steps (T = max(1, round(alpha L)) unless given),
    each a dense layer of nearest-neighbour gates on one edge pattern of
    random orientation and parity, every gate an independent Haar SU(4),
    except on pairs with a site inside a cavity (`_cavity_layers`).  The
    cavity draws come first in the seeded stream, so the two-qubit gate
    counts equal `cavity_circuit_gate_counts(L, seed, ...)`."""
    rng = _rng(seed)
    T = _cavity_steps(L, alpha, T)
    if lam is None:
        lam = 5e4 * (L / 200.0) ** 3.5
    free, pats = _cavity_layers(L, rng, T, S, sigma, lam)
    gates = []
    for t in range(T):
        pat = int(pats[t])
        start = 0 if pat in (0, 1) else 1
        for a in range(L):
            for b in range(start, L - 1, 2):
                # P0/P2: horizontal pair (a, b)-(a, b+1); P1/P3: vertical (b, a)-(b+1, a)
                (r1, c1), (r2, c2) = (((a, b), (a, b + 1)) if pat in (0, 2)
                                      else ((b, a), (b + 1, a)))
                if free[t, r1, c1] and free[t, r2, c2]:
                    gates.append(Gate((r1 * L + c1, r2 * L + c2), haar_su4(rng), "SU4"))
    return Circuit(L * L, gates, lattice_positions(L, L), f"cavity{L}x{L}_T{T}",
                   {"L": L, "T": T, "alpha": alpha, "S": S, "sigma": sigma, "lam": lam,
                    "seed": seed, "free_sites": int(free.sum()),
                    "patterns": [int(x) for x in pats]})


def stack3d_circuit(X, Y, Z, layers, seed, name=""):
    """(2+1)-dimensional-style random circuit on an X x Y x Z qubit stack
    (q = x + X*y + X*Y*z).  Each layer picks an axis uniformly from {x,y,z}
    and a parity uniformly from {0,1}; the candidate gates are the
    nearest-neighbour pairs along that axis whose lower coordinate has that
    parity; each candidate is kept with probability rho_t ~ U[0.5, 1.0] and
    is an independent Haar SU(4)."""
    rng = _rng(seed)
    n = X * Y * Z
    dims = (X, Y, Z)
    gates = []
    rhos = []
    for t in range(layers):
        axis = int(rng.integers(3))
        parity = int(rng.integers(2))
        rho = float(rng.uniform(0.5, 1.0))
        rhos.append(rho)
        cands = []
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    c = [x, y, z]
                    if c[axis] % 2 != parity or c[axis] + 1 >= dims[axis]:
                        continue
                    d = list(c)
                    d[axis] += 1
                    qa = c[0] + X * c[1] + X * Y * c[2]
                    qb = d[0] + X * d[1] + X * Y * d[2]
                    cands.append((min(qa, qb), max(qa, qb)))
        for e in sorted(cands):
            if rng.random() < rho:
                gates.append(Gate(e, haar_su4(rng), "su4"))
    pos = np.array([[q % X, (q // X) % Y, q // (X * Y)] for q in range(n)],
                   dtype=np.float64)
    return Circuit(n, gates, pos, name or f"stack{X}x{Y}x{Z}_L{layers}",
                   {"dims": [X, Y, Z], "layers": layers, "seed": seed,
                    "rhos": rhos})


def product_circuit(n, depth, seed):
    """Single-qubit gates only (Haar SU(2)), qubits on a line."""
    rng = _rng(seed)
    gates = [Gate((q,), haar_su2(rng), "su2") for _ in range(depth) for q in range(n)]
    pos = np.array([[q, 0.0] for q in range(n)], dtype=np.float64)
    return Circuit(n, gates, pos, f"product{n}_d{depth}", {"seed": seed})


def mirror(circ):
    """C followed by its inverse: every gate reversed in order and replaced by
    its conjugate transpose, so <x|C^dag C|0> = [x == 0]."""
    inv = [Gate(g.qubits, g.matrix.conj().T.copy(), g.name + "_dg")
           for g in reversed(circ.gates)]
    return Circuit(circ.n, list(circ.gates) + inv, circ.positions.copy(),
                   circ.name + "_mirror", dict(circ.meta, mirror=True))


def pack_bits(bits):
    """(B, n) array of 0/1 -> (B,) uint64 with bit q = bits[:, q]."""
    bits = np.asarray(bits, dtype=np.uint64)
    out = np.zeros(bits.shape[0], dtype=np.uint64)
    for q in range(bits.shape[1]):
        out |= bits[:, q] << np.uint64(q)
    return out


def unpack_bits(words, n):
    words = np.asarray(words, dtype=np.uint64)
    return np.array([[(int(w) >> q) & 1 for q in range(n)] for w in words],
                    dtype=np.uint8)


def random_bitstrings(n, count, seed):
    """Uniform random output bitstrings, packed into uint64."""
    rng = _rng(seed)
    bits = rng.integers(0, 2, size=(count, n), dtype=np.uint8)
    return pack_bits(bits)


def circuit_seed(k):
    return 1000 * k


def bitstring_seed(k):
    return 1000 * k + 1


CONFIGS = {
    # name: (builder, batch, slices log2, description)
    "cfg1": dict(k=1, batch=8, slices_log2=0,
                 desc="4x4 lattice, depth 8, sqrt(X/Y/W) + CZ, 8 bitstrings"),
    "cfg2": dict(k=2, batch=256, slices_log2=None,
                 desc="6x6 lattice, depth 12, sqrt(X/Y/W) + fSim(pi/2,pi/6), 256 bitstrings"),
    "cfg3": dict(k=3, batch=64, slices_log2=10,
                 desc="8x8 lattice, depth 16, Haar SU(2) + CZ, 2^10 slices, 64 bitstrings"),
    "cfg4": dict(k=4, batch=1024, slices_log2=None,
                 desc="IQP on a 6x8 grid, CP on pairs within distance 2, 1024 bitstrings"),
}


def config_names():
    return sorted(CONFIGS)


def make_config(name, seed=None):
    """Return (circuit, bitstrings uint64[B], info dict) for a named workload."""
    info = dict(CONFIGS[name])
    k = info["k"]
    cs = circuit_seed(k) if seed is None else seed
    if name == "cfg1":
        c = lattice_circuit(4, 4, 8, cs, "sqrt", "cz", "cfg1_4x4_d8")
    elif name == "cfg2":
        c = lattice_circuit(6, 6, 12, cs, "sqrt", "fsim", "cfg2_6x6_d12")
    elif name == "cfg3":
        c = lattice_circuit(8, 8, 16, cs, "haar", "cz", "cfg3_8x8_d16")
    elif name == "cfg4":
        c = iqp_lattice_circuit(6, 8, cs, 2, "cfg4_iqp6x8")
    else:
        raise KeyError(name)
    bits = random_bitstrings(c.n, info["batch"], bitstring_seed(k) if seed is None else seed + 1)
    info["name"] = name
    return c, bits, info


def serving_pool(seed=5100):
    """Circuit families of the served mixed stream, three instances each:
    5x5 depth 10, 6x6 depth 12 and 8x8 depth 16 lattice circuits of the
    headline family (Haar SU(2) + CZ; the stream does not name a gate set),
    and the (2+1)-dimensional 3x3x4 stack with 10 layers of SU(4) gates.
    Returns a list of (family, circuit, slices log2)."""
    pool = []
    for j in range(3):
        pool.append(("5x5d10", lattice_circuit(5, 5, 10, seed + j, "haar", "cz", f"mix5x5d10_{j}"), 0))
        pool.append(("6x6d12", lattice_circuit(6, 6, 12, seed + 10 + j, "haar", "cz", f"mix6x6d12_{j}"), 0))
        pool.append(("8x8d16", lattice_circuit(8, 8, 16, seed + 20 + j, "haar", "cz", f"mix8x8d16_{j}"), 10))
        pool.append(("3x3x4", stack3d_circuit(3, 3, 4, 10, seed + 30 + j, f"mix3x3x4_{j}"), 0))
    return pool
