"""Circuit -> tensor network of factors with labelled binary indices.

The network is the paper's circuit network (single- and two-qubit gates as
rank-2 and rank-4 tensors, the initial |0> and the projection <x| on every
wire, section on classical simulation around Theorem 2), written so that the
executor can run it efficiently:

* a wire index (label) starts at a gate whose matrix is not diagonal and ends
  at the next such gate on that qubit; a diagonal gate (CZ, CP, Z(theta))
  keeps the index of each of its qubits, so its factor is indexed by its input
  labels only and one label can be shared by several factors (a hyperedge);
  optionally, a two-qubit gate of the form SWAP . D with D diagonal
  (fSim(pi/2, phi)) is the diagonal factor D on its input labels followed by
  an exchange of the two wires between the qubits (the plan builder keeps
  whichever form gives the cheaper contraction);
* a wire still in |0> (no non-diagonal gate yet) is a fixed index 0, which is
  substituted into every factor that touches it;
* the last label of each qubit is the output index O_q: it is replaced by
  the bitstring value x_q at run time, turning it into the batch index b;
* the absorption of single-qubit gates and projectors into the two-qubit
  gates (stated as what keeps only the two-qubit gates relevant for the cost)
  is done by merging factors whenever the merge does not increase the number
  of indices (rank-non-increasing simplification).

Each factor carries the set of gate indices it was built from, so the same
tree can be re-evaluated from the circuit by an independent contractor.
"""
import numpy as np

FIXED0 = -1


class Label:
    __slots__ = ("id", "dim", "kind", "qubit", "gate")

    def __init__(self, id, dim, kind, qubit, gate):
        self.id, self.dim, self.kind, self.qubit, self.gate = id, dim, kind, qubit, gate

    def __repr__(self):
        return f"L{self.id}({self.kind},q{self.qubit},g{self.gate})"


class Factor:
    __slots__ = ("data", "labels", "gates", "pos", "weight")

    def __init__(self, data, labels, gates, pos, weight=1.0):
        self.data = data
        self.labels = list(labels)
        self.gates = set(gates)
        self.pos = np.asarray(pos, dtype=np.float64)
        self.weight = weight


class Network:
    """Factors, labels and a global scalar.  Output labels have kind 'out'."""

    def __init__(self, n_qubits, labels, factors, scale, positions):
        self.n_qubits = n_qubits
        self.labels = labels          # id -> Label
        self.factors = factors        # list of Factor
        self.scale = scale            # complex
        self.positions = positions    # qubit coordinates
        self.out_label = {l.qubit: l.id for l in labels.values() if l.kind == "out"}
        self.doubled = False          # U and its conjugate (projector mode)

    def label_users(self):
        users = {}
        for i, f in enumerate(self.factors):
            for l in f.labels:
                users.setdefault(l, set()).add(i)
        return users


# entries below this fraction of the largest are structural zeros (cos(pi/2)
# evaluates to 6e-17, not 0)
ZERO_TOL = 1e-14


def _nz(m):
    return np.abs(m) > ZERO_TOL * np.max(np.abs(m))


def _is_diag(m):
    return not np.any(_nz(m) & ~np.eye(m.shape[0], dtype=bool))


_SWAP_PATTERN = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=bool)


def _is_swap_diag(m):
    """A two-qubit matrix SWAP . D with D diagonal (nonzero pattern of SWAP),
    e.g. fSim(pi/2, phi)."""
    return m.shape == (4, 4) and np.array_equal(_nz(m), _SWAP_PATTERN)


def _gate_pos(circ, qs):
    return np.mean([circ.positions[q] for q in qs], axis=0)


def _svd_halves(m):
    """A two-qubit gate G[2 o1 + o2, 2 i1 + i2] as two rank-3 halves joined
    by a bond (the proof of Theorem 2, Fig. 3a): G = sum_k A[o1, i1, k]
    B[o2, i2, k] from the SVD of G regrouped as a matrix over (o1 i1) x
    (o2 i2); singular values above 1e-12 of the largest are kept (2 for
    CZ and CP, 4 for fSim and generic SU(4)) and absorbed into A; the bond
    is padded with zero columns to a power of two (it becomes one binary
    label per bit)."""
    t = m.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)    # (o1 i1) x (o2 i2)
    U, S, Vh = np.linalg.svd(t)
    r = int(np.sum(S > 1e-12 * S[0]))
    d = 1 if r <= 1 else (2 if r <= 2 else 4)
    A = np.zeros((4, d), dtype=np.complex128)
    Bm = np.zeros((4, d), dtype=np.complex128)
    A[:, :r] = U[:, :r] * S[:r]
    Bm[:, :r] = Vh[:r, :].T
    return A.reshape(2, 2, d), Bm.reshape(2, 2, d), d


def build_network(circ, simplify=True, swap_relabel=False, coarsen=0, svd_split=False):
    """The circuit's network.  Diagonal gates keep their wires' labels
    (hyperedges) unless ``svd_split``, the paper-faithful form of the proof
    of Theorem 2: every two-qubit gate becomes two rank-3 halves joined by a
    bond of its Schmidt rank (2 or 4; a bond of 4 is two binary labels),
    every one-qubit gate a rank-2 tensor, each half placed at its qubit."""
    n = circ.n
    labels = {}
    factors = []
    scale = 1.0 + 0.0j
    scalar_gates = []
    cur = [FIXED0] * n
    nxt = [0]

    def new_label(q, g):
        lid = nxt[0]
        nxt[0] += 1
        labels[lid] = Label(lid, 2, "wire", q, g)
        return lid

    def add_factor(data, labs, gi, qs):
        nonlocal scale
        # substitute fixed |0> inputs
        idx = []
        keep = []
        for l in labs:
            if l == FIXED0:
                idx.append(0)
            else:
                idx.append(slice(None))
                keep.append(l)
        data = data[tuple(idx)]
        if len(set(keep)) != len(keep):
            raise ValueError("gate acts twice on one wire")
        if not keep:
            scale *= complex(data)
            scalar_gates.append((gi, qs))
            return
        factors.append(Factor(np.ascontiguousarray(data, dtype=np.complex128), keep,
                              {gi}, _gate_pos(circ, qs)))

    for gi, g in enumerate(circ.gates):
        qs = g.qubits
        if svd_split:
            if len(qs) == 1:
                o = new_label(qs[0], gi)
                add_factor(g.matrix.copy(), [o, cur[qs[0]]], gi, qs)
                cur[qs[0]] = o
                continue
            A, Bh, d = _svd_halves(g.matrix)
            nb = int(round(np.log2(d)))
            bond = [new_label(qs[0], gi) for _ in range(nb)]
            outs = [new_label(q, gi) for q in qs]
            for b in bond:
                labels[b].kind = "wire"
            sh = (2, 2) + (2,) * nb
            add_factor(A.reshape(sh), [outs[0], cur[qs[0]]] + bond, gi, qs[:1])
            add_factor(Bh.reshape(sh), [outs[1], cur[qs[1]]] + bond, gi, qs[1:])
            cur[qs[0]], cur[qs[1]] = outs
            continue
        if _is_diag(g.matrix):
            d = np.diag(g.matrix).reshape((2,) * len(qs))
            add_factor(d, [cur[q] for q in qs], gi, qs)
        elif swap_relabel and len(qs) == 2 and _is_swap_diag(g.matrix):
            # G = SWAP . D: a diagonal weight on the input wires, then the two
            # wires exchange qubits (no new index)
            m = g.matrix
            d = np.array([[m[0, 0], m[2, 1]], [m[1, 2], m[3, 3]]], dtype=np.complex128)
            add_factor(d, [cur[q] for q in qs], gi, qs)
            cur[qs[0]], cur[qs[1]] = cur[qs[1]], cur[qs[0]]
        else:
            outs = [new_label(q, gi) for q in qs]
            t = g.matrix.reshape((2,) * (2 * len(qs)))
            add_factor(t, outs + [cur[q] for q in qs], gi, qs)
            for q, o in zip(qs, outs):
                cur[q] = o
    # outputs
    for q in range(n):
        if cur[q] == FIXED0:
            lid = new_label(q, -1)
            factors.append(Factor(np.array([1.0, 0.0], dtype=np.complex128), [lid],
                                  set(), circ.positions[q]))
            labels[lid].kind = "out"
        else:
            # after wire exchanges the last label of qubit q may have been
            # started on another qubit: it is measured on q
            labels[cur[q]].kind = "out"
            labels[cur[q]].qubit = q
    net = Network(n, labels, factors, scale, circ.positions)
    if simplify:
        simplify_network(net)
        if coarsen:
            coarsen_network(net, coarsen)
    _attach_scalar_gates(net, circ, scalar_gates)
    return net


def build_doubled_network(circ, traced=(), simplify=True, swap_relabel=False):
    """The paper's quantity c = <0|U^dag (x)_q P_q U|0> for product
    projectors (the problem statement around Theorem 2): the network of U
    and its complex conjugate, with P_q = |x_q><x_q| on the qubits not in
    `traced` (both output indices of qubit q are fixed to x_q at run time)
    and P_q = 1 on the qubits in `traced` (the two output indices become one
    summed index).  With no qubit traced, c(x) = |<x|C|0>|^2; tracing a set
    of qubits gives the marginal probability of the others.  Gate ids of the
    conjugate layer are offset by the number of gates."""
    traced = set(int(q) for q in traced)
    one = build_network(circ, simplify=simplify, swap_relabel=swap_relabel)
    off = max(one.labels) + 1
    G = len(circ.gates)
    labels = {}
    for l, L in one.labels.items():
        labels[l] = Label(l, L.dim, L.kind, L.qubit, L.gate)
        labels[l + off] = Label(l + off, L.dim, L.kind, L.qubit, L.gate + G if L.gate >= 0 else L.gate)
    out1 = {L.qubit: l for l, L in one.labels.items() if L.kind == "out"}
    ren = {}
    for q in traced:
        o = out1[q]
        ren[o + off] = o
        labels[o].kind = "wire"
        del labels[o + off]
    factors = [Factor(f.data.copy(), f.labels, f.gates, f.pos, f.weight) for f in one.factors]
    for f in one.factors:
        factors.append(Factor(np.conj(f.data), [ren.get(l + off, l + off) for l in f.labels],
                              {g + G for g in f.gates}, f.pos, f.weight))
    scale = one.scale * np.conj(one.scale)
    net = Network(circ.n, labels, factors, complex(scale), circ.positions)
    net.doubled = True
    if simplify:
        simplify_network(net)
    return net


def _attach_scalar_gates(net, circ, scalar_gates):
    """A gate that reduced to a constant (a diagonal gate on wires still in
    |0>) is recorded in the leaf holding the nearest gate on one of its
    qubits, so that every gate belongs to exactly one leaf."""
    owner = {}
    for i, f in enumerate(net.factors):
        for g in f.gates:
            owner[g] = i
    for gi, qs in scalar_gates:
        best = None
        for gj, g in enumerate(circ.gates):
            if gj in owner and set(g.qubits) & set(qs):
                key = (abs(gj - gi), gj)
                if best is None or key < best[0]:
                    best = (key, owner[gj])
        if best is None:
            best = (None, 0)
        if net.factors:
            net.factors[best[1]].gates.add(gi)


def contract_factors(f, g, keep):
    """Dense FP64 contraction of two factors, keeping labels in ``keep``."""
    la, lb = f.labels, g.labels
    allab = list(dict.fromkeys(la + lb))
    letters = {l: chr(ord('a') + i) if i < 26 else chr(ord('A') + i - 26)
               for i, l in enumerate(allab)}
    out = [l for l in allab if l in keep]
    spec = "%s,%s->%s" % ("".join(letters[l] for l in la), "".join(letters[l] for l in lb),
                          "".join(letters[l] for l in out))
    data = np.einsum(spec, f.data, g.data)
    wsum = f.weight + g.weight
    pos = (f.pos * f.weight + g.pos * g.weight) / wsum
    return Factor(np.ascontiguousarray(data), out, f.gates | g.gates, pos, wsum)


def simplify_network(net, max_rank=None):
    """Merge neighbouring factors while the merge does not raise the rank."""
    labels = net.labels
    alive = {i: f for i, f in enumerate(net.factors)}
    users = {}
    for i, f in alive.items():
        for l in f.labels:
            users.setdefault(l, set()).add(i)
    nid = len(net.factors)
    changed = True
    while changed:
        changed = False
        for i in sorted(alive):
            if i not in alive:
                continue
            f = alive[i]
            best = None
            for l in f.labels:
                for j in users[l]:
                    if j == i or j not in alive:
                        continue
                    g = alive[j]
                    u = set(f.labels) | set(g.labels)
                    keep = set(x for x in u if labels[x].kind == "out" or
                               len(users[x] - {i, j}) > 0)
                    if len(keep) <= max(len(f.labels), len(g.labels)):
                        key = (len(keep), j)
                        if best is None or key < best[0]:
                            best = (key, j, keep)
            if best is None:
                continue
            _, j, keep = best
            g = alive[j]
            h = contract_factors(f, g, keep)
            for x in f.labels:
                users[x].discard(i)
            for x in g.labels:
                users[x].discard(j)
            del alive[i]
            del alive[j]
            alive[nid] = h
            for x in h.labels:
                users.setdefault(x, set()).add(nid)
            nid += 1
            changed = True
    # rank-0 factors become scalars
    facs = []
    for i in sorted(alive):
        f = alive[i]
        if not f.labels:
            net.scale *= complex(f.data)
        else:
            facs.append(f)
    if facs:
        for i in sorted(alive):
            if not alive[i].labels:
                facs[0].gates |= alive[i].gates
    net.factors = facs
    return net


def coarsen_network(net, max_rank):
    """Merge neighbouring factors (in float64, on the host) while the merged
    factor keeps at most ``max_rank`` labels and at most one label more than
    the larger of the two: fewer, larger leaves, so each amplitude term passes
    through fewer single-precision roundings of leaf entries and the plan has
    fewer tiny steps."""
    labels = net.labels
    alive = {i: f for i, f in enumerate(net.factors)}
    users = {}
    for i, f in alive.items():
        for l in f.labels:
            users.setdefault(l, set()).add(i)
    nid = len(net.factors)

    def merged(i, j):
        f, g = alive[i], alive[j]
        u = set(f.labels) | set(g.labels)
        return set(x for x in u if labels[x].kind == "out" or len(users[x] - {i, j}) > 0)

    while True:
        best = None
        for i in sorted(alive):
            f = alive[i]
            for l in f.labels:
                for j in users[l]:
                    if j <= i or j not in alive:
                        continue
                    g = alive[j]
                    keep = merged(i, j)
                    if len(keep) > max_rank or len(keep) > max(len(f.labels), len(g.labels)) + 1:
                        continue
                    key = (len(keep), -len(set(f.labels) & set(g.labels)), i, j)
                    if best is None or key < best[0]:
                        best = (key, i, j, keep)
        if best is None:
            break
        _, i, j, keep = best
        f, g = alive[i], alive[j]
        h = contract_factors(f, g, keep)
        for x in f.labels:
            users[x].discard(i)
        for x in g.labels:
            users[x].discard(j)
        del alive[i]
        del alive[j]
        alive[nid] = h
        for x in h.labels:
            users.setdefault(x, set()).add(nid)
        nid += 1
    net.factors = [alive[i] for i in sorted(alive)]
    return net
