"""Naive pairwise tensor-network contraction in complex128 (test
infrastructure only).

The network follows the paper's construction of a circuit as a tensor network
(section on classical simulation of quantum circuits, around Theorem 2):
every gate is a tensor over its input and output wires (rank 2 for single-
qubit gates, rank 4 for two-qubit gates, T[o1,o2,i1,i2] = G[2o1+o2, 2i1+i2]),
the initial state |0> fixes every input wire to 0 and the projection onto
<x| fixes every output wire to x_q (each piece carrying such a wire is
indexed at that value).  Nothing is absorbed, split or pre-contracted across
gates: every piece stays a plain dense tensor.

One optional, exact re-labelling: with ``diagonal_hyperedges`` a gate whose
matrix is diagonal keeps its wires' labels (output wire = input wire), so its
tensor is indexed by the input labels only and a label may be shared by more
than two tensors.  This is an identity of the sum, not an approximation, and
it keeps intermediates small when the order being followed treats diagonal
gates that way.  Both forms are checked against each other and against the
state vector in the tests.

A pairwise step multiplies the two tensors entry by entry over the union of
their indices and sums the indices that no other live tensor still carries;
a step over index union U costs prod_{i in U} dim(i) multiplications, the
quantity of Eq. (3).  Here a step is a transpose to [kept-shared, free-A,
summed] x [kept-shared, summed, free-B], one batched matmul and a reshape.

Orders: the oracle's own greedy (smallest result first), or an order imported
as data: leaves given as sets of gate indices and a list of pairwise steps.
Index slicing: the wires listed as (qubit, gate) -- the wire of that qubit
immediately after that gate -- are fixed to every assignment in turn, in
ascending assignment order s (wire j takes bit j of s), and the contracted
values are summed in complex128.
"""
import itertools
import numpy as np

def _is_diag(m):
    return np.count_nonzero(m - np.diag(np.diag(m))) == 0


class OracleNetwork:
    """Pieces (array, labels, gate tag) of the network of one amplitude.

    The tag of a piece is its gate's index in the circuit; a qubit whose wire
    never leaves |0> contributes the scalar <x_q|0> to ``const``.
    """

    def __init__(self, circ, word, diagonal_hyperedges=True):
        n = circ.n
        self.pieces = []          # [array, labels(list of int), tag]
        self.wire_after = {}      # (qubit, gate index) -> label
        self.const = 1.0 + 0.0j
        nxt = itertools.count()
        cur = {}
        last = {}
        for gi, g in enumerate(circ.gates):
            for q in g.qubits:
                last[q] = gi
        for q in range(n):
            cur[q] = next(nxt)
            self.wire_after[(q, -1)] = cur[q]
        for gi, g in enumerate(circ.gates):
            qs = g.qubits
            ins = [cur[q] for q in qs]
            if diagonal_hyperedges and _is_diag(g.matrix):
                d = np.diag(g.matrix).reshape((2,) * len(qs))
                if len(qs) == 2 and ins[0] == ins[1]:
                    raise ValueError("two-qubit gate on one wire")
                self.pieces.append([d.astype(np.complex128), list(ins), gi])
            else:
                outs = [next(nxt) for _ in qs]
                t = g.matrix.reshape((2,) * (2 * len(qs)))
                self.pieces.append([t.astype(np.complex128), outs + ins, gi])
                for q, o in zip(qs, outs):
                    cur[q] = o
            for q in qs:
                self.wire_after[(q, gi)] = cur[q]
        # the initial |0> and the projection onto <x| fix the first and the
        # last wire of every qubit: each piece carrying such a wire is
        # indexed at that value (the paper absorbs the projectors into the
        # gate tensors); a qubit no gate touches contributes <x_q|0>
        fixed = {}
        for q in range(n):
            xq = (int(word) >> q) & 1
            fixed[self.wire_after[(q, -1)]] = 0
            if cur[q] != self.wire_after[(q, -1)]:
                fixed[cur[q]] = xq
            elif xq == 1:
                # the wire never leaves |0> (no gate, or diagonal gates only)
                self.const = 0.0 + 0.0j
        self.pieces = _restrict(self.pieces, fixed)

    def labels_of_slice_spec(self, spec):
        return [self.wire_after[(q, g)] for (q, g) in spec]


def _counts(labels_list):
    c = {}
    for ls in labels_list:
        for l in ls:
            c[l] = c.get(l, 0) + 1
    return c


def contract_pair(A, la, B, lb, keep):
    """Contract two dense tensors.  Indices of both operands that are in
    ``keep`` survive (as batch indices if shared); shared indices not in keep
    are summed; an index of one operand only that is not in keep is summed
    within that operand first.  Returns (C, labels of C)."""
    la, lb = list(la), list(lb)
    for l in [l for l in la if l not in lb and l not in keep]:
        ax = la.index(l)
        A = A.sum(axis=ax)
        la.pop(ax)
    for l in [l for l in lb if l not in la and l not in keep]:
        ax = lb.index(l)
        B = B.sum(axis=ax)
        lb.pop(ax)
    shared = [l for l in la if l in lb]
    batch = [l for l in shared if l in keep]
    summed = [l for l in shared if l not in keep]
    fa = [l for l in la if l not in lb]
    fb = [l for l in lb if l not in la]
    dim = {}
    for l, s in zip(la, A.shape):
        dim[l] = s
    for l, s in zip(lb, B.shape):
        if l in dim and dim[l] != s:
            raise ValueError("dimension mismatch on label %r" % (l,))
        dim[l] = s
    At = np.transpose(A, [la.index(l) for l in batch + fa + summed])
    Bt = np.transpose(B, [lb.index(l) for l in batch + summed + fb])
    nb = int(np.prod([dim[l] for l in batch])) if batch else 1
    m = int(np.prod([dim[l] for l in fa])) if fa else 1
    k = int(np.prod([dim[l] for l in summed])) if summed else 1
    nn = int(np.prod([dim[l] for l in fb])) if fb else 1
    C = np.matmul(At.reshape(nb, m, k), Bt.reshape(nb, k, nn))
    lc = batch + fa + fb
    return C.reshape([dim[l] for l in lc]), lc


def _restrict(pieces, fixed):
    out = []
    for arr, ls, tag in pieces:
        idx = []
        nl = []
        for l in ls:
            if l in fixed:
                idx.append(fixed[l])
            else:
                idx.append(slice(None))
                nl.append(l)
        out.append([arr[tuple(idx)], nl, tag])
    return out


def _contract_group(items, outside_counts):
    """Contract a list of (array, labels) into one tensor, keeping labels
    that appear in ``outside_counts`` (tensors outside the group)."""
    items = [list(x) for x in items]
    while len(items) > 1:
        cnt = _counts([ls for _, ls in items])
        best = None
        for i in range(len(items)):
            for j in range(i + 1, len(items)):
                la, lb = items[i][1], items[j][1]
                if not (set(la) & set(lb)) and best is not None:
                    continue
                u = set(la) | set(lb)
                res = [l for l in u if outside_counts.get(l, 0) > 0 or
                       cnt[l] - (l in la) - (l in lb) > 0]
                key = (len(res), len(u), i, j)
                if best is None or key < best[0]:
                    best = (key, i, j)
        _, i, j = best
        keep = set(l for l in set(items[i][1]) | set(items[j][1])
                   if outside_counts.get(l, 0) > 0 or
                   cnt[l] - (l in items[i][1]) - (l in items[j][1]) > 0)
        C, lc = contract_pair(items[i][0], items[i][1], items[j][0], items[j][1], keep)
        items = [items[k] for k in range(len(items)) if k not in (i, j)] + [[C, lc]]
    arr, ls = items[0]
    # sum any label nobody else needs
    for l in [l for l in ls if outside_counts.get(l, 0) == 0]:
        ax = ls.index(l)
        arr = arr.sum(axis=ax)
        ls = ls[:ax] + ls[ax + 1:]
    return arr, ls


def _evaluate(pieces, order):
    if order is None:
        arr, ls = _contract_group([(a, l) for a, l, _ in pieces], {})
        return complex(arr.reshape(-1)[0]) if arr.size == 1 else complex(arr.sum())
    leaves = order["leaves"]
    steps = order["steps"]
    by_tag = {}
    for a, l, t in pieces:
        by_tag.setdefault(t, []).append((a, l))
    assigned = set()
    groups = []
    for leaf in leaves:
        grp = []
        for g in leaf:
            if g in assigned:
                raise ValueError("gate %d in two leaves" % g)
            assigned.add(g)
            grp += by_tag.get(g, [])
        groups.append(grp)
    missing = set(by_tag) - assigned
    if missing:
        raise ValueError("gates not covered by the imported leaves: %s" % sorted(missing)[:10])
    # leaf tensors: keep labels used by pieces in other groups
    all_counts = _counts([l for _, l, _ in pieces])
    live = {}
    for i, grp in enumerate(groups):
        inside = _counts([l for _, l in grp])
        outside = {l: all_counts[l] - inside.get(l, 0) for l in inside}
        outside = {l: c for l, c in outside.items() if c > 0}
        if grp:
            live[i] = _contract_group(grp, outside)
        else:
            live[i] = (np.array(1.0 + 0j), [])
    nid = len(groups)
    for a, b in steps:
        A, la = live.pop(a)
        B, lb = live.pop(b)
        others = _counts([l for _, l in live.values()])
        keep = set(l for l in set(la) | set(lb) if others.get(l, 0) > 0)
        live[nid] = contract_pair(A, la, B, lb, keep)
        nid += 1
    if len(live) != 1:
        raise ValueError("imported order leaves %d tensors" % len(live))
    (arr, ls), = live.values()
    if ls:
        arr = arr.sum()
    return complex(np.asarray(arr).reshape(-1)[0])


def pairwise_amplitude(circ, word, order=None, sliced=(), diagonal_hyperedges=True):
    """<x|C|0> by pairwise contraction.  ``order``: None for the oracle's own
    greedy, or {"leaves": [[gate indices]], "steps": [[a, b]]} where step ids
    count leaves first, then step results.  ``sliced``: (qubit, gate) wires
    fixed slice by slice."""
    net = OracleNetwork(circ, word, diagonal_hyperedges)
    if net.const == 0:
        return 0j
    labels = net.labels_of_slice_spec(list(sliced))
    if len(set(labels)) != len(labels):
        raise ValueError("sliced wires coincide")
    total = 0j
    for s in range(1 << len(labels)):
        fixed = {l: (s >> j) & 1 for j, l in enumerate(labels)}
        total += _evaluate(_restrict(net.pieces, fixed), order)
    return net.const * total


def pairwise_amplitudes(circ, words, order=None, sliced=(), diagonal_hyperedges=True):
    return np.array([pairwise_amplitude(circ, w, order, sliced, diagonal_hyperedges)
                     for w in words], dtype=np.complex128)
