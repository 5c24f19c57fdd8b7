"""Hierarchy from planar separators (the Planar Separator Theorem passage
after Theorem 1: a planar graph on n vertices splits into parts of at most
2n/3 vertices by removing O(sqrt(n)) of them).

For a two-dimensional circuit the paper applies the theorem to the
time-collapsed network: the tensors of qubit i all sit at its site x_i
(displaced by a vanishing epsilon'), and crossing vertices make the drawing
planar.  A separator of that planar graph cuts whole world lines, so here
the separator of a cluster is a set of qubits.  Its qubit graph (qubits
adjacent when a leaf of the cluster carries labels of both) is searched
breadth first from a pseudo-peripheral qubit, the first phase of the
Lipton-Tarjan construction: every BFS level separates the qubits before it
from those after it.  Among the levels that leave at most 2n/3 of the
cluster's leaves on either side (a leaf is on a side when all its qubits
are), the one whose leaves carry the fewest label bits is the separator; on
a lattice these levels are the anti-diagonal fronts of the search, of size
O(sqrt(N)) qubits.  The separator's leaves are given to the side they share
more index size with, as for the sphere separators.  The Lipton-Tarjan
cycle phase (for a middle part heavier than 2n/3) is not built: such a
cluster takes its most balanced level.  A cluster on fewer than three
levels of qubits (one world line, or two neighbours) is split at the median
gate index.
"""
from collections import deque

import numpy as np

from .hierarchy import TreeBuilder


class PlanarTreeBuilder(TreeBuilder):
    def __init__(self, net, rng, bottom=8):
        super().__init__(net, rng, bottom=bottom)
        self.split_sources = {"planar": 0, "planar_unbalanced": 0, "time": 0}

    def _qubits(self, i):
        return {self.net.labels[l].qubit for l in self.facs[i].labels}

    @staticmethod
    def _bfs(adj, src):
        dist = {src: 0}
        q = deque([src])
        while q:
            x = q.popleft()
            for y in sorted(adj[x]):
                if y not in dist:
                    dist[y] = dist[x] + 1
                    q.append(y)
        return dist

    def level_split(self, idx):
        """(inner side, outer side, balanced?) from the best BFS level of the
        cluster's qubit graph, or None when it has fewer than three levels."""
        qs = {i: self._qubits(i) for i in idx}
        adj = {}
        for i in idx:
            for a in qs[i]:
                adj.setdefault(a, set()).update(b for b in qs[i] if b != a)
        start = min(adj)
        for _ in range(2):
            d = self._bfs(adj, start)
            far = max(d.values())
            start = min(v for v, x in d.items() if x == far)
        dist = self._bfs(adj, start)
        top = max(dist.values()) + 1
        for a in adj:
            dist.setdefault(a, top)        # another component: one more level
        nlev = max(dist.values()) + 1
        if nlev < 3:
            return None
        lo_lev = {i: min(dist[a] for a in qs[i]) for i in idx}
        hi_lev = {i: max(dist[a] for a in qs[i]) for i in idx}
        n = len(idx)
        best = None
        for l in range(1, nlev - 1):
            before = sum(1 for i in idx if hi_lev[i] < l)
            after = sum(1 for i in idx if lo_lev[i] > l)
            cut = [i for i in idx if lo_lev[i] <= l <= hi_lev[i]]
            balanced = before <= 2 * n / 3 and after <= 2 * n / 3 and before > 0 and after > 0
            bits = sum(self.lbits(self.facs[i].labels) for i in cut)
            key = (0 if balanced else 1, bits if balanced else abs(before - after), l)
            if best is None or key < best[0]:
                best = (key, l, balanced)
        _, l, balanced = best
        idx_arr = np.array(idx)
        side = np.array([1 if hi_lev[i] < l else (-1 if lo_lev[i] > l else 0) for i in idx])
        pts = np.array([self.facs[i].pos for i in idx])
        side = self.assign(idx_arr, side, pts)
        sc = self.split_score(idx_arr, side)
        if sc is None:
            return None
        return sc[1], sc[2], balanced

    def build(self, idx=None):
        if idx is None:
            idx = list(range(len(self.facs)))
        idx = list(idx)
        if len(idx) <= self.bottom:
            return self.greedy([self.leaf_node(i) for i in idx])
        got = self.level_split(idx)
        if got is not None:
            A, B, balanced = got
            self.split_sources["planar" if balanced else "planar_unbalanced"] += 1
        else:
            A, B = self.time_split(idx)
            self.split_sources["time"] += 1
        return self.merge(self.build(sorted(A)), self.build(sorted(B)))
