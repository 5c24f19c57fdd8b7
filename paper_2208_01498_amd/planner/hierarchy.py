"""Separator hierarchy -> binary contraction tree (proof of Theorem 1 and the
supplemental section on the numerical implementation).

* A cluster of leaves is split by a sphere separator S (Algorithm 1); the
  cut leaves Gamma_O(S) are each given to the side with which they share
  index dimension of larger total (log2) size; ties go to the side with
  fewer leaves, then to the inner side.
* Splitting recurses until clusters are of constant size; each bottom
  cluster is contracted with a greedy order (smallest result first, then
  fewest multiplications, then lowest ids).
* Above the bottom, the hierarchy fixes the pairwise order: the two halves
  T_{..0} and T_{..1} of every split are merged, and a merge over the union
  of both halves' indices costs the product of their dimensions (Eq. (3)).

Candidate separators at each split are Algorithm 1's random great circles
and (unless separators="ssa") the median coordinate hyperplanes; among
candidates that satisfy the balance condition Eq. (2), the one whose merge
has the smallest index union is kept (the paper accepts the first candidate
passing Eqs. (1)-(2)).  When all leaves of a cluster sit at one or two
points of the time-collapsed embedding (one qubit's world line), no sphere
separates them, and the cluster is split at the median gate index instead.
`split_sources` counts where each kept split came from.
"""
import math
import numpy as np

from .ssa import ssa_candidates, plane_candidates, classify, eq_checks, max_overlap


class Node:
    __slots__ = ("left", "right", "leaf", "labels", "leaves")

    def __init__(self, left=None, right=None, leaf=None, labels=None, leaves=None):
        self.left, self.right, self.leaf = left, right, leaf
        self.labels = labels
        self.leaves = leaves


class TreeBuilder:
    def __init__(self, net, rng, bottom=8, n_circles=24, radius=0.26, centerpoint="radon",
                 separators="ssa+planes"):
        self.net = net
        self.centerpoint = centerpoint
        # candidate separators per split: Algorithm 1's spheres and great
        # circles ("ssa"), plus the median coordinate hyperplanes
        # ("ssa+planes"); the split source of every kept split is counted
        self.separators = separators
        self.split_sources = {"ssa": 0, "ssa_eq1": 0, "plane": 0, "time": 0}
        self.rng = rng
        self.bottom = bottom
        self.n_circles = n_circles
        self.radius = radius
        self.facs = net.factors
        self.users = net.label_users()
        self.bits = {l: math.log2(lab.dim) if lab.kind != "out" else 0.0
                     for l, lab in net.labels.items()}
        self.is_out = {l: lab.kind == "out" for l, lab in net.labels.items()}
        self.tmin = [min(f.gates) if f.gates else 0 for f in self.facs]

    # label bookkeeping -------------------------------------------------
    def ext_labels(self, leafset, cand):
        out = set()
        for l in cand:
            if self.is_out[l] or not self.users[l] <= leafset:
                out.add(l)
        return out

    def leaf_node(self, i):
        s = frozenset([i])
        return Node(leaf=i, labels=self.ext_labels(s, self.facs[i].labels), leaves=s)

    def merge(self, a, b):
        s = a.leaves | b.leaves
        return Node(a, b, labels=self.ext_labels(s, a.labels | b.labels), leaves=s)

    def lbits(self, labels):
        return sum(self.bits[l] for l in labels)

    # bottom clusters ----------------------------------------------------
    def greedy(self, nodes, alpha=1.0):
        """Greedy pairwise order inside a bottom cluster: repeatedly merge
        the pair of neighbouring tensors with the smallest
        size(result) - alpha * (size(a) + size(b)), ties by the size of the
        index union (the step's cost), then by position."""
        nodes = {k: nd for k, nd in enumerate(nodes)}
        nxt = len(nodes)
        while len(nodes) > 1:
            where = {}
            for k, nd in nodes.items():
                for l in nd.labels:
                    where.setdefault(l, []).append(k)
            pairs = set()
            for ks in where.values():
                for x in range(len(ks)):
                    for y in range(x + 1, len(ks)):
                        pairs.add((min(ks[x], ks[y]), max(ks[x], ks[y])))
            if not pairs:
                ks = sorted(nodes)
                pairs = {(ks[0], ks[1])}
            best = None
            for a, b in pairs:
                A, B = nodes[a], nodes[b]
                m = self.merge(A, B)
                sz = 2.0 ** self.lbits(m.labels) - alpha * (2.0 ** self.lbits(A.labels) + 2.0 ** self.lbits(B.labels))
                key = (sz, self.lbits(A.labels | B.labels), a, b)
                if best is None or key < best[0]:
                    best = (key, a, b, m)
            _, a, b, m = best
            del nodes[a]
            del nodes[b]
            nodes[nxt] = m
            nxt += 1
        return next(iter(nodes.values()))

    # splitting ----------------------------------------------------------
    def assign(self, idx, side, pts):
        """Give the cut leaves Gamma_O to the side they share more index size
        with.  Leaves whose spheres coincide (the same point of the
        time-collapsed embedding) are one geometric object and are assigned
        together, by their summed affinity."""
        side = side.copy()
        pos_of = {int(i): k for k, i in enumerate(idx)}
        groups = {}
        for k in range(len(idx)):
            if side[k] == 0:
                groups.setdefault(tuple(np.round(pts[k], 6)), []).append(k)
        nE = int(np.sum(side == 1))
        nI = int(np.sum(side == -1))
        pending = set(groups)
        while pending:
            best = None
            for gkey in pending:
                members = groups[gkey]
                mset = set(int(idx[k]) for k in members)
                w = {1: 0.0, -1: 0.0}
                for k in members:
                    i = int(idx[k])
                    for l in self.facs[i].labels:
                        sides = set()
                        for u in self.users[l]:
                            if u in mset:
                                continue
                            kk = pos_of.get(u)
                            if kk is not None and side[kk] != 0:
                                sides.add(int(side[kk]))
                        for s_ in sides:
                            w[s_] += self.bits[l]
                key = (-max(w[1], w[-1]), gkey)
                if best is None or key < best[0]:
                    best = (key, gkey, w)
            _, gkey, w = best
            if w[1] > w[-1]:
                s_ = 1
            elif w[-1] > w[1]:
                s_ = -1
            else:
                s_ = 1 if nE < nI else -1
            for k in groups[gkey]:
                side[k] = s_
            if s_ == 1:
                nE += len(groups[gkey])
            else:
                nI += len(groups[gkey])
            pending.discard(gkey)
        return side

    def split_score(self, idx, side):
        A = frozenset(int(i) for i, s in zip(idx, side) if s == 1)
        B = frozenset(int(i) for i, s in zip(idx, side) if s == -1)
        if not A or not B:
            return None
        la = set()
        for i in A:
            la.update(self.facs[i].labels)
        lb = set()
        for i in B:
            lb.update(self.facs[i].labels)
        ea = self.ext_labels(A, la)
        eb = self.ext_labels(B, lb)
        merge_bits = self.lbits(ea | eb)
        bal = max(len(A), len(B)) / (len(A) + len(B))
        child = max(self.lbits(ea), self.lbits(eb))
        return (merge_bits + 0.5 * child + 4.0 * max(0.0, bal - 0.6), A, B)

    def time_split(self, idx):
        order = sorted(idx, key=lambda i: (self.tmin[i], i))
        best = None
        n = len(order)
        for cut in range(max(1, n // 3), min(n - 1, 2 * n // 3) + 1):
            side = np.array([1 if k < cut else -1 for k in range(n)])
            sc = self.split_score(np.array(order), side)
            if sc and (best is None or sc[0] < best[0]):
                best = sc
        return best[1], best[2]

    def components(self, idx):
        """Connected components of the leaves `idx` (leaves sharing a
        contracted label are connected; output labels connect nothing)."""
        parent = {i: i for i in idx}

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        for l, us in self.users.items():
            if self.is_out[l]:
                continue
            us = [u for u in us if u in parent]
            for u in us[1:]:
                ra, rb = find(us[0]), find(u)
                if ra != rb:
                    parent[ra] = rb
        comps = {}
        for i in idx:
            comps.setdefault(find(i), []).append(i)
        return sorted(comps.values(), key=min)

    def component_groups(self):
        """Leaves grouped for separate hierarchies: one group per connected
        component larger than a bottom cluster; a small component (say a
        diagonal factor on output labels only) joins a large one that shares
        one of its output labels (else the largest), so that it stays placed
        among its neighbours."""
        comps = self.components(list(range(len(self.facs))))
        big = [c for c in comps if len(c) > self.bottom]
        if len(big) < 2:
            return [sorted(range(len(self.facs)))]
        owner = {}
        for gi, c in enumerate(big):
            for i in c:
                owner[i] = gi
        groups = [list(c) for c in big]
        largest = max(range(len(big)), key=lambda g: len(big[g]))
        for c in comps:
            if len(c) > self.bottom:
                continue
            target = largest
            for i in c:
                for l in self.facs[i].labels:
                    if self.is_out[l]:
                        hit = [owner[u] for u in self.users[l] if u in owner]
                        if hit:
                            target = hit[0]
                            break
                else:
                    continue
                break
            groups[target].extend(c)
        return [sorted(g) for g in groups]

    def build(self, idx=None):
        if idx is None:
            idx = list(range(len(self.facs)))
        idx = list(idx)
        if len(idx) <= self.bottom:
            return self.greedy([self.leaf_node(i) for i in idx])
        pts = np.array([self.facs[i].pos for i in idx])
        uniq = np.unique(np.round(pts, 9), axis=0)
        A = B = None
        if len(uniq) >= 3:
            radii = np.full(len(idx), self.radius)
            d = pts.shape[1]
            k = max_overlap(pts, radii)
            cands = [("ssa", c) for c in ssa_candidates(pts, radii, self.rng, self.n_circles,
                                                        self.centerpoint)]
            if self.separators == "ssa+planes":
                cands += [("plane", c) for c in plane_candidates(pts)]
            best = None
            idx_arr = np.array(idx)
            for src, sep in cands:
                side = classify(sep, pts, radii)
                ok1, ok2 = eq_checks(side, d, k)
                if not ok2:
                    continue
                side = self.assign(idx_arr, side, pts)
                sc = self.split_score(idx_arr, side)
                if sc is None:
                    continue
                key = (0 if ok1 else 1, sc[0])
                if best is None or key < best[0]:
                    best = (key, sc[1], sc[2], src, ok1)
            if best is not None:
                A, B = best[1], best[2]
                self.split_sources[best[3]] += 1
                if best[3] == "ssa" and best[4]:
                    self.split_sources["ssa_eq1"] += 1
        if A is None:
            A, B = self.time_split(idx)
            self.split_sources["time"] += 1
        left = self.build(sorted(A))
        right = self.build(sorted(B))
        return self.merge(left, right)


def tree_steps(root, n_leaves):
    """Post-order list of (a, b) with leaves 0..n_leaves-1 and step results
    numbered from n_leaves in order."""
    steps = []
    counter = [n_leaves]

    def rec(node):
        if node.leaf is not None:
            return node.leaf
        a = rec(node.left)
        b = rec(node.right)
        steps.append((a, b))
        cid = counter[0]
        counter[0] += 1
        return cid

    if root.leaf is not None:
        return steps
    rec(root)
    return steps
