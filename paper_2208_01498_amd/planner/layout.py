"""Label orders of every tensor, chosen so that each pairwise step runs as
one strided-batched complex GEMM, with index permutations only where an
operand's stored order does not fit.

Order convention: a tensor over labels (l_0, ..., l_{r-1}) stores the entry
with label values v_i at element sum_i v_i * 2^(r-1-i) (C order, l_0 most
significant); a tensor that carries the bitstring batch has b above all
labels.

For a step A x B -> C the labels fall in four classes: batch (in A, B and
still needed later), K (in A and B only: summed), MA (A only), NB (B only).
The GEMM accepts A as [batch][MA][K] or [batch][K][MA], B as [batch][K][NB]
or [batch][NB][K], with the same batch order and K order in both, and writes
C as [batch][MA][NB] or [batch][NB][MA] with MA, NB in their operand orders.
A leaf is gathered into whatever order its first use wants; an intermediate
keeps the order it was written in and is permuted when it does not fit.
"""


def _blocks_ok(order, blocks):
    """order (list) is the concatenation of the label sets in blocks, in that
    block order (inner order free)."""
    pos = 0
    for blk in blocks:
        n = len(blk)
        if set(order[pos:pos + n]) != set(blk):
            return False
        pos += n
    return pos == len(order)


def _sub(order, s):
    return [l for l in order if l in s]


class Layout:
    def __init__(self, net, steps, sliced):
        self.net = net
        self.steps = steps
        self.sliced = set(sliced)
        self.is_out = {l: lab.kind == "out" for l, lab in net.labels.items()}

    def prepass(self):
        """Label set of every tensor and the kept labels of every step."""
        net = self.net
        nf = len(net.factors)
        lab = {}
        for i, f in enumerate(net.factors):
            lab[i] = set(l for l in f.labels if not self.is_out[l] and l not in self.sliced)
        cnt = {}
        for ls in lab.values():
            for l in ls:
                cnt[l] = cnt.get(l, 0) + 1
        self.lab_of = dict(lab)
        self.keep_of = []
        nid = nf
        for a, b in self.steps:
            la, lb = lab.pop(a), lab.pop(b)
            u = la | lb
            keep = set(l for l in u if cnt[l] - (l in la) - (l in lb) > 0)
            for l in la:
                cnt[l] -= 1
            for l in lb:
                cnt[l] -= 1
            for l in keep:
                cnt[l] += 1
            lab[nid] = keep
            self.lab_of[nid] = keep
            self.keep_of.append(keep)
            nid += 1

    def run(self):
        self.prepass()
        net = self.net
        nf = len(net.factors)
        labels = {}
        hasb = {}
        fixed = {}             # tensor id -> order if fixed (intermediates / used leaves)
        for i, f in enumerate(net.factors):
            labels[i] = [l for l in f.labels if not self.is_out[l] and l not in self.sliced]
            hasb[i] = any(self.is_out[l] for l in f.labels)
        cnt = {}
        for ls in labels.values():
            for l in ls:
                cnt[l] = cnt.get(l, 0) + 1
        # parent of each tensor (for look-ahead)
        parent = {}
        nid = nf
        for si, (a, b) in enumerate(self.steps):
            parent[a] = (si, b)
            parent[b] = (si, a)
            nid += 1
        leaf_order = {}
        out = []
        live_labels = dict((k, set(v)) for k, v in labels.items())
        nid = nf
        self.permute_elems = 0.0
        for si, (a, b) in enumerate(self.steps):
            la, lb = live_labels.pop(a), live_labels.pop(b)
            u = la | lb
            keep = set(l for l in u if cnt[l] - (l in la) - (l in lb) > 0)
            for l in la:
                cnt[l] -= 1
            for l in lb:
                cnt[l] -= 1
            batch = la & lb & keep
            K = (la & lb) - keep
            MA = la - lb
            NB = lb - la
            # anchor = operand with a fixed order, larger first
            def size(t, ls):
                return len(ls) + (6 if hasb[t] else 0)
            cand = [(a, la, MA), (b, lb, NB)]
            cand.sort(key=lambda x: (x[0] not in fixed, -size(x[0], x[1])))
            (t1, l1, F1), (t2, l2, F2) = cand
            # orders of the anchor
            permA = permB = None
            if t1 in fixed:
                o1 = fixed[t1]
                if _blocks_ok(o1, [batch, F1, K]) or _blocks_ok(o1, [batch, K, F1]):
                    new1 = None
                else:
                    new1 = self._canonical(o1, batch, F1, K, parent.get(nid))
                    self.permute_elems += 2.0 ** len(l1) * (64 if hasb[t1] else 1)
            else:
                o1 = None
                new1 = None
            fresh = set()        # leaves whose order is chosen at this step
            if o1 is None:
                o1 = self._canonical(None, batch, F1, K, parent.get(nid), l1)
                leaf_order[t1] = o1
                fresh.add(t1)
            elif new1 is not None:
                if t1 == a:
                    permA = new1
                else:
                    permB = new1
                o1 = new1
            bo = _sub(o1, batch)
            ko = _sub(o1, K)
            # second operand must match batch and K orders
            want_kf = bo + ko + self._free_order(F2, None, parent.get(nid))
            if t2 in fixed:
                o2 = fixed[t2]
                if (o2[:len(bo)] == bo and (_sub(o2, K) == ko) and
                        (_blocks_ok(o2, [batch, K, F2]) or _blocks_ok(o2, [batch, F2, K]))):
                    new2 = None
                else:
                    new2 = bo + ko + _sub(o2, F2)
                    self.permute_elems += 2.0 ** len(l2) * (64 if hasb[t2] else 1)
                if new2 is not None:
                    if t2 == a:
                        permA = new2
                    else:
                        permB = new2
                    o2 = new2
            else:
                o2 = want_kf
                leaf_order[t2] = o2
                fresh.add(t2)
            oa, ob = (o1, o2) if t1 == a else (o2, o1)
            ma = _sub(oa, MA)
            nb = _sub(ob, NB)
            # C orientation: prefer the one that fits the parent step
            cands = [bo + ma + nb, bo + nb + ma]
            oc = cands[0]
            pinfo = parent.get(nid)
            if pinfo is not None:
                psi = pinfo[0]
                lc = self.lab_of[nid]
                lsib = self.lab_of[pinfo[1]]
                keep_p = self.keep_of[psi]
                bP = lc & lsib & keep_p
                kP = (lc & lsib) - keep_p
                fP = lc - lsib
                fitted = False
                for o in cands:
                    if _blocks_ok(o, [bP, fP, kP]) or _blocks_ok(o, [bP, kP, fP]):
                        oc = o
                        fitted = True
                        break
                if not fitted:
                    sc = self._scatter(a, b, oa, ob, bo, ma, nb, MA, NB, bP, fP, kP,
                                       fixed, fresh, permA, permB, hasb, len(lc))
                    if sc is not None:
                        oc, oa2, ob2, cost = sc
                        self.permute_elems += cost
                        for t, o_old, o_new in ((a, oa, oa2), (b, ob, ob2)):
                            if o_new == o_old:
                                continue
                            if t in fresh:
                                leaf_order[t] = o_new
                            elif t == a:
                                permA = o_new
                            else:
                                permB = o_new
                        oa, ob = oa2, ob2
            lc = batch | MA | NB
            for l in lc:
                cnt[l] = cnt.get(l, 0) + 1
            live_labels[nid] = lc
            hasb[nid] = hasb[a] or hasb[b]
            fixed[nid] = oc
            fixed[a] = oa
            fixed[b] = ob
            out.append(dict(a=a, b=b, permA=permA, permB=permB, c_order=oc))
            nid += 1
        for i in range(nf):
            if i not in leaf_order:
                leaf_order[i] = labels[i]
        return leaf_order, out

    def _scatter(self, a, b, oa, ob, bo, ma, nb, MA, NB, bP, fP, kP, fixed, fresh,
                 permA, permB, hasb, rank_c):
        """An output order that the parent step can use without a permute,
        written by the GEMM as an interleaving of its row and column index
        bits: C = bo + [bP - bo] + X + Y with {X, Y} = {fP, kP}, the M labels
        in A's order and the N labels in B's order.  A or B is re-sorted
        (stable, by block) when its own order does not list its labels
        block by block; returns None when that costs more than permuting C
        or when the step's batch labels are not all parent batch labels."""
        if not set(bo) <= bP:
            return None
        size = lambda t, n: 2.0 ** n * (64 if hasb[t] else 1)
        c_cost = 2.0 ** rank_c * (64 if (hasb[a] or hasb[b]) else 1)
        best = None
        for X, Y in ((fP, kP), (kP, fP)):
            blocks = [bP - set(bo), X, Y]
            blk = lambda l: next(i for i, s_ in enumerate(blocks) if l in s_)
            ma2 = sorted(ma, key=blk)
            nb2 = sorted(nb, key=blk)
            cost = 0.0
            for t, o, old_sub, new_sub, already in ((a, oa, ma, ma2, permA is not None),
                                                    (b, ob, nb, nb2, permB is not None)):
                if old_sub != new_sub and t not in fresh and not already:
                    cost += size(t, len(o))
            if cost >= c_cost:
                continue
            oc = list(bo)
            for s_ in blocks:
                oc += [l for l in ma2 if l in s_] + [l for l in nb2 if l in s_]
            if best is None or cost < best[3]:
                it = iter(ma2)
                oa2 = [next(it) if l in MA else l for l in oa]
                it = iter(nb2)
                ob2 = [next(it) if l in NB else l for l in ob]
                best = (oc, oa2, ob2, cost)
        return best

    def _free_order(self, F, cur, pinfo):
        return sorted(F)

    def _canonical(self, cur, batch, F, K, pinfo, allowed=None):
        """[batch][F][K] keeping the current relative order where known."""
        def keyed(s):
            if cur is not None:
                return _sub(cur, s)
            return sorted(s)
        return keyed(batch) + keyed(F) + keyed(K)
