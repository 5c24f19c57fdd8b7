"""Exact pairwise order for the top of a contraction tree.

The separator hierarchy fixes the order of every merge above its bottom
clusters.  Near the root those merges join a handful of large subtrees, and
their cost (Eq. (3): a merge over index union U costs 8 * prod dim(U) real
flops) dominates the whole contraction.  Here the root is opened into a
frontier of F subtrees (repeatedly replacing the frontier node whose own
merge is the most expensive by its two children), and the best pairwise
order of the frontier is found by dynamic programming over its 2^F subsets;
the subtrees below the frontier keep the hierarchy's order.  Merges whose
result carries no bitstring index are weighted by 1/B (computed once per
batch of B bitstrings), as in the executor.
"""


def _popcount(x):
    return bin(x).count("1")


def refine_top(root, tb, B=1, frontier=13):
    """Return a tree whose top is the cheapest order of a frontier of at
    most `frontier` subtrees of `root` (TreeBuilder nodes, merged with
    tb.merge).  The tree below the frontier is unchanged."""
    if root.leaf is not None or frontier < 3:
        return root
    is_out = tb.is_out

    def has_b(node):
        return any(is_out[l] for l in node.labels)

    def step_cost(a, b, m):
        u = sum(tb.bits[l] for l in (a.labels | b.labels))
        return 8.0 * 2.0 ** u * (1.0 if has_b(m) else 1.0 / B)

    def own(node):
        return step_cost(node.left, node.right, node)

    front = [root]
    while len(front) < frontier:
        inner = [n for n in front if n.leaf is None]
        if not inner:
            break
        n = max(inner, key=own)
        front.remove(n)
        front += [n.left, n.right]
    K = len(front)
    if K < 3:
        return root
    # label bit masks over the frontier's summed labels
    ids = {}
    masks = []
    for n in front:
        m = 0
        for l in n.labels:
            if not is_out[l] and tb.bits[l] > 0:
                if l not in ids:
                    ids[l] = len(ids)
                m |= 1 << ids[l]
        masks.append(m)
    bflag = [has_b(n) for n in front]
    full = (1 << K) - 1
    union = [0] * (1 << K)
    hb = [False] * (1 << K)
    for s in range(1, 1 << K):
        low = s & -s
        i = low.bit_length() - 1
        union[s] = union[s ^ low] | masks[i]
        hb[s] = hb[s ^ low] or bflag[i]
    res = [0] * (1 << K)
    for s in range(1, 1 << K):
        res[s] = union[s] & union[full ^ s]
    best = [0.0] * (1 << K)
    split = [0] * (1 << K)
    order = sorted(range(1, 1 << K), key=_popcount)
    for s in order:
        if s & (s - 1) == 0:
            continue
        w = 1.0 if hb[s] else 1.0 / B
        bc = None
        sub = (s - 1) & s
        while sub:
            o = s ^ sub
            if sub < o:
                c = best[sub] + best[o] + w * 8.0 * 2.0 ** _popcount(res[sub] | res[o])
                if bc is None or c < bc:
                    bc = c
                    split[s] = sub
            sub = (sub - 1) & s
        best[s] = bc

    def build(s):
        if s & (s - 1) == 0:
            return front[s.bit_length() - 1]
        a = split[s]
        return tb.merge(build(a), build(s ^ a))

    return build(full)
