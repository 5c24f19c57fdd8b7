"""Index slicing (the paper names slicing as a technique to combine with its
orders; the choice of indices here is this planner's own).

Fixing a label to each of its values splits the amplitude into 2^S exactly
summed terms ("slices") and removes the label from every tensor.  For a fixed
tree, a step whose subtree holds no sliced label is the same in every slice
and is computed once ("hoisted"); every other step runs once per slice with
its sliced labels removed.  The greedy below adds, one label at a time, the
wire label that minimises the total multiplications under this model,
preferring labels that shrink the largest per-slice intermediate while it is
above the target.
"""
import math


class SliceModel:
    def __init__(self, net, steps, B=1, peak_flops=157.3e12 * 0.6, peak_bw=8.0e12 * 0.6,
                 launch=4e-6, objective="time", blocked=True, width_with_batch=True):
        self.net = net
        self.steps = steps
        self.B = B
        # the width a target is compared with: log2 elements of the widest
        # per-slice tensor with its bitstring batch, or per bitstring (the
        # executor then runs the batch in chunks that fit the arena)
        self.width_with_batch = width_with_batch
        self.blocked = blocked
        self.peak_flops, self.peak_bw, self.launch = peak_flops, peak_bw, launch
        self.objective = objective
        self.is_out = {l: lab.kind == "out" for l, lab in net.labels.items()}
        self.bits = {l: math.log2(lab.dim) for l, lab in net.labels.items()}
        nf = len(net.factors)
        live = {}
        hb = {}
        leafl = {}
        for i, f in enumerate(net.factors):
            live[i] = set(l for l in f.labels if not self.is_out[l])
            hb[i] = any(self.is_out[l] for l in f.labels)
            leafl[i] = set(live[i])
        cnt = {}
        for s in live.values():
            for l in s:
                cnt[l] = cnt.get(l, 0) + 1
        self.rec = []          # (union labels, result labels, subtree labels, has_b)
        sub = dict(leafl)
        nid = nf
        for a, b in steps:
            la, lb = live.pop(a), live.pop(b)
            u = la | lb
            lc = set(l for l in u if cnt[l] - (l in la) - (l in lb) > 0)
            for l in la:
                cnt[l] -= 1
            for l in lb:
                cnt[l] -= 1
            for l in lc:
                cnt[l] += 1
            ha, hbb = hb.pop(a), hb.pop(b)
            hc = ha or hbb
            st = sub.pop(a) | sub.pop(b)
            self.rec.append((frozenset(u), frozenset(lc), frozenset(st), hc,
                             frozenset(la), frozenset(lb), ha, hbb))
            live[nid] = lc
            hb[nid] = hc
            sub[nid] = st
            nid += 1
        # candidates: labels of the widest intermediates and of the costliest
        # steps (slicing anything else cannot help)
        wmax = max((sum(self.bits[l] for l in r[1]) for r in self.rec), default=0)
        umax = max((sum(self.bits[l] for l in r[0]) for r in self.rec), default=0)
        cand = set()
        for r in self.rec:
            u, lc = r[0], r[1]
            if sum(self.bits[l] for l in lc) >= wmax - 6 or sum(self.bits[l] for l in u) >= umax - 3:
                cand |= set(lc) | set(u)
        self.candidates = sorted(cand)

    def order_bits(self, sliced):
        """Bit positions for the sliced labels: slice s gives label j the
        value of bit j of s.  Walking s upwards, bit j flips 2^(S-j) times,
        so a step whose subtree holds sliced labels D is recomputed
        2^(S - min bit of D) times and otherwise reuses its last result.
        Labels whose dependent steps cost least get the low bits."""
        S = list(sliced)
        dep = {l: 0.0 for l in S}
        for r in self.rec:
            u, lc, st, hc = r[:4]
            hit = st & set(S)
            if hit:
                ub = sum(self.bits[x] for x in u if x not in set(S))
                c = 2.0 ** ub * (self.B if hc else 1)
                for l in hit:
                    dep[l] += c
        return sorted(S, key=lambda l: (dep[l], l))

    def evaluate(self, sliced, ordered=False):
        """(total flops over all slices with reuse, widest per-slice tensor in
        log2 elements, including the batch unless width_with_batch is off)."""
        S = list(sliced) if ordered else self.order_bits(sliced)
        pos = {l: j for j, l in enumerate(S)}
        Sset = set(S)
        nS = len(S)
        total = 0.0
        width = 0.0
        self.last_flops = 0.0
        for u, lc, st, hc, la, lb, ha, hb in self.rec:
            bsz = self.B if hc else 1
            hit = [pos[l] for l in st if l in Sset]
            ub = sum(self.bits[l] for l in u if l not in Sset)
            cb = sum(self.bits[l] for l in lc if l not in Sset)
            f = 8.0 * 2.0 ** ub * bsz
            if self.objective == "oracle":
                # every step of every slice, no reuse (the CPU oracle)
                reps = 2.0 ** nS
            elif self.blocked:
                # all slices in one pass: one copy per value of the sliced
                # labels in the step's subtree
                reps = 2.0 ** len(hit)
            else:
                reps = 2.0 ** (nS - min(hit)) if hit else 1.0
            self.last_flops += f * reps
            if self.objective == "time":
                ab = sum(self.bits[l] for l in la if l not in Sset)
                bbits = sum(self.bits[l] for l in lb if l not in Sset)
                byt = 8.0 * (2.0 ** ab * (self.B if ha else 1) + 2.0 ** bbits * (self.B if hb else 1)
                             + 2.0 ** cb * bsz)
                if self.blocked:
                    total += max(reps * f / self.peak_flops, reps * byt / self.peak_bw) + self.launch
                else:
                    total += reps * (max(f / self.peak_flops, byt / self.peak_bw) + self.launch)
            else:
                total += f * reps
            width = max(width, cb + (math.log2(bsz) if self.width_with_batch else 0.0))
        return total, width

    def greedy(self, n_slices=None, target_width=None, max_slices=30):
        chosen = []
        cur_total, cur_width = self.evaluate(chosen)
        while True:
            if n_slices is not None and len(chosen) >= n_slices:
                break
            if n_slices is None and (target_width is None or cur_width <= target_width):
                break
            if len(chosen) >= max_slices:
                break
            best = None
            for l in self.candidates:
                if l in chosen:
                    continue
                t, w = self.evaluate(chosen + [l])
                over = target_width is not None and cur_width > target_width
                key = (w if over else 0.0, t, w, l)
                if best is None or key < best[0]:
                    best = (key, l, t, w)
            if best is None:
                break
            chosen.append(best[1])
            cur_total, cur_width = best[2], best[3]
        chosen = self.order_bits(chosen)
        return chosen, cur_total, cur_width
