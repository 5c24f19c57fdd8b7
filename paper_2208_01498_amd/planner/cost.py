"""Cost accounting of a pairwise contraction sequence (Eq. (3)).

A step contracting A and B multiplies entries over the union of both index
sets: prod_{i in idx(A) u idx(B)} dim(i) complex multiplications and at most
as many additions; with complex scalars one multiply-add is 8 real flops, so
a step costs 8 * prod dims real flops.  The bitstring batch b counts as an
index of size B wherever it appears (it is never summed).
"""
import math


class CostModel:
    """Roofline estimate of a step on MI355X: max(flops / MFMA peak,
    bytes / HBM peak), with the FP32 MFMA peak derated by ``eff``."""

    def __init__(self, peak_flops=157.3e12, peak_bw=8.0e12, eff=0.6, launch=4e-6):
        self.peak_flops, self.peak_bw, self.eff, self.launch = peak_flops, peak_bw, eff, launch

    def step_time(self, flops, bytes_):
        return max(flops / (self.peak_flops * self.eff), bytes_ / self.peak_bw) + self.launch


def plan_stats(net, steps, sliced=(), B=1):
    """Flops, largest intermediate and bytes of the step list, per slice."""
    sliced = set(sliced)
    is_out = {l: lab.kind == "out" for l, lab in net.labels.items()}
    bits = {l: math.log2(lab.dim) for l, lab in net.labels.items()}
    live = {}
    hb = {}
    for i, f in enumerate(net.factors):
        live[i] = set(l for l in f.labels if not is_out[l] and l not in sliced)
        hb[i] = any(is_out[l] for l in f.labels)
    cnt = {}
    for s in live.values():
        for l in s:
            cnt[l] = cnt.get(l, 0) + 1
    flops = 0.0
    max_bits = 0.0
    max_elems = 0.0
    nid = len(net.factors)
    per_step = []
    for a, b in steps:
        la, lb = live.pop(a), live.pop(b)
        ha, hbb = hb.pop(a), hb.pop(b)
        u = la | lb
        lc = set(l for l in u if cnt[l] - (l in la) - (l in lb) > 0)
        for l in la:
            cnt[l] -= 1
        for l in lb:
            cnt[l] -= 1
        for l in lc:
            cnt[l] += 1
        hc = ha or hbb
        ub = sum(bits[l] for l in u)
        f = 8.0 * 2.0 ** ub * (B if hc else 1)
        cb = sum(bits[l] for l in lc)
        flops += f
        max_bits = max(max_bits, cb)
        max_elems = max(max_elems, 2.0 ** cb * (B if hc else 1))
        live[nid] = lc
        hb[nid] = hc
        per_step.append((a, b, nid, ub, cb, ha, hbb, hc, f))
        nid += 1
    return dict(flops=flops, log2_flops=math.log2(flops) if flops else 0.0,
                max_bits=max_bits, max_elems=max_elems, steps=per_step)
