"""Plan builder: circuit -> network -> separator hierarchy -> steps -> slices
-> layout -> TNP1 blob.

TNP1 (little-endian; every integer u32 unless noted):
  header   "TNP1", version=1, n_qubits, n_labels, n_leaves, n_steps,
           n_sliced, flags, scale (2 x f64: re, im)
  labels   n_labels x {dim u8, kind u8 (0 wire, 1 output), pad u16,
           qubit i32}
  leaves   n_leaves x {rank, labels[rank] (storage order, C order: first
           label most significant), n_mat, mat_order[n_mat], n_gates,
           gate_ids[n_gates], data: 2^rank x (re f64, im f64)}
           mat_order is the order the leaf is gathered into (its labels
           minus output and sliced labels); output labels are replaced by
           the bitstring value of their qubit (giving the batch index b),
           sliced labels by the slice's bit.
  sliced   n_sliced label ids; slice s gives sliced label j bit j of s
  steps    n_steps x {a, b, nA, permA[nA], nB, permB[nB], nC, c_order[nC]}
           operand ids count leaves first, then step results in order;
           nA = 0 means A is used as stored, else A is first permuted to
           permA (same for B); C is written in c_order
  meta     n_meta, n_meta x f64 (flops per slice per bitstring, log2 width,
           ...)
"""
import math
import struct

import numpy as np

from .network import build_network
from .hierarchy import TreeBuilder, tree_steps
from .toporder import refine_top
from .slicer import SliceModel
from .layout import Layout
from .cost import plan_stats

MAGIC = b"TNP1"
VERSION = 1


class Plan:
    def __init__(self, circ, net, steps, sliced, leaf_order, step_layout, stats, options):
        self.circ = circ
        self.net = net
        self.steps = steps
        self.sliced = sliced
        self.leaf_order = leaf_order
        self.step_layout = step_layout
        self.stats = stats
        self.options = options

    @property
    def n_slices(self):
        return 1 << len(self.sliced)

    def order_spec(self):
        """The contraction order as data for an independent evaluator: leaves
        as gate-index sets, steps as id pairs, sliced wires as (qubit, gate
        that starts the wire)."""
        leaves = [sorted(int(g) for g in f.gates) for f in self.net.factors]
        sl = [(self.net.labels[l].qubit, self.net.labels[l].gate) for l in self.sliced]
        return {"leaves": leaves, "steps": [[int(a), int(b)] for a, b in self.steps],
                "sliced": sl}

    def to_blob(self):
        net = self.net
        used = sorted(set(l for f in net.factors for l in f.labels))
        remap = {l: i for i, l in enumerate(used)}
        out = bytearray()
        out += MAGIC
        flags = 1 if getattr(net, "doubled", False) else 0
        out += struct.pack("<7I", VERSION, net.n_qubits, len(used), len(net.factors),
                           len(self.steps), len(self.sliced), flags)
        out += struct.pack("<2d", net.scale.real, net.scale.imag)
        for l in used:
            lab = net.labels[l]
            out += struct.pack("<BBHi", lab.dim, 1 if lab.kind == "out" else 0, 0,
                               lab.qubit)
        for i, f in enumerate(net.factors):
            out += struct.pack("<I", len(f.labels))
            out += struct.pack("<%dI" % len(f.labels), *[remap[l] for l in f.labels])
            mo = self.leaf_order[i]
            out += struct.pack("<I", len(mo))
            out += struct.pack("<%dI" % len(mo), *[remap[l] for l in mo])
            gs = sorted(f.gates)
            out += struct.pack("<I", len(gs))
            out += struct.pack("<%dI" % len(gs), *gs)
            d = np.ascontiguousarray(f.data, dtype=np.complex128).reshape(-1)
            out += d.view(np.float64).astype("<f8").tobytes()
        out += struct.pack("<%dI" % len(self.sliced), *[remap[l] for l in self.sliced])
        for st in self.step_layout:
            out += struct.pack("<2I", st["a"], st["b"])
            for key in ("permA", "permB"):
                p = st[key] or []
                out += struct.pack("<I", len(p))
                out += struct.pack("<%dI" % len(p), *[remap[l] for l in p])
            oc = st["c_order"]
            out += struct.pack("<I", len(oc))
            out += struct.pack("<%dI" % len(oc), *[remap[l] for l in oc])
        meta = [self.stats["flops_per_b"], self.stats["max_bits"], float(len(self.sliced)),
                self.stats["total_flops_per_b"]]
        out += struct.pack("<I", len(meta))
        out += struct.pack("<%dd" % len(meta), *meta)
        return bytes(out)


def make_plan(circ, n_slices=0, target_width=None, B=1, bottom=40, seed=0,
              n_circles=24, trials=3, objective="time", coarsen=0, projector=None,
              top_exact=13, centerpoint="lp", width_per_bitstring=False,
              separators="ssa+planes", svd_split=False):
    """Build a plan.  ``n_slices``: number of sliced labels (log2 of the slice
    count), or None to slice until the widest per-slice intermediate is at
    most ``target_width`` (log2 elements, batch included; per bitstring with
    ``width_per_bitstring``, when the batch runs in chunks).  ``projector``:
    None for amplitudes <x|C|0>; otherwise the set of traced qubits of the
    projector quantity <0|C^dag (x)_q P_q C|0> (P_q = |x_q><x_q| elsewhere).
    ``top_exact``: size of the frontier below the root whose pairwise order
    is chosen exactly (0 keeps the hierarchy's order everywhere).
    ``centerpoint``: Algorithm 1's centerpoint by the LP over a random
    subset ("lp", the paper's route) or by iterated Radon points ("radon").
    ``separators``: the candidates of each split of the hierarchy:
    Algorithm 1's spheres plus median coordinate hyperplanes
    ("ssa+planes"), Algorithm 1's alone ("ssa"), or the planar separator of
    the qubit graph ("planar", see planar.py).  The kept plan's
    ``stats["split_sources"]`` counts where its splits came from.
    ``svd_split``: the paper-faithful network of the proof of Theorem 2
    (rank-3 SVD halves of every two-qubit gate, no diagonal hyperedges)."""
    from .network import _is_swap_diag, build_doubled_network
    forms = [False]
    if not svd_split and any(len(g.qubits) == 2 and _is_swap_diag(g.matrix) for g in circ.gates):
        forms.append(True)
    do_slice = bool(n_slices) or target_width is not None
    best = None
    for swap_relabel in forms:
        if projector is None:
            net = build_network(circ, swap_relabel=swap_relabel, coarsen=coarsen,
                                svd_split=svd_split)
        else:
            net = build_doubled_network(circ, traced=projector, swap_relabel=swap_relabel)
        for t in range(trials):
            if separators == "planar":
                from .planar import PlanarTreeBuilder
                tb = PlanarTreeBuilder(net, np.random.Generator(np.random.PCG64(seed + t)),
                                       bottom=bottom)
            else:
                tb = TreeBuilder(net, np.random.Generator(np.random.PCG64(seed + t)),
                                 bottom=bottom, n_circles=n_circles, centerpoint=centerpoint,
                                 separators=separators)
            # a network that falls apart (the two layers of a doubled
            # network with every qubit projected) gets one hierarchy and one
            # exact top order per component; component results multiply last
            base = [tb.build(grp) for grp in tb.component_groups()]
            # The exact top order weighs merges without a bitstring index by
            # 1/B.  Under a width cap a large B makes those merges look free
            # and their wide results are then sliced at a cost the order did
            # not see, so a cap with a batch above 8 also tries the weight 8;
            # every candidate is costed at the real B below.
            weights = [B] + ([8] if target_width is not None and B > 8 and top_exact else [])
            for wB in weights:
                roots = [refine_top(r, tb, B=wB, frontier=top_exact) if top_exact else r
                         for r in base]
                root = roots[0] if len(roots) == 1 else tb.greedy(roots)
                steps = tree_steps(root, len(net.factors))
                # Trials compete on the cost that is actually executed: the
                # summed cost over all slices when slicing is asked for, the
                # unsliced Eq. (3) cost otherwise.
                sliced, sm = [], None
                if steps:
                    sm = SliceModel(net, steps, B=B, objective=objective,
                                    width_with_batch=not width_per_bitstring)
                    if do_slice:
                        sliced, _, _ = sm.greedy(n_slices=n_slices if n_slices else None,
                                                 target_width=target_width)
                    cost = sm.evaluate(sliced, ordered=True)[0]
                else:
                    cost = plan_stats(net, steps, B=1)["flops"]
                if best is None or cost < best[0]:
                    best = (cost, steps, net, sliced, sm, dict(tb.split_sources))
    _, steps, net, sliced, sm, sources = best
    total = None
    predicted = None
    if sm is not None:
        predicted, _ = sm.evaluate(sliced, ordered=True)
        total = sm.last_flops
    lay = Layout(net, steps, sliced)
    leaf_order, step_layout = lay.run()
    st = plan_stats(net, steps, sliced=sliced, B=1)
    if total is None:
        total = st["flops"] * (1 << len(sliced))
    stats = dict(flops_per_b=st["flops"], max_bits=st["max_bits"],
                 total_flops_per_b=(total / B) if total else st["flops"],
                 predicted=predicted,
                 permute_elems=lay.permute_elems, n_leaves=len(net.factors),
                 n_steps=len(steps), split_sources=sources)
    return Plan(circ, net, steps, sliced, leaf_order, step_layout, stats,
                dict(n_slices=n_slices, target_width=target_width, B=B, bottom=bottom,
                     seed=seed, width_per_bitstring=width_per_bitstring))
