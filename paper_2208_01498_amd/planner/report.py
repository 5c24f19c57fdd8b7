"""Counted plan cost next to the paper's bounds, per circuit (host only).

For each circuit: log2 of the scalar operations (multiplications and
additions, the paper's unit: 2 per complex multiply-add of Eq. (3)) of this
planner's plan for one amplitude <x|C|0> and for the paper's own quantity
c = <0|C^dag (x)_q P_q C|0> (the doubled network), next to the Theorem 2
bound, its planar d = 2 form, side-wise contraction and explicit time
evolution (module `bounds`).  This reproduces the method of the paper's
figures (bounds and counted costs as logarithms per family and size) on
single realizations; the paper's figure data and its comparison system are
not used.

Usage: python -m paper_2208_01498_amd.planner.report [--L 4 5 6] [--json]
"""
import argparse
import json
import math

from .bounds import circuit_bounds
from .plan import make_plan


def counted_log2(circ, projector=None, trials=3):
    """log2 of the scalar operations of the plan (FP64 count of Eq. (3))."""
    plan = make_plan(circ, B=1, trials=trials, projector=projector)
    flops = plan.stats["total_flops_per_b"]     # 8 real flops per complex multiply-add
    return math.log2(flops / 4.0), plan.stats["max_bits"]


def family_rows(Ls=(4, 5, 6, 7, 8), doubled=True):
    from circuits import paper_family_instances
    rows = []
    for L in Ls:
        for name, circ, T in paper_family_instances(L):
            row = {"family": name, "L": L, "n": circ.n, "T": T}
            row.update(circuit_bounds(circ, T))
            row["log2_plan_amplitude"], row["max_rank_amplitude"] = counted_log2(circ)
            if doubled:
                row["log2_plan_doubled"], row["max_rank_doubled"] = counted_log2(circ, projector=())
            rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[4, 5, 6, 7, 8])
    ap.add_argument("--no-doubled", action="store_true")
    ap.add_argument("--json", action="store_true")
    args = ap.parse_args()
    rows = family_rows(args.L, doubled=not args.no_doubled)
    if args.json:
        print(json.dumps(rows))
        return
    cols = ["family", "L", "n", "sum_f", "F", "log2_plan_amplitude", "log2_plan_doubled",
            "log2_theorem2", "log2_theorem2_planar", "log2_sidewise", "log2_explicit"]
    print("| " + " | ".join(cols) + " |")
    print("|" + "---|" * len(cols))
    for r in rows:
        cells = []
        for c in cols:
            v = r.get(c)
            cells.append("-" if v is None else ("%.1f" % v if isinstance(v, float) else str(v)))
        print("| " + " | ".join(cells) + " |", flush=True)


if __name__ == "__main__":
    main()
