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
       python -m paper_2208_01498_amd.planner.report --separators
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


SEPARATORS = ("ssa+planes", "ssa", "planar")


def separator_rows(cases, trials=3):
    """Counted cost (log2 scalar operations per amplitude, all slices) of the
    plans whose hierarchies come from Algorithm 1 with the median coordinate
    planes beside its candidates (the default), from Algorithm 1 alone, and
    from planar level separators (planar.py), with the sources of the kept
    hierarchy's splits.  `cases`: (name, circuit, make_plan keywords)."""
    rows = []
    for name, circ, kw in cases:
        row = {"workload": name, "n": circ.n}
        for sep in SEPARATORS:
            plan = make_plan(circ, trials=trials, separators=sep, **kw)
            row["log2_ops_" + sep] = math.log2(plan.stats["total_flops_per_b"] / 4.0)
            row["max_rank_" + sep] = plan.stats["max_bits"]
            row["splits_" + sep] = plan.stats["split_sources"]
        rows.append(row)
    return rows


def workload_cases():
    from circuits import make_config, paper_family_instances
    cases = []
    for cfg, kw in (("cfg1", dict(n_slices=0, B=8)), ("cfg3", dict(n_slices=10, B=64)),
                    ("cfg2", dict(n_slices=None, target_width=28, B=256, width_per_bitstring=True)),
                    ("cfg4", dict(n_slices=0, B=1024))):
        cases.append((cfg, make_config(cfg)[0], kw))
    for name, circ, _ in paper_family_instances(6):
        cases.append((name + "_L6", circ, dict(n_slices=None, target_width=30, B=64)))
    return cases


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


def large_size_rows(kind, L, reps=10):
    """Bounds only, at the paper's large sizes, from two-qubit gate counts
    (no gate list): `kind` "sycamore" (5 periods, p = 0.88, T = 40 cycles)
    or "cavity" ((2+1)-D with cavities, T = round(0.1 L)).  Per realization:
    log2 of Theorem 2 (general and planar d = 2 forms), side-wise and
    explicit evolution; returns the list of dicts."""
    import numpy as np
    from circuits import sycamore_type_gate_counts, cavity_circuit_gate_counts
    from .bounds import (theorem2_log2, theorem2_planar_log2, sidewise_log2, explicit_log2)
    rows = []
    for r in range(reps):
        if kind == "sycamore":
            f = sycamore_type_gate_counts(L, 5, 0.88, 7000 + 31 * L + r)
            T = 40
        else:
            f, T = cavity_circuit_gate_counts(L, 8000 + 31 * L + r)
        f = f.ravel()
        act = f[f > 0]
        rows.append({"L": L, "T": T, "idle": int((f == 0).sum()), "F": int(f.max()),
                     "log2_theorem2": theorem2_log2(act, 2, 1.0),
                     "log2_theorem2_planar": theorem2_planar_log2(act),
                     "log2_sidewise": sidewise_log2(int(f.max()), L, 2),
                     "log2_explicit": explicit_log2(T, L * L, int((f == 0).sum()))})
    return rows


def crossover_table(kind, Ls, reps=10):
    """Mean log2 of each bound and the fraction of realizations in which the
    planar Theorem 2 bound beats side-wise contraction, explicit evolution,
    and both."""
    import numpy as np
    out = []
    for L in Ls:
        rs = large_size_rows(kind, L, reps)
        mean = lambda k: float(np.mean([r[k] for r in rs]))
        out.append({"family": kind, "L": L, "reps": reps,
                    "log2_theorem2": mean("log2_theorem2"),
                    "log2_theorem2_planar": mean("log2_theorem2_planar"),
                    "log2_sidewise": mean("log2_sidewise"), "log2_explicit": mean("log2_explicit"),
                    "frac_below_sidewise": float(np.mean([r["log2_theorem2_planar"] < r["log2_sidewise"] for r in rs])),
                    "frac_below_explicit": float(np.mean([r["log2_theorem2_planar"] < r["log2_explicit"] for r in rs])),
                    "frac_below_both": float(np.mean([r["log2_theorem2_planar"] < min(r["log2_sidewise"], r["log2_explicit"]) for r in rs]))})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[4, 5, 6, 7, 8])
    ap.add_argument("--no-doubled", action="store_true")
    ap.add_argument("--json", action="store_true")
    ap.add_argument("--separators", action="store_true",
                    help="counted cost of the workloads' plans under each separator family")
    ap.add_argument("--large", action="store_true",
                    help="bounds only at the paper's large sizes (Sycamore-type L = 200..1600, "
                         "cavity circuits L = 150..300)")
    args = ap.parse_args()
    if args.separators:
        rows = separator_rows(workload_cases())
        if args.json:
            print(json.dumps(rows))
            return
        print("| workload | n | " + " | ".join("log2 ops %s (max rank) | splits %s" % (x, x)
                                             for x in SEPARATORS) + " |")
        print("|" + "---|" * (2 + 2 * len(SEPARATORS)))
        for r in rows:
            cells = [r["workload"], str(r["n"])]
            for x in SEPARATORS:
                cells.append("%.2f (%d)" % (r["log2_ops_" + x], r["max_rank_" + x]))
                cells.append(", ".join("%s %d" % kv for kv in r["splits_" + x].items() if kv[1]))
            print("| " + " | ".join(cells) + " |", flush=True)
        return
    if args.large:
        rows = (crossover_table("sycamore", (200, 400, 800, 1600))
                + crossover_table("cavity", (150, 200, 250, 300)))
        if args.json:
            print(json.dumps(rows))
            return
        cols = ["family", "L", "log2_theorem2", "log2_theorem2_planar", "log2_sidewise",
                "log2_explicit", "frac_below_sidewise", "frac_below_explicit", "frac_below_both"]
        print("| " + " | ".join(cols) + " |")
        print("|" + "---|" * len(cols))
        for r in rows:
            print("| " + " | ".join(("%.0f" % r[c]) if c.startswith("log2") else
                                    ("%.1f" % r[c]) if c.startswith("frac") else str(r[c])
                                    for c in cols) + " |", flush=True)
        return
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
