"""Writes fullsize_oracle_amplitudes.json: amplitudes of the 8x8 depth-16
and 6x6 depth-12 fSim workloads for their first four bitstrings, computed by
the CPU oracle alone (complex128 pairwise contraction of its own dense gate
tensors, every slice summed).  The contraction order and the sliced wires
come from a plan used as data (the oracle's own greedy order would not fit
in host memory at these sizes); they change the result only at rounding
level.  Run from the repository root:

    python tests/golden/make_fullsize_golden.py [--meta-only] [--count N] [cfg3|cfg2 ...]

It stores the first N bitstrings of each workload (default 4), computing only
those not stored yet.  It takes about ten minutes per 8x8 amplitude and two
per 6x6 amplitude on a few cores.  Each entry
also records the bitstrings and a SHA-256 of the circuit's JSON form, so a
change of the circuit generators shows up as a stale fixture;
`--meta-only` rewrites only that record for entries already stored.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from circuits import make_config                       # noqa: E402
from oracle import pairwise_amplitude                  # noqa: E402
from paper_2208_01498_amd.planner.plan import make_plan  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_oracle_amplitudes.json")


def circuit_sha256(circ):
    return hashlib.sha256(circ.to_json().encode()).hexdigest()


def main(names, meta_only=False, count=4):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        circ, words, _ = make_config(name)
        words = [int(w) for w in words[:count]]
        if meta_only:
            if name in data:
                data[name]["circuit_sha256"] = circuit_sha256(circ)
                json.dump(data, open(OUT, "w"), indent=1)
            continue
        # order and slices for tensors of at most 2^27 entries (2 GiB in
        # complex128)
        plan = make_plan(circ, n_slices=None, target_width=27, B=1, objective="oracle", trials=1)
        spec = plan.order_spec()
        rows = []
        old = data.get(name, {})
        if old.get("circuit_sha256") == circuit_sha256(circ):
            rows = [r for r in old["amplitudes"] if int(r["bitstring"]) in words]
        for w in words:
            if any(int(r["bitstring"]) == w for r in rows):
                continue
            t0 = time.perf_counter()
            a = pairwise_amplitude(circ, w, order=spec, sliced=spec["sliced"])
            rows.append({"bitstring": str(w), "re": a.real, "im": a.imag,
                         "seconds": time.perf_counter() - t0})
            print(name, w, a, "%.0f s" % rows[-1]["seconds"], flush=True)
            data[name] = {"method": "oracle pairwise contraction, complex128, %d sliced wires "
                                    "summed, plan order as data" % len(spec["sliced"]),
                          "circuit_sha256": circuit_sha256(circ),
                          "amplitudes": rows}
            json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    args = sys.argv[1:]
    meta = "--meta-only" in args
    args = [a for a in args if a != "--meta-only"]
    count = 4
    if "--count" in args:
        i = args.index("--count")
        count = int(args[i + 1])
        del args[i:i + 2]
    main(args or ["cfg3", "cfg2"], meta_only=meta, count=count)
