"""Benchmark: amplitudes/s of the 8x8 depth-16 random circuit (Haar SU(2) +
CZ, 2^10 slices, 64 bitstrings) on one MI355X, with the roofline of the
dominant GEMM kernel and the CPU oracle timed beside it.

One step = one tn_contract_amplitudes call over the whole batch (all slices,
all chunks), inputs resident: the plan is built and loaded before timing.

  python bench.py [--steps K] [--warmup W] [--precision fp32_3m|fp32|bf16x3|fp16x3]
                  [--config cfg3] [--batch B] [--slices S] [--width W]
                  [--no-cpu]

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3e12, "fp32_3m": 157.3e12, "bf16x3": 2516.6e12, "fp16x3": 2516.6e12,
        "bf16x1": 2516.6e12}
# executed MFMA flops per algorithmic flop (8 real flops per complex
# multiply-add): 4M executes exactly those, 3M three real products instead
# of four, split bf16 and fp16 three 16-bit products of the 4M form
EXEC = {"fp32": 1.0, "fp32_3m": 0.75, "bf16x3": 3.0, "fp16x3": 3.0, "bf16x1": 1.0}

# HBM traffic per launch of a kernel class, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) over `bench.py --warmup 0 --steps 1 --no-cpu`
# (the launches of one timed step), each scaled by the counter's reading
# for a plain 1 GiB device
# copy (`bench.py --copy-calibration`).  Keyed by the SHA-256 of the kernel's
# source file, the plan's work per amplitude and the bitstring chunk: a
# changed kernel or plan reports null until it is measured again.
TRAFFIC = [
    {"class": "cgemm_mfma_128x128", "precision": "fp32_3m", "source": "gemm.hip",
     "source_sha256": "a2d73b6a7fe485b7e2eb77a3007b4a9c96b1706633db6faded8abc6ff2fae01e",
     "chunk": 30, "flops_per_amplitude": 40093516002040.0,
     "bytes_per_launch": 1.633e11,
     "note": "HBM fetch 1.534e11 + write 9.890e9 bytes per launch (the 153 launches of one "
             "timed step; FETCH_SIZE x2.0 and WRITE_SIZE x1.0 from a 1 GiB copy); algorithmic "
             "1.678e10"},
]


def source_hash(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2208_01498_amd", "csrc", name)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, the scale for the HBM
    byte counters."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "launches": reps}), flush=True)


def stored_oracle_errors(config, words, amps, n):
    """Errors of the timed step's results for the bitstrings whose oracle
    amplitudes are stored (complex128, every slice summed, written by the
    golden script from the oracle alone): plain relative error per result,
    and the error and |a_ref| in units of the typical magnitude 2^(-n/2)."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize_oracle_amplitudes.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path)).get(config)
    if not data:
        return None
    typ = 2.0 ** (-n / 2)
    rows = []
    for r in data["amplitudes"]:
        w = int(r["bitstring"])
        hit = [i for i in range(len(words)) if int(words[i]) == w]
        if not hit:
            continue
        ref = complex(r["re"], r["im"])
        err = abs(complex(amps[hit[0]]) - ref)
        rows.append({"bitstring": str(w), "plain_relative": err / abs(ref),
                     "err_over_typical": err / typ, "abs_ref_over_typical": abs(ref) / typ})
    if not rows:
        return None
    return {"reference": "stored oracle amplitudes (" + data["method"] + ")",
            "results": rows,
            "max_plain_relative": max(x["plain_relative"] for x in rows)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(circ, word, seconds=20.0, width=24, seed=0):
    """The oracle (pairwise contraction in complex128, plan order imported
    as data) on a bounded sample: slices of one amplitude under a slicing of
    the same network whose widest tensor has 2^width entries, timed until
    ``seconds`` pass; the rate is scaled to amplitudes/s by the slice count."""
    import numpy as np
    from oracle.pairwise import OracleNetwork, _restrict, _evaluate
    from paper_2208_01498_amd.planner.plan import make_plan
    plan = make_plan(circ, n_slices=None, target_width=width, B=1, seed=seed, objective="oracle")
    spec = plan.order_spec()
    net = OracleNetwork(circ, word)
    labels = net.labels_of_slice_spec(spec["sliced"])
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    t0 = time.perf_counter()
    done = 0
    while True:
        s = done
        fixed = {l: (s >> j) & 1 for j, l in enumerate(labels)}
        _evaluate(_restrict(net.pieces, fixed), spec)
        done += 1
        if time.perf_counter() - t0 >= seconds or done >= (1 << len(labels)):
            break
    el = time.perf_counter() - t0
    per_amp = el / done * (1 << len(labels))
    return {"value": 1.0 / per_amp, "unit": "amplitudes/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d of 2^%d slices of one amplitude (bitstring 0 of the batch), "
                      "oracle pairwise contraction in plan order, %.1f s; scaled by the "
                      "slice count" % (done, len(labels), el)}


def _serving_plan(item):
    from paper_2208_01498_amd.planner.plan import make_plan
    _, c, ns = item
    return make_plan(c, n_slices=ns, B=32)


def serving_plans(pool):
    """The pool's plans (deterministic: seeded hierarchies), built in
    parallel worker processes before the GPU is touched."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    with ProcessPoolExecutor(max_workers=min(len(pool), 12),
                             mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_serving_plan, pool))


def serve_check(args, pool, plans):
    """Second half of the alone-versus-mixed check for the requests a served
    run wrote out (--serve-dump): the same bitstrings, run alone on the same
    plans (one call per plan), must give bitwise the served amplitudes."""
    import numpy as np
    from paper_2208_01498_amd import binding as B
    dump = json.load(open(args.serve_check))
    prec = B.PRECISIONS[dump["precision"]]
    import torch
    free, _ = torch.cuda.mem_get_info(0)
    eng = B.Engine(0, arena_bytes=int(free - (8 << 30)))
    hs = {}
    mismatched = checked = 0
    by_plan = {}
    for r in dump["requests"]:
        by_plan.setdefault(r["plan"], []).append(r)
    for k, rs in sorted(by_plan.items()):
        if k not in hs:
            hs[k] = eng.load(plans[k].to_blob())
        allw = np.array([int(w) for r in rs for w in r["bitstrings"]], dtype=np.uint64)
        alone = eng.amplitudes(hs[k], allw, prec)
        pos = 0
        for r in rs:
            served = np.array(r["re"]) + 1j * np.array(r["im"])
            n = len(served)
            mismatched += not np.array_equal(alone[pos:pos + n], served)
            checked += 1
            pos += n
        log("plan %d (%s): %d served requests rerun alone" % (k, pool[k][0], len(rs)))
    print(json.dumps({"metric": "served results rerun alone", "checked": checked,
                      "mismatched": mismatched, "families": sorted(set(pool[k][0] for k in by_plan)),
                      "precision": dump["precision"]}), flush=True)
    eng.close()


def serve_bench(args):
    """The served mixed stream: requests drawn uniformly from four circuit
    families (three instances each, all plans resident), 1..64 bitstrings
    each, Poisson arrivals at a fixed fraction of the saturation rate.  The
    saturation rate is 1 / E[service time], with each family's time per
    bitstring measured alone first."""
    import numpy as np
    import torch
    from circuits import random_bitstrings
    from circuits.families import serving_pool
    from paper_2208_01498_amd.planner.plan import make_plan
    from paper_2208_01498_amd import binding as B
    pool = serving_pool()
    prec = B.PRECISIONS[args.precision]
    t = time.perf_counter()
    plans = serving_plans(pool)
    log("%d plans built in %.1f s" % (len(plans), time.perf_counter() - t))
    if args.serve_check:
        return serve_check(args, pool, plans)
    free, _ = torch.cuda.mem_get_info(0)
    eng = B.Engine(0, arena_bytes=int(free - (8 << 30)))
    B.tn_server_config(eng.ctx, args.slots, 64)
    B.tn_server_set_heavy(eng.ctx, 1e14, args.max_heavy)
    hs = [eng.load(p.to_blob()) for p in plans]
    fams = sorted(set(f for f, _, _ in pool))
    # time per bitstring of each family, alone (first instance, 8 bitstrings)
    per_b = {}
    for f in fams:
        k = [i for i, (ff, _, _) in enumerate(pool) if ff == f][0]
        w = random_bitstrings(pool[k][1].n, 8, 89000 + k)
        eng.amplitudes(hs[k], w[:1], prec)
        t0 = time.perf_counter()
        eng.amplitudes(hs[k], w, prec)
        per_b[f] = (time.perf_counter() - t0) / len(w)
        log("family %s: %.4f s per bitstring alone" % (f, per_b[f]))
    mean_nb = 32.5
    e_service = sum(per_b[f] * mean_nb for f in fams) / len(fams)
    sat = 1.0 / e_service
    lam = args.serve_load * sat
    log("E[service] %.2f s -> saturation %.4f req/s, arrivals at %.4f req/s" % (e_service, sat, lam))
    rng = np.random.Generator(np.random.PCG64(5002))

    def draw(i):
        f = fams[int(rng.integers(len(fams)))]
        idx = [k for k, (ff, _, _) in enumerate(pool) if ff == f]
        k = idx[int(rng.integers(len(idx)))]
        nb = int(rng.integers(1, 65))
        return k, random_bitstrings(pool[k][1].n, nb, 90000 + i)

    reqs = [draw(1000 + i) for i in range(args.serve_requests)]
    gaps = rng.exponential(1.0 / lam, size=len(reqs))
    arrivals = np.cumsum(gaps) - gaps[0]
    # requests arriving after the cap are not submitted; the stream drains
    cap = args.serve_cap_s
    n_sub = int(np.searchsorted(arrivals, cap, side="right")) if cap > 0 else len(reqs)
    reqs, arrivals = reqs[:n_sub], arrivals[:n_sub]
    log("%d requests arrive within the %.0f s cap" % (len(reqs), cap))
    t0 = time.perf_counter()
    pending = {}
    done = {}
    i = 0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and arrivals[i] <= now:
            k, w = reqs[i]
            pending[B.tn_submit(eng.ctx, hs[k], w, prec)] = (i, len(w))
            log("request %d (%s, %d bitstrings) submitted at %.1f s" % (i, pool[k][0], len(w), now))
            i += 1
        for tk in list(pending):
            j, n = pending[tk]
            r = B.tn_poll(eng.ctx, tk, n)
            if r is not None:
                done[j] = r
                del pending[tk]
                log("request %d (%s, %d bitstrings) done after %.2f s" % (
                    j, pool[reqs[j][0]][0], n, (r[1]["t_end_ns"] - r[1]["t_arrive_ns"]) * 1e-9))
        time.sleep(0.0005)
    el = time.perf_counter() - t0
    lat = np.array([(done[j][1]["t_end_ns"] - done[j][1]["t_arrive_ns"]) * 1e-9 for j in range(len(reqs))])
    amps = sum(len(w) for _, w in reqs)
    # every served result against the same bitstrings run alone: one call
    # per plan over all of its requests' bitstrings (a result does not
    # depend on the batch or chunk it runs in)
    same = True
    mismatched = 0
    dumped = []
    for k in sorted(set(k for k, _ in reqs)):
        js = [j for j, (kk, _) in enumerate(reqs) if kk == k]
        if args.serve_dump and pool[k][0] in args.serve_dump_families:
            # rerun alone in a later process (--serve-check on the dump)
            for j in js:
                a = done[j][0]
                dumped.append({"request": j, "plan": k, "bitstrings": [str(int(x)) for x in reqs[j][1]],
                               "re": a.real.tolist(), "im": a.imag.tolist()})
            continue
        allw = np.concatenate([reqs[j][1] for j in js])
        alone = eng.amplitudes(hs[k], allw, prec)
        pos = 0
        for j in js:
            nb_j = len(reqs[j][1])
            ok = bool(np.array_equal(alone[pos:pos + nb_j], done[j][0]))
            mismatched += not ok
            same &= ok
            pos += nb_j
        log("plan %d (%s): %d requests, %d bitstrings checked against the alone run"
            % (k, pool[k][0], len(js), len(allw)))
    if args.serve_dump:
        json.dump({"precision": args.precision, "requests": dumped}, open(args.serve_dump, "w"))
        log("%d served results written to %s for the alone check" % (len(dumped), args.serve_dump))
    per_fam = {}
    for j, (k, w) in enumerate(reqs):
        per_fam.setdefault(pool[k][0], []).append(lat[j])
    out = {"metric": "p50/p99 served latency, mixed stream", "unit": "s",
           "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
           "req_per_s": len(reqs) / el, "amplitudes_per_s": amps / el,
           "lambda_req_per_s": lam, "saturation_req_per_s": sat, "load": args.serve_load,
           "n_requests": len(reqs), "cap_s": cap, "slots": args.slots,
           "max_heavy": args.max_heavy,
           "alone_equals_mixed": same, "checked_against_alone": len(reqs) - len(dumped),
           "written_for_alone_check": len(dumped), "mismatched": mismatched,
           "precision": args.precision,
           "seconds_per_bitstring_alone": per_b,
           "p50_by_family": {f: float(np.percentile(v, 50)) for f, v in per_fam.items()},
           "p99_by_family": {f: float(np.percentile(v, 99)) for f, v in per_fam.items()},
           "config": {"workload": "served mix: 5x5 d10, 6x6 d12, 8x8 d16 (2^10 slices) "
                                  "Haar SU(2)+CZ lattices and 3x3x4 SU(4) stack, "
                                  "1-64 bitstrings per request, Poisson arrivals"},
           "data": "synthetic"}
    print(json.dumps(out), flush=True)
    eng.close()


def paper_families_bench(args):
    """The paper's own circuit families at executable sizes, through the
    planner and the executor: the IQP family (T = L^2 steps, gamma = 3) and
    the Sycamore-type family (5 periods of 8 cycles, qubits inaccessible for
    a period with probability 0.88, and 0.5 as a denser variant).  Reports
    the counted cost of each plan (the paper's measure: real flops per
    amplitude, Eq. (3)) beside the measured time."""
    import numpy as np
    from circuits import paper_family_instances, random_bitstrings
    from paper_2208_01498_amd.planner.bounds import circuit_bounds
    from paper_2208_01498_amd.planner.plan import make_plan
    from paper_2208_01498_amd import binding as B
    import torch
    free, _ = torch.cuda.mem_get_info(0)
    eng = B.Engine(0, arena_bytes=int(free - (8 << 30)))
    prec = B.PRECISIONS[args.precision]
    rows = []
    for L in range(4, 9):
        for fam, circ, T in paper_family_instances(L):
            words = random_bitstrings(circ.n, 64, 5500 + L)
            t = time.perf_counter()
            plan = make_plan(circ, n_slices=None, target_width=30, B=len(words))
            t_plan = time.perf_counter() - t
            h = eng.load(plan.to_blob())
            eng.amplitudes(h, words, prec)
            torch.cuda.synchronize()
            t = time.perf_counter()
            eng.amplitudes(h, words, prec)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            rows.append({"family": fam, "L": L, "n": circ.n, "gates": len(circ.gates),
                         "flops_per_amplitude": plan.stats["total_flops_per_b"],
                         "max_rank": plan.stats["max_bits"], "slices": 1 << len(plan.sliced),
                         "plan_s": t_plan, "amplitudes_per_s": len(words) / el,
                         "log2_ops_plan": math.log2(plan.stats["total_flops_per_b"] / 4.0)})
            rows[-1].update(circuit_bounds(circ, T))
            log(json.dumps(rows[-1]))
            eng.unload(h)
    print(json.dumps({"metric": "paper families: counted flops and measured amplitudes/s",
                      "precision": args.precision, "rows": rows, "data": "synthetic"}), flush=True)
    eng.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg3")
    ap.add_argument("--precision", default="fp32_3m", choices=["fp32", "fp32_3m", "bf16x3", "fp16x3", "bf16x1"])
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--slices", type=int, default=10)
    ap.add_argument("--width", type=float, default=None,
                    help="slice until the widest per-slice tensor has 2^width entries")
    ap.add_argument("--per-bitstring-width", action="store_true",
                    help="--width counts one bitstring's entries (the batch runs in chunks)")
    ap.add_argument("--svd-split", action="store_true",
                    help="the paper-faithful network: rank-3 SVD halves of every two-qubit gate, "
                         "no diagonal hyperedges")
    ap.add_argument("--arena-gb", type=float, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-after", action="store_true",
                    help="time the steps without per-launch events (captured HIP graphs replay), "
                         "then run one more step with events for the per-kernel figures: for "
                         "launch-bound workloads")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--serve", action="store_true", help="served mixed stream instead")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="arrival rate as a fraction of the saturation rate")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-heavy", type=int, default=1,
                    help="served batches of at least 1e14 flops running at once")
    ap.add_argument("--serve-cap-s", type=float, default=600.0,
                    help="submit only requests arriving within this many seconds (0: all)")
    ap.add_argument("--serve-dump", default=None,
                    help="write the served results of --serve-dump-families here instead of "
                         "rerunning them alone in this process")
    ap.add_argument("--serve-dump-families", nargs="*", default=["8x8d16"])
    ap.add_argument("--serve-check", default=None,
                    help="rerun the requests of a --serve-dump file alone and compare bitwise")
    ap.add_argument("--paper-families", action="store_true",
                    help="the paper's IQP and Sycamore-type families at L = 4..8 instead")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a 1 GiB device copy, to scale the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(slices would shard across GPUs with one all-reduce of the FP64 sums)",
              file=sys.stderr)
        sys.exit(2)
    if args.serve or args.serve_check:
        return serve_bench(args)
    if args.copy_calibration:
        return copy_calibration()
    if args.paper_families:
        return paper_families_bench(args)

    import numpy as np
    import torch
    from circuits import make_config
    from paper_2208_01498_amd.planner.plan import make_plan
    from paper_2208_01498_amd import binding as B

    circ, words, info = make_config(args.config)
    if args.batch:
        words = words[:args.batch]
    nb = len(words)
    t = time.perf_counter()
    plan = make_plan(circ, n_slices=args.slices, target_width=args.width, B=nb, seed=args.seed,
                     width_per_bitstring=args.per_bitstring_width, svd_split=args.svd_split)
    blob = plan.to_blob()
    log("plan built in %.1f s: %d leaves, %d steps, %d sliced labels" %
        (time.perf_counter() - t, plan.stats["n_leaves"], plan.stats["n_steps"], len(plan.sliced)))
    free, total = torch.cuda.mem_get_info(0)
    arena = int((args.arena_gb * 2 ** 30) if args.arena_gb else (free - (6 << 30)))
    eng = B.Engine(0, arena_bytes=arena)
    p = eng.load(blob)
    pinfo = B.tn_plan_info(p)
    log("plan info", pinfo)
    prec = B.PRECISIONS[args.precision]
    for _ in range(args.warmup):
        eng.amplitudes(p, words, prec)
        log("warmup step done", B.tn_last_exec_stats(eng.ctx)["chunk"])
    # per-kernel HIP events on the executing stream, recorded inside the
    # timed region (read back only every few thousand launches); with
    # --profile-after the timed steps run without them and one more step
    # records them
    B.tn_ctx_set_profiling(eng.ctx, 0 if args.profile_after else 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        amps = eng.amplitudes(p, words, prec)
        log("timed step %d done" % k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    graph_replays = B.tn_last_exec_stats(eng.ctx)["graph_replays"]
    if args.profile_after:
        B.tn_ctx_set_profiling(eng.ctx, 1)
        eng.amplitudes(p, words, prec)
        torch.cuda.synchronize()
    B.tn_ctx_set_profiling(eng.ctx, 0)
    st = B.tn_last_exec_stats(eng.ctx)
    el = t1 - t0
    value = nb * args.steps / el
    prof = st   # the last timed step
    kinds = B.KERNEL_CLASSES
    per_kind = {kinds[i]: {"launches": prof["launches"][i], "ms": prof["time_ms"][i],
                           "flops": prof["flops"][i], "bytes": prof["bytes"][i]}
                for i in range(len(kinds))}
    log("per kernel class", json.dumps(per_kind))
    dom = max(B.GEMM_CLASSES, key=lambda i: prof["time_ms"][i])
    ms = prof["time_ms"][dom]
    alg = prof["flops"][dom] / (ms * 1e-3) if ms > 0 else 0.0
    achieved = alg * EXEC[args.precision]
    peak = PEAK[args.precision]
    roofline = {"bound": "mfma", "kernel": kinds[dom],
                "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "flops_per_launch": prof["flops"][dom] * EXEC[args.precision] / max(1, prof["launches"][dom]),
                "algorithmic_tflops": alg / 1e12,
                "avg_launch_ms": ms / max(1, prof["launches"][dom]),
                "gemm_time_frac": sum(prof["time_ms"][i] for i in B.GEMM_CLASSES) / max(1e-9, sum(prof["time_ms"]))}
    # the permute kernels against HBM (algorithmic bytes: one read and one
    # write of every element)
    pm = prof["time_ms"][4]
    permute = {"bound": "hbm", "achieved": prof["bytes"][4] / (pm * 1e-3) / 1e9 if pm > 0 else 0.0,
               "peak": 8000.0, "unit": "GB/s", "launches": prof["launches"][4], "ms": pm}
    permute["frac"] = permute["achieved"] / permute["peak"]
    for rec in TRAFFIC:
        # the same kernel source, precision and launches (the plan's work per
        # amplitude and the bitstring chunk fix the launch shapes)
        if (rec["class"] == kinds[dom] and rec["precision"] == args.precision and
                rec["source_sha256"] == source_hash(rec["source"]) and
                rec.get("chunk") == st["chunk"] and
                abs(rec.get("flops_per_amplitude", 0) / (st["algorithmic_flops"] / nb) - 1) < 1e-6):
            roofline["traffic"] = rec["bytes_per_launch"]
            roofline["traffic_note"] = rec["note"]
    accuracy = stored_oracle_errors(args.config, words, amps, circ.n)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(circ, int(words[0]), seconds=args.cpu_seconds)
    out = {
        "metric": ("amplitudes/s, 8x8 depth-16 circuit (2^10 slices, 64 bitstrings)"
                   if args.config == "cfg3" else "amplitudes/s, " + info["desc"]),
        "value": value, "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "c64/f32-mfma", "fp32_3m": "c64/f32-mfma-3m",
                  "bf16x3": "bf16x3-mfma/f32-acc", "fp16x3": "fp16x3-mfma/f32-acc",
                  "bf16x1": "bf16-mfma/f32-acc"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.config, info["desc"]), "batch": nb,
                   "slices": 1 << len(plan.sliced), "precision": args.precision,
                   "chunk": st["chunk"], "n_chunks": st["n_chunks"],
                   "slice_block": st["slice_block"],
                   "timing": ("steps without per-launch events (graph replays in the last: %d), "
                              "kernel figures from one more step with events" % graph_replays)
                   if args.profile_after else "per-launch events inside the timed steps",
                   "algorithmic_flops_per_amplitude": st["algorithmic_flops"] / nb,
                   "network": "svd halves" if args.svd_split else "diagonal hyperedges",
                   "arena_bytes": arena},
        "roofline": roofline,
        "achieved_algorithmic_tflops": st["algorithmic_flops"] * args.steps / el / 1e12,
        "permute_roofline": permute,
        "accuracy": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    eng.close()


if __name__ == "__main__":
    main()
