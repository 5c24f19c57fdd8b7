"""Serving loop: continuous batching through tn_submit / tn_poll."""
import time

import numpy as np
import pytest

from circuits import lattice_circuit, stack3d_circuit, random_bitstrings
from oracle import statevector_amplitudes

import fp_error

pytestmark = pytest.mark.gpu


def _plans():
    from paper_2208_01498_amd.planner.plan import make_plan
    circs = [lattice_circuit(4, 4, 8, 601, "haar", "cz"),
             lattice_circuit(3, 5, 10, 602, "sqrt", "fsim"),
             stack3d_circuit(2, 2, 4, 8, 603),
             lattice_circuit(4, 5, 12, 604, "haar", "cz")]
    return circs, [make_plan(c, n_slices=ns, B=16) for c, ns in zip(circs, (2, 0, 0, 4))]


def _wait(B, ctx, tickets, sizes, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, n in zip(tickets, sizes):
            if t in out:
                continue
            r = B.tn_poll(ctx, t, n)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "served requests did not finish"
        time.sleep(0.002)
    return out


@pytest.mark.parametrize("prec", [0, 3])
def test_mixed_stream_equals_alone_runs(prec):
    """Requests on four plans, batch sizes 1..16, submitted together: each
    result is bitwise the alone-run result and matches the state vector
    (FP32 4M, and the split fp16 mode, whose scratch the serving loop
    reserves per batch)."""
    from paper_2208_01498_amd import binding as B
    circs, plans = _plans()
    eng = B.Engine(0, arena_bytes=512 << 20)
    try:
        B.tn_server_config(eng.ctx, 3, 32)
        hs = [eng.load(p.to_blob()) for p in plans]
        rng = np.random.Generator(np.random.PCG64(610))
        reqs = []
        for i in range(24):
            k = int(rng.integers(len(plans)))
            nb = int(rng.integers(1, 17))
            words = random_bitstrings(circs[k].n, nb, 700 + i)
            reqs.append((k, words))
        alone = [eng.amplitudes(hs[k], w, prec) for k, w in reqs]
        print("submitting", len(reqs), "requests", flush=True)
        tickets = [B.tn_submit(eng.ctx, hs[k], w, prec) for k, w in reqs]
        res = _wait(B, eng.ctx, tickets, [len(w) for _, w in reqs])
        merged = 0
        for (k, w), t, a in zip(reqs, tickets, alone):
            amps, st = res[t]
            assert np.array_equal(amps, a)
            assert st["t_arrive_ns"] <= st["t_admit_ns"] <= st["t_start_ns"] <= st["t_end_ns"]
            merged += st["batch"] > len(w)
        print("requests served inside a merged batch:", merged, flush=True)
        for i, ((k, w), a) in enumerate(zip(reqs, alone)):
            ref = statevector_amplitudes(circs[k], w)
            typ = 2.0 ** (-circs[k].n / 2)
            fp_error.check(a, ref, typ, 1e-5 if prec == 0 else 1e-3,
                           fp_error.floor(plans[k], prec, typ), "request %d plan %d" % (i, k))
    finally:
        eng.close()


def test_cancel_poll_and_unload_busy():
    from paper_2208_01498_amd import binding as B
    circs, plans = _plans()
    eng = B.Engine(0, arena_bytes=256 << 20)
    try:
        B.tn_server_config(eng.ctx, 1, 16)
        h = eng.load(plans[3].to_blob())
        words = random_bitstrings(circs[3].n, 16, 801)
        ts = [B.tn_submit(eng.ctx, h, words, 0) for _ in range(6)]
        B.tn_cancel(eng.ctx, ts[-1])
        with pytest.raises(B.TnError) as e:
            B.tn_plan_unload(eng.ctx, h)
        assert e.value.code in (B.TN_EBUSY,)
        got = {}
        t0 = time.time()
        while len(got) < len(ts):
            for t in ts:
                if t in got:
                    continue
                try:
                    r = B.tn_poll(eng.ctx, t, 16)
                except B.TnError as err:
                    got[t] = err.code
                    continue
                if r is not None:
                    got[t] = r
            assert time.time() - t0 < 60
            time.sleep(0.002)
        assert got[ts[-1]] == B.TN_ECANCELLED
        assert all(not isinstance(got[t], int) for t in ts[:-1])
        with pytest.raises(B.TnError) as e:
            B.tn_poll(eng.ctx, ts[0], 16)
        assert e.value.code == B.TN_ENOTFOUND
    finally:
        eng.close()


def test_submit_rejects_requests_that_never_fit():
    """A plan whose one-bitstring workspace (about 2.9 MB for this 5x6
    depth-12 circuit, unsliced) exceeds the whole 1 MiB arena is refused at
    submit with TN_ENOMEM, in every precision mode."""
    from paper_2208_01498_amd import binding as B
    from paper_2208_01498_amd.planner.plan import make_plan
    c = lattice_circuit(5, 6, 12, 812, "haar", "cz")
    blob = make_plan(c, n_slices=0, B=2, trials=1).to_blob()
    info = B.tn_plan_validate(blob)
    need = info["peak_bytes_fixed"] + info["peak_bytes_per_b"]
    assert need > (1 << 20)
    eng = B.Engine(0, arena_bytes=1 << 20)
    try:
        h = eng.load(blob)
        for prec in (0, 1, 2, 3):
            with pytest.raises(B.TnError) as e:
                B.tn_submit(eng.ctx, h, random_bitstrings(c.n, 2, 811), prec)
            assert e.value.code == B.TN_ENOMEM
            with pytest.raises(B.TnError) as e:
                eng.amplitudes(h, random_bitstrings(c.n, 2, 811), prec)
            assert e.value.code == B.TN_ENOMEM
    finally:
        eng.close()


def test_light_request_passes_a_waiting_heavy_batch():
    """With one heavy batch allowed at a time, a second heavy request waits
    for the first while a light request submitted after it is admitted at
    once; every result equals its alone run."""
    from paper_2208_01498_amd import binding as B
    from paper_2208_01498_amd.planner.plan import make_plan
    heavy_c = lattice_circuit(6, 6, 12, 620, "haar", "cz")
    light_c = lattice_circuit(3, 3, 6, 621, "haar", "cz")
    hp, lp = make_plan(heavy_c, B=16), make_plan(light_c, B=2)
    eng = B.Engine(0, arena_bytes=2 << 30)
    try:
        B.tn_server_config(eng.ctx, 3, 16)
        hh, hl = eng.load(hp.to_blob()), eng.load(lp.to_blob())
        info = B.tn_plan_info(hh)
        B.tn_server_set_heavy(eng.ctx, info["flops_total_per_b"] * 16, 1)
        w1 = random_bitstrings(36, 16, 622)
        w2 = random_bitstrings(36, 16, 623)
        wl = random_bitstrings(9, 2, 624)
        alone = [eng.amplitudes(hh, w1, 0), eng.amplitudes(hh, w2, 0), eng.amplitudes(hl, wl, 0)]
        print("submitting heavy, heavy, light", flush=True)
        ts = [B.tn_submit(eng.ctx, hh, w1, 0), B.tn_submit(eng.ctx, hh, w2, 0),
              B.tn_submit(eng.ctx, hl, wl, 0)]
        res = _wait(B, eng.ctx, ts, [16, 16, 2])
        (a1, s1), (a2, s2), (al, sl) = res[ts[0]], res[ts[1]], res[ts[2]]
        print("heavy 1 %.3f-%.3f s, heavy 2 admitted %.3f s, light %.3f-%.3f s" % (
            (s1["t_start_ns"] - s1["t_arrive_ns"]) * 1e-9, (s1["t_end_ns"] - s1["t_arrive_ns"]) * 1e-9,
            (s2["t_admit_ns"] - s1["t_arrive_ns"]) * 1e-9, (sl["t_start_ns"] - s1["t_arrive_ns"]) * 1e-9,
            (sl["t_end_ns"] - s1["t_arrive_ns"]) * 1e-9), flush=True)
        assert s2["t_admit_ns"] >= s1["t_end_ns"]
        assert sl["t_admit_ns"] <= s2["t_admit_ns"]
        for got, want in zip((a1, a2, al), alone):
            assert np.array_equal(got, want)
    finally:
        eng.close()


def test_unload_twice_is_an_error():
    """A plan unloaded once is no longer known to the context: a second
    unload returns TN_EINVAL instead of touching freed memory, and
    destroying the context afterwards is clean."""
    from paper_2208_01498_amd import binding as B
    circs, plans = _plans()
    eng = B.Engine(0, arena_bytes=64 << 20)
    try:
        h = eng.load(plans[0].to_blob())
        eng.load(plans[1].to_blob())          # left for the context to release
        eng.unload(h)
        with pytest.raises(B.TnError) as e:
            B.tn_plan_unload(eng.ctx, h)
        assert e.value.code == B.TN_EINVAL
    finally:
        eng.close()


def test_served_mix_families_vs_oracle():
    """The served mix's circuit families at their sizes (5x5 depth 10 and
    6x6 depth 12 Haar + CZ lattices, the 3x3x4 SU(4) stack; three instances
    each, all plans resident; the 8x8 depth-16 family is left to the bench)
    under a stream of 30 requests of 1-64 bitstrings: every result is
    bitwise the same bitstrings run alone, and the first four bitstrings of
    every request match the oracle (pairwise complex128 contraction in the
    plan's order)."""
    from circuits.families import serving_pool
    from oracle import pairwise_amplitudes
    from paper_2208_01498_amd import binding as B
    from paper_2208_01498_amd.planner.plan import make_plan
    pool = [p for p in serving_pool() if p[0] != "8x8d16"]
    plans = [make_plan(c, n_slices=ns, B=32) for _, c, ns in pool]
    eng = B.Engine(0, arena_bytes=8 << 30)
    try:
        B.tn_server_config(eng.ctx, 4, 64)
        hs = [eng.load(p.to_blob()) for p in plans]
        rng = np.random.Generator(np.random.PCG64(5002))
        reqs = []
        for i in range(30):
            k = int(rng.integers(len(pool)))
            reqs.append((k, random_bitstrings(pool[k][1].n, int(rng.integers(1, 65)), 91000 + i)))
        print("submitting", len(reqs), "requests on", len(pool), "plans", flush=True)
        tickets = [B.tn_submit(eng.ctx, hs[k], w, 0) for k, w in reqs]
        res = _wait(B, eng.ctx, tickets, [len(w) for _, w in reqs], timeout=120)
        for i, ((k, w), t) in enumerate(zip(reqs, tickets)):
            got = res[t][0]
            assert np.array_equal(got, eng.amplitudes(hs[k], w, 0)), i
            spec = plans[k].order_spec()
            ref = pairwise_amplitudes(pool[k][1], w[:4], order=spec, sliced=spec["sliced"])
            typ = 2.0 ** (-pool[k][1].n / 2)
            fp_error.check(got[:4], ref, typ, 1e-5, fp_error.floor(plans[k], 0, typ),
                           "served %s request %d" % (pool[k][0], i))
    finally:
        eng.close()
