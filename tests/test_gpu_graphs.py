"""Captured HIP graphs of the executor: replays equal direct launches."""
import numpy as np
import pytest

from circuits import lattice_circuit, random_bitstrings
from oracle import statevector_amplitudes

import fp_error

pytestmark = pytest.mark.gpu


def _plan(circ, ns, B):
    from paper_2208_01498_amd.planner.plan import make_plan
    return make_plan(circ, n_slices=ns, B=B, trials=1)


@pytest.mark.parametrize("prec", [0, 1, 3])
@pytest.mark.parametrize("block", [-1, 0])
def test_graph_replays_equal_direct_runs(prec, block):
    """Two bitstring sets alternate over six calls on a context with graphs
    (the first call of the shape runs directly, the second is captured, the
    rest replay) and on one without: every result is bitwise the direct
    one, replays are counted, and the amplitudes match the state vector.
    block 0 runs the slices as 2^3 passes inside one chunk."""
    from paper_2208_01498_amd import binding as B
    circ = lattice_circuit(4, 4, 10, 1301, "haar", "cz")
    w1 = random_bitstrings(16, 12, 1302)
    w2 = random_bitstrings(16, 12, 1303)
    plan = _plan(circ, 3, 12)
    blob = plan.to_blob()
    direct = B.Engine(0, arena_bytes=128 << 20)
    graphed = B.Engine(0, arena_bytes=128 << 20)
    try:
        B.tn_ctx_set_graphs(direct.ctx, 0)
        B.tn_ctx_set_slice_block(direct.ctx, block)
        B.tn_ctx_set_slice_block(graphed.ctx, block)
        pd, pg = direct.load(blob), graphed.load(blob)
        ref = {0: direct.amplitudes(pd, w1, prec), 1: direct.amplitudes(pd, w2, prec)}
        replays = []
        for call in range(6):
            which = call % 2
            got = graphed.amplitudes(pg, w1 if which == 0 else w2, prec)
            replays.append(B.tn_last_exec_stats(graphed.ctx)["graph_replays"])
            print("call", call, "replays", replays[-1], flush=True)
            assert np.array_equal(got, ref[which]), call
        assert replays[:2] == [0, 0] and all(r > 0 for r in replays[2:])
        tol = 1e-5 if prec in (0, 1) else 1e-3
        for which, w in ((0, w1), (1, w2)):
            sv = statevector_amplitudes(circ, w)
            fp_error.check(ref[which], sv, 2.0 ** -8, tol, fp_error.floor(plan, prec, 2.0 ** -8),
                           "graphs set %d prec %d" % (which, prec))
    finally:
        direct.close()
        graphed.close()


def test_graphs_over_chunks_and_unload():
    """A small arena makes several chunks of one shape (the later ones
    replay); unloading the plan drops its graphs, and a reloaded plan runs
    correctly again."""
    from paper_2208_01498_amd import binding as B
    circ = lattice_circuit(5, 5, 10, 1311, "haar", "cz")
    words = random_bitstrings(25, 40, 1312)
    blob = _plan(circ, 2, 40).to_blob()
    info = B.tn_plan_validate(blob)
    small = int(max(1 << 20, info["peak_bytes_fixed"] + 8 * info["peak_bytes_per_b"]))
    ref_eng = B.Engine(0, arena_bytes=256 << 20)
    eng = B.Engine(0, arena_bytes=small)
    try:
        B.tn_ctx_set_graphs(ref_eng.ctx, 0)
        ref = ref_eng.amplitudes(ref_eng.load(blob), words, 0)
        for rnd in range(2):
            p = eng.load(blob)
            for call in range(3):
                got = eng.amplitudes(p, words, 0)
                st = B.tn_last_exec_stats(eng.ctx)
                print("round", rnd, "call", call, "chunks", st["n_chunks"], "replays", st["graph_replays"],
                      flush=True)
                assert st["n_chunks"] > 1
                assert np.array_equal(got, ref)
            assert st["graph_replays"] >= st["n_chunks"] - 1
            eng.unload(p)
    finally:
        ref_eng.close()
        eng.close()


def _small_arena_engine(B, blob, chunk_target):
    info = B.tn_plan_validate(blob)
    arena = int(max(1 << 20, info["peak_bytes_fixed"] + (chunk_target + 0.5) * info["peak_bytes_per_b"]))
    eng = B.Engine(0, arena_bytes=arena)
    B.tn_ctx_set_slice_block(eng.ctx, 0)
    return eng, arena


@pytest.mark.parametrize("prec", [0, 3])
def test_graph_key_includes_chunk_size(prec):
    """A call of c + c/2 bitstrings runs chunks of c and c/2; a call of c/2
    runs one chunk of c/2 under a layout planned for c/2.  The two last
    chunks have the same bitstring count but different workspace layouts, so
    alternating the calls (direct, captured, replayed) must never replay one
    layout's graph for the other: every result is bitwise the graphs-off
    result on the same arena, and matches the state vector."""
    from paper_2208_01498_amd import binding as B
    circ = lattice_circuit(5, 5, 10, 1321, "haar", "cz")
    words = random_bitstrings(25, 48, 1322)
    plan = _plan(circ, 2, 48)
    blob = plan.to_blob()
    eng, arena = _small_arena_engine(B, blob, 20)
    ref_eng = B.Engine(0, arena_bytes=arena)
    try:
        B.tn_ctx_set_slice_block(ref_eng.ctx, 0)
        B.tn_ctx_set_graphs(ref_eng.ctx, 0)
        p, pr = eng.load(blob), ref_eng.load(blob)
        eng.amplitudes(p, words, prec)
        c = B.tn_last_exec_stats(eng.ctx)["chunk"]
        print("chunk", c, "arena", arena, flush=True)
        assert 4 <= c < 48
        sizes = [c + c // 2, c // 2]
        ref = {n: ref_eng.amplitudes(pr, words[:n], prec) for n in sizes}
        for call in range(8):
            n = sizes[call % 2]
            got = eng.amplitudes(p, words[:n], prec)
            st = B.tn_last_exec_stats(eng.ctx)
            print("call", call, "nb", n, "chunk", st["chunk"], "chunks", st["n_chunks"],
                  "replays", st["graph_replays"], flush=True)
            assert np.array_equal(got, ref[n]), (call, n)
        sv = statevector_amplitudes(circ, words[:sizes[0]])
        typ = 2.0 ** (-circ.n / 2)
        fp_error.check(ref[sizes[0]], sv, typ, 1e-5 if prec == 0 else 1e-3,
                       fp_error.floor(plan, prec, typ), "chunk-key prec %d" % prec)
    finally:
        eng.close()
        ref_eng.close()


def test_served_batches_of_different_sizes_replay_their_own_graphs():
    """One slot, so every served batch starts at the same arena offset;
    batches of c + c/2 and c/2 bitstrings alternate (each waits for the
    previous one), and every result is bitwise the graphs-off direct run."""
    import time
    from paper_2208_01498_amd import binding as B
    circ = lattice_circuit(5, 5, 10, 1331, "haar", "cz")
    words = random_bitstrings(25, 48, 1332)
    blob = _plan(circ, 2, 48).to_blob()
    # a served batch takes at most half the arena, so the graphs-off
    # reference runs on half of it and chunks exactly as the server does
    eng, arena = _small_arena_engine(B, blob, 40)
    ref_eng = B.Engine(0, arena_bytes=arena // 2)
    try:
        B.tn_server_config(eng.ctx, 1, 64)
        B.tn_ctx_set_slice_block(ref_eng.ctx, 0)
        B.tn_ctx_set_graphs(ref_eng.ctx, 0)
        p, pr = eng.load(blob), ref_eng.load(blob)
        ref_eng.amplitudes(pr, words, 0)
        c = B.tn_last_exec_stats(ref_eng.ctx)["chunk"]
        print("served chunk", c, "arena", arena, flush=True)
        assert 4 <= c < 48
        sizes = [c + c // 2, c // 2]
        ref = {n: ref_eng.amplitudes(pr, words[:n], 0) for n in sizes}
        for call in range(8):
            n = sizes[call % 2]
            t = B.tn_submit(eng.ctx, p, words[:n], 0)
            deadline = time.time() + 60
            res = None
            while res is None:
                assert time.time() < deadline, "served batch did not finish"
                res = B.tn_poll(eng.ctx, t, n)
                if res is None:
                    time.sleep(0.002)
            print("served call", call, "nb", n, flush=True)
            assert np.array_equal(res[0], ref[n]), (call, n)
    finally:
        eng.close()
        ref_eng.close()
