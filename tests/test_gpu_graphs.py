"""Captured HIP graphs of the executor: replays equal direct launches."""
import numpy as np
import pytest

from circuits import lattice_circuit, random_bitstrings
from oracle import statevector_amplitudes

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
    blob = _plan(circ, 3, 12).to_blob()
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
            err = np.abs(ref[which] - sv) / np.maximum(np.abs(sv), 2.0 ** (-8))
            assert err.max() <= tol
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
