"""The C-ABI library on the host: it loads, exports every symbol the header
declares, and its plan validator accepts good blobs and rejects malformed
ones (no device calls)."""
import os
import re
import struct

import pytest

from circuits import make_config
from paper_2208_01498_amd.planner.plan import make_plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2208_01498_amd import binding
    binding.load_library()
    return binding


def test_exports_every_declared_symbol(B):
    hdr = open(os.path.join(ROOT, "include", "tnamp.h")).read()
    names = set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(tn_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 15
    lib = B.load_library()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(B.EXPORTED) <= names


@pytest.fixture(scope="module")
def blob():
    circ, _, _ = make_config("cfg1")
    return make_plan(circ, n_slices=2, B=8).to_blob()


def test_valid_blob(B, blob):
    info = B.tn_plan_validate(blob)
    assert info["n_qubits"] == 16
    assert info["n_sliced"] == 2
    assert info["flops_total_per_b"] > 0


def _rejects(B, data):
    with pytest.raises(B.TnError) as e:
        B.tn_plan_validate(data)
    assert e.value.code == B.TN_EINVAL


def test_rejects_malformed(B, blob):
    _rejects(B, b"XXXX" + blob[4:])                                  # magic
    _rejects(B, blob[:4] + struct.pack("<I", 7) + blob[8:])          # version
    for cut in (10, 60, len(blob) // 2, len(blob) - 3):
        _rejects(B, blob[:cut])                                      # truncated
    _rejects(B, blob + b"\0")                                        # trailing bytes


def test_rejects_bad_steps(B):
    circ, _, _ = make_config("cfg1")
    plan = make_plan(circ, n_slices=0, B=8)
    # an operand used twice
    st = plan.step_layout
    saved = dict(st[3])
    st[3]["b"] = st[2]["a"]
    with pytest.raises(B.TnError):
        B.tn_plan_validate(plan.to_blob())
    st[3].update(saved)
    B.tn_plan_validate(plan.to_blob())
    # an output order that is not a GEMM layout
    for s in st:
        if len(s["c_order"]) >= 3:
            s["c_order"] = s["c_order"][1:] + s["c_order"][:1]
            break
    with pytest.raises(B.TnError):
        B.tn_plan_validate(plan.to_blob())


def test_rejects_label_out_of_range(B, blob):
    # the first leaf's first label id sits right after the label table
    n_labels = struct.unpack_from("<I", blob, 12)[0]
    off = 4 + 7 * 4 + 16 + 8 * n_labels + 4
    bad = bytearray(blob)
    struct.pack_into("<I", bad, off, n_labels + 5)
    _rejects(B, bytes(bad))


def _scattered_step(plan):
    """Index of a step whose output order interleaves its row and column
    labels, and that step's (A order, B order)."""
    order = {i: plan.leaf_order[i] for i in range(len(plan.net.factors))}
    nid = len(plan.net.factors)
    for si, ((a, b), lay) in enumerate(zip(plan.steps, plan.step_layout)):
        oa = lay["permA"] or order[a]
        ob = lay["permB"] or order[b]
        MA, NB = set(oa) - set(ob), set(ob) - set(oa)
        rest = [l for l in lay["c_order"] if l in MA or l in NB]
        ma = [l for l in oa if l in MA]
        nb = [l for l in ob if l in NB]
        if rest != ma + nb and rest != nb + ma and len(ma) >= 2:
            return si, ma
        order[nid] = lay["c_order"]
        nid += 1
    return None, None


def test_interleaved_output_order(B):
    """An output order that interleaves the row labels (in A's order) with
    the column labels (in B's order) is accepted; the same order with two
    row labels exchanged is not a bit deposit of the GEMM's row index and
    is rejected with the loader's message for it."""
    circ, _, _ = make_config("cfg1")
    plan = make_plan(circ, n_slices=0, B=8)
    si, ma = _scattered_step(plan)
    assert si is not None, "planner produced no interleaved output order"
    B.tn_plan_validate(plan.to_blob())
    oc = plan.step_layout[si]["c_order"]
    i, j = oc.index(ma[0]), oc.index(ma[1])
    bad = list(oc)
    bad[i], bad[j] = bad[j], bad[i]
    plan.step_layout[si]["c_order"] = bad
    with pytest.raises(B.TnError) as e:
        B.tn_plan_validate(plan.to_blob())
    assert e.value.code == B.TN_EINVAL
    assert "interleaved" in str(e.value)
