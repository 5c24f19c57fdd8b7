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
