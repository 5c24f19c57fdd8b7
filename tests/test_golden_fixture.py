"""The stored full-size oracle amplitudes still describe the circuits and
bitstrings that the generators produce (a changed generator would make the
fixture stale and the full-size GPU comparison meaningless)."""
import hashlib
import json
import os

import pytest

from circuits import make_config

PATH = os.path.join(os.path.dirname(__file__), "golden", "fullsize_oracle_amplitudes.json")


@pytest.mark.parametrize("name", ["cfg3", "cfg2"])
def test_stored_oracle_fixture_matches_generators(name):
    data = json.load(open(PATH))
    assert name in data
    entry = data[name]
    circ, words, _ = make_config(name)
    assert hashlib.sha256(circ.to_json().encode()).hexdigest() == entry["circuit_sha256"]
    stored = [int(r["bitstring"]) for r in entry["amplitudes"]]
    # the first bitstrings of the batch, in order (16 of the 6x6 workload's 256)
    assert len(stored) >= (16 if name == "cfg2" else 4)
    assert stored == [int(w) for w in words[:len(stored)]]
    for r in entry["amplitudes"]:
        a = complex(r["re"], r["im"])
        # a contracted amplitude of a random circuit: finite, nonzero, far below 1
        assert 0.0 < abs(a) < 2.0 ** (-circ.n / 2 + 8)
