"""Circuit container: an ordered gate list with complex128 matrices plus the
spatial position of every qubit (used by the geometric order search)."""
from dataclasses import dataclass, field
import json
import numpy as np


@dataclass
class Gate:
    qubits: tuple
    matrix: np.ndarray      # (2,2) or (4,4) complex128
    name: str = ""

    @property
    def arity(self):
        return len(self.qubits)


@dataclass
class Circuit:
    n: int
    gates: list
    positions: np.ndarray           # (n, d) float64 qubit coordinates
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __len__(self):
        return len(self.gates)

    def n_2q(self):
        return sum(1 for g in self.gates if g.arity == 2)

    def to_json(self):
        return json.dumps({
            "n": self.n, "name": self.name, "meta": self.meta,
            "positions": self.positions.tolist(),
            "gates": [{"q": list(g.qubits), "name": g.name,
                       "re": g.matrix.real.ravel().tolist(),
                       "im": g.matrix.imag.ravel().tolist()} for g in self.gates],
        })

    @staticmethod
    def from_json(s):
        d = json.loads(s)
        gates = []
        for g in d["gates"]:
            k = len(g["q"])
            m = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(2 ** k, 2 ** k)
            gates.append(Gate(tuple(g["q"]), m, g.get("name", "")))
        return Circuit(d["n"], gates, np.array(d["positions"], dtype=np.float64),
                       d.get("name", ""), d.get("meta", {}))
