"""Circuit reader of the oracle (test infrastructure only).

Reads the JSON circuits written by `workloads.circuits` into plain Python:
gate matrices U[out][in] as complex numpy arrays (Sec. 2, one- and two-qubit
tables; a two-qubit index is s_{q0} + 2 s_{q1} as in Eq. (ET2)).
"""
from __future__ import annotations

import json

import numpy as np


class Gate:
    def __init__(self, layer, qubits, U, kind=""):
        self.layer = int(layer)
        self.qubits = [int(q) for q in qubits]
        self.U = np.asarray(U, dtype=np.complex128)
        self.kind = kind
        a = len(self.qubits)
        assert self.U.shape == (2 ** a, 2 ** a), "gate matrix shape"

    @property
    def arity(self):
        return len(self.qubits)


class Circuit:
    def __init__(self, n, d, K, input_state, gates, name=""):
        self.n, self.d, self.K = int(n), int(d), int(K)
        self.input = int(input_state)
        self.name = name
        # the oracle's gate order: by layer, then by lowest qubit
        self.gates = sorted(gates, key=lambda g: (g.layer, min(g.qubits)))
        for g in self.gates:
            assert 1 <= g.layer <= self.d
            assert all(0 <= q < self.n for q in g.qubits)
            assert len(set(g.qubits)) == len(g.qubits)
        seen = {}
        for g in self.gates:
            for q in g.qubits:
                key = (g.layer, q)
                assert key not in seen, "gates of one layer must be disjoint"
                seen[key] = g


def from_dict(c):
    gates = []
    for g in c["gates"]:
        m = g if "re" in g else c["matrices"][g["kind"]]
        U = np.array(m["re"], dtype=np.float64) + 1j * np.array(m["im"], dtype=np.float64)
        gates.append(Gate(g["layer"], g["qubits"], U, g.get("kind", "")))
    return Circuit(c["n"], c["d"], c["K"], c.get("input", 0), gates, c.get("name", ""))


def load(path):
    with open(path) as f:
        return from_dict(json.load(f))
