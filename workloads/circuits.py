"""Seeded synthetic circuit generators (input data only).

This module builds the quantum circuits that both the HIP path and the CPU
checker consume.  It holds gate matrices and random circuit layouts and none
of the path-sampling arithmetic: no energies, no lattice, no sampling.

Conventions (the paper's, Sec. 2, two-qubit table Eq. (ET2)):
  * a gate matrix is indexed U[out][in];
  * a two-qubit gate acting on qubits (q0, q1) uses the index s_{q0} + 2*s_{q1}
    for both rows and columns (the paper orders the columns |00>, |10>, |01>,
    |11>, i.e. the first listed qubit is the low bit);
  * basis states of the register are little-endian: qubit q is bit q.

A circuit is a dict, serialised as JSON:
  {"name", "n", "d", "K", "input",
   "matrices": {kind: {"re": [[..]], "im": [[..]]}},
   "gates": [{"layer", "qubits", "kind"}]}
with layers numbered 1..d and the gates of one layer on disjoint qubits.
"""
from __future__ import annotations

import json
import math
import os
import random

R2 = 1.0 / math.sqrt(2.0)
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


# ----------------------------------------------------------------------------
# gate matrices, U[out][in] as (re, im) lists
# ----------------------------------------------------------------------------
def _c(z):
    z = complex(z)
    return z.real, z.imag


def _mat(rows):
    re = [[_c(z)[0] for z in r] for r in rows]
    im = [[_c(z)[1] for z in r] for r in rows]
    return re, im


def mat_h():
    return _mat([[R2, R2], [R2, -R2]])


def mat_s():
    return _mat([[1, 0], [0, 1j]])


def mat_t():
    return _mat([[1, 0], [0, complex(R2, R2)]])


def mat_sx():
    # sqrt(X) = 1/2 [[1+i, 1-i], [1-i, 1+i]]
    return _mat([[complex(0.5, 0.5), complex(0.5, -0.5)],
                 [complex(0.5, -0.5), complex(0.5, 0.5)]])


def mat_x():
    return _mat([[0, 1], [1, 0]])


def mat_rz(gamma):
    return _mat([[complex(math.cos(gamma / 2), -math.sin(gamma / 2)), 0],
                 [0, complex(math.cos(gamma / 2), math.sin(gamma / 2))]])


def mat_rh(theta):
    """Rotated Hadamard of Eq. (HadT): [[cos, sin], [sin, -cos]]."""
    c, s = math.cos(theta), math.sin(theta)
    return _mat([[c, s], [s, -c]])


def mat_cnot_tc():
    """CNOT on qubits (target, control): the paper's CNOT matrix of the
    Appendix, where the second listed qubit is the control."""
    return _mat([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]])


def mat_cz():
    return _mat([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, -1]])


def mat_cp(k):
    """Controlled phase with angle 2*pi/2**k (k = 1 is CZ)."""
    phi = 2.0 * math.pi / (2 ** k)
    if k == 1:
        return mat_cz()
    if k == 2:
        e = 1j
    else:
        e = complex(math.cos(phi), math.sin(phi))
    return _mat([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, e]])


def mat_hs():
    """H S = 1/sqrt(2) [[1, i], [1, -i]] (not symmetric)."""
    return _mat([[R2, complex(0, R2)], [R2, complex(0, -R2)]])


def mat_sh():
    """S H = 1/sqrt(2) [[1, 1], [i, -i]] (not symmetric)."""
    return _mat([[R2, R2], [complex(0, R2), complex(0, -R2)]])


ONE_Q = {"H": mat_h, "S": mat_s, "T": mat_t, "SX": mat_sx, "X": mat_x, "HS": mat_hs, "SH": mat_sh}


def gate1(layer, q, kind, mat=None):
    re, im = mat if mat is not None else ONE_Q[kind]()
    return {"layer": layer, "qubits": [q], "kind": kind, "re": re, "im": im}


def cnot(layer, control, target):
    re, im = mat_cnot_tc()
    return {"layer": layer, "qubits": [target, control], "kind": "CNOT",
            "re": re, "im": im}


def cz(layer, a, b):
    re, im = mat_cz()
    return {"layer": layer, "qubits": [a, b], "kind": "CZ", "re": re, "im": im}


def cp(layer, a, b, k):
    re, im = mat_cp(k)
    return {"layer": layer, "qubits": [a, b], "kind": "CP%d" % k,
            "re": re, "im": im}


def circuit(name, n, d, K, gates, input_state=0):
    """Assemble a circuit; matrices are stored once per gate kind under
    "matrices" and each gate names its kind."""
    mats = {}
    slim = []
    for g in gates:
        m = {"re": g["re"], "im": g["im"]}
        if g["kind"] in mats and mats[g["kind"]] != m:
            raise ValueError("two matrices for gate kind %s" % g["kind"])
        mats[g["kind"]] = m
        slim.append({"layer": g["layer"], "qubits": g["qubits"],
                     "kind": g["kind"]})
    return {"name": name, "n": n, "d": d, "K": K, "input": input_state,
            "matrices": mats, "gates": slim}


def gate_matrix(c, g):
    """(re, im) of gate g of circuit c."""
    m = g if "re" in g else c["matrices"][g["kind"]]
    return m["re"], m["im"]


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def tiny_ghz_t():
    """n=3, d=5: H(q0), CNOT(0->1), CNOT(1->2), T(q2), H(q1); input |000>."""
    g = [gate1(1, 0, "H"), cnot(2, 0, 1), cnot(3, 1, 2), gate1(4, 2, "T"),
         gate1(5, 1, "H")]
    return circuit("tiny_n3_d5", 3, 5, 3, g, 0)


def hadamard_chain(d, K=3, input_state=0):
    """One qubit driven by d Hadamard gates (Sec. 4, Fig. 3/4)."""
    g = [gate1(l, 0, "H") for l in range(1, d + 1)]
    return circuit("hchain_d%d" % d, 1, d, K, g, input_state)


def rotated_hadamard_chain(d, theta, K=1, input_state=0):
    """One qubit driven by d rotated Hadamards of Eq. (HadT)."""
    g = [gate1(l, 0, "RH", mat_rh(theta)) for l in range(1, d + 1)]
    return circuit("rhchain_d%d" % d, 1, d, K, g, input_state)


def random_clifford_t(n, d, seed, K=3, p1=0.6, name=None):
    """Random Clifford+T layers.  Per layer the qubits are visited in a
    shuffled order; an unused qubit gets, with probability p1, a one-qubit
    gate drawn uniformly from {H, S, T}; otherwise it is paired with a
    uniformly drawn unused partner and gets CNOT (itself as control) or CZ
    with probability 1/2 each.  With no partner left it gets a one-qubit
    gate instead."""
    rng = random.Random(seed)
    gates = []
    for layer in range(1, d + 1):
        order = list(range(n))
        rng.shuffle(order)
        used = set()
        for q in order:
            if q in used:
                continue
            if rng.random() < p1:
                gates.append(gate1(layer, q, rng.choice(["H", "S", "T"])))
                used.add(q)
                continue
            free = [p for p in range(n) if p not in used and p != q]
            if not free:
                gates.append(gate1(layer, q, rng.choice(["H", "S", "T"])))
                used.add(q)
                continue
            p = rng.choice(free)
            if rng.random() < 0.5:
                gates.append(cnot(layer, q, p))
            else:
                gates.append(cz(layer, min(q, p), max(q, p)))
            used.add(q)
            used.add(p)
    return circuit(name or "rct_n%d_d%d_s%d" % (n, d, seed), n, d, K, gates, 0)


def brickwork(n, d, seed, K=4, one_q=("H", "S", "T", "SX"), kmax=4,
              name=None):
    """Odd layers: every qubit gets a one-qubit gate drawn uniformly from
    one_q.  Even layer 2m: neighbour pairs (0,1),(2,3),... when m is odd and
    (1,2),(3,4),... when m is even; each pair gets CP(2*pi/2**k) with k
    uniform in 1..kmax (k = 1 is CZ)."""
    rng = random.Random(seed)
    gates = []
    for layer in range(1, d + 1):
        if layer % 2 == 1:
            for q in range(n):
                gates.append(gate1(layer, q, rng.choice(list(one_q))))
        else:
            m = layer // 2
            start = 0 if m % 2 == 1 else 1
            for a in range(start, n - 1, 2):
                k = rng.randint(1, kmax)
                gates.append(cp(layer, a, a + 1, k))
    return circuit(name or "brick_n%d_d%d_s%d" % (n, d, seed), n, d, K,
                   gates, 0)


def rotated_brickwork(n, d, seed, theta, K=3, name=None):
    """Brickwork whose odd layers hold rotated Hadamards U(theta) or T on
    each qubit and whose even layers hold CNOTs on neighbour pairs, so that
    non-uniform real energies couple wires through the XOR cones."""
    rng = random.Random(seed)
    gates = []
    for layer in range(1, d + 1):
        if layer % 2 == 1:
            for q in range(n):
                if rng.random() < 0.75:
                    gates.append(gate1(layer, q, "RH", mat_rh(theta)))
                else:
                    gates.append(gate1(layer, q, "T"))
        else:
            m = layer // 2
            start = 0 if m % 2 == 1 else 1
            for a in range(start, n - 1, 2):
                gates.append(cnot(layer, a, a + 1))
    return circuit(name or "rbrick_n%d_d%d_s%d" % (n, d, seed), n, d, K,
                   gates, 0)


def batched_set(count=256, total_chains=1 << 22, seed0=1000):
    """`count` random Clifford+T circuits with n ~ U{4..16}, d ~ U{4..32}
    (circuit i drawn from seed seed0 + i) and chain counts proportional to
    2**n in units of 64 (largest remainders first, at least 64 each)."""
    circs = []
    for i in range(count):
        rng = random.Random(seed0 + i)
        n = rng.randint(4, 16)
        d = rng.randint(4, 32)
        c = random_clifford_t(n, d, seed0 + i, K=3,
                              name="batch%03d_n%d_d%d" % (i, n, d))
        circs.append(c)
    units = total_chains // 64
    weights = [2 ** c["n"] for c in circs]
    tot = float(sum(weights))
    raw = [units * w / tot for w in weights]
    alloc = [max(1, int(math.floor(r))) for r in raw]
    rest = units - sum(alloc)
    order = sorted(range(count), key=lambda i: -(raw[i] - math.floor(raw[i])))
    j = 0
    while rest > 0:
        alloc[order[j % count]] += 1
        rest -= 1
        j += 1
    while rest < 0:  # only if the minimum of one unit overshot
        i = max(range(count), key=lambda i: alloc[i])
        alloc[i] -= 1
        rest += 1
    chains = [64 * a for a in alloc]
    return circs, chains


# ----------------------------------------------------------------------------
# named workloads and JSON io
# ----------------------------------------------------------------------------
WORKLOADS = {
    "tiny": dict(make=tiny_ghz_t, chains=1024, burn_in=200, sweeps=2000),
    "rct12": dict(make=lambda: random_clifford_t(12, 40, 1, K=3),
                  chains=65536, burn_in=200, sweeps=10000),
    "brick20": dict(make=lambda: brickwork(20, 24, 1, K=4),
                    chains=262144, burn_in=200, sweeps=20000),
    "brick16": dict(make=lambda: brickwork(16, 24, 1, K=3,
                                           one_q=("H", "S", "T", "SX"),
                                           kmax=1),
                    chains=131072, burn_in=200, sweeps=2000),
    # rct12's shape with Toffoli and Peres gates (three-qubit products)
    "rctt12": dict(make=lambda: random_clifford_t_toffoli(12, 40, 1, K=3),
                   chains=65536, burn_in=200, sweeps=10000),
    # rct12's shape with controlled Hadamards as soft zeros (J = 4)
    "rctch12": dict(make=lambda: random_clifford_t_ch(12, 40, 1, K=3, p_ch=0.15),
                    chains=65536, burn_in=200, sweeps=2000, soft_J=4.0),
}


def save(c, path):
    with open(path, "w") as f:
        json.dump(c, f, separators=(",", ":"))


def load(path):
    with open(path) as f:
        return json.load(f)


def workload_circuit(name):
    """Return the committed JSON circuit of a named workload (generated by
    `python -m workloads.circuits` and checked into workloads/data)."""
    p = os.path.join(DATA_DIR, name + ".json")
    if os.path.exists(p):
        return load(p)
    return WORKLOADS[name]["make"]()


def main():
    os.makedirs(DATA_DIR, exist_ok=True)
    for name, w in WORKLOADS.items():
        save(w["make"](), os.path.join(DATA_DIR, name + ".json"))
    circs, chains = batched_set()
    with open(os.path.join(DATA_DIR, "batch256.json"), "w") as f:
        json.dump({"circuits": circs, "chains": chains}, f,
                  separators=(",", ":"))


if __name__ == "__main__":
    main()


def random_asymmetric(n, d, seed, K=3):
    """Random layers whose one-qubit gates include the non-symmetric H S and
    S H (so a transposed gate matrix changes the result): per layer each
    qubit gets, with probability 0.6, a gate from {H, S, T, HS, SH}, else
    CNOT or CZ with an unused partner.  For checks of gate orientation."""
    rng = random.Random(seed)
    gates = []
    for layer in range(1, d + 1):
        order = list(range(n))
        rng.shuffle(order)
        used = set()
        for q in order:
            if q in used:
                continue
            free = [p for p in range(n) if p not in used and p != q]
            if rng.random() < 0.6 or not free:
                gates.append(gate1(layer, q, rng.choice(["H", "S", "T", "HS", "SH"])))
                used.add(q)
                continue
            p = rng.choice(free)
            if rng.random() < 0.5:
                gates.append(cnot(layer, q, p))
            else:
                gates.append(cz(layer, min(q, p), max(q, p)))
            used.add(q)
            used.add(p)
    return circuit(f"rasym_n{n}_d{d}_s{seed}", n, d, K, gates, 0)


def mat_perm3(perm):
    """Three-qubit permutation gate: input index i (s_{q0} + 2 s_{q1} +
    4 s_{q2}) goes to output perm[i]."""
    U = [[0] * 8 for _ in range(8)]
    for i in range(8):
        U[perm[i]][i] = 1
    return _mat(U)


# Toffoli on qubits (target, c1, c2): s_t XOR (s_c1 AND s_c2), the Appendix's
# CCNOT; Peres = Toffoli then CNOT(c1 -> c2), a permutation that is not its
# own inverse (so a transposed matrix changes the result)
TOFFOLI_PERM = [i ^ ((i >> 1) & (i >> 2) & 1) for i in range(8)]
PERES_PERM = [(lambda j: j ^ (((j >> 1) & 1) << 2))(i ^ ((i >> 1) & (i >> 2) & 1)) for i in range(8)]


def toffoli(layer, target, c1, c2):
    re, im = mat_perm3(TOFFOLI_PERM)
    return {"layer": layer, "qubits": [target, c1, c2], "kind": "CCNOT", "re": re, "im": im}


def peres(layer, target, c1, c2):
    re, im = mat_perm3(PERES_PERM)
    return {"layer": layer, "qubits": [target, c1, c2], "kind": "PERES", "re": re, "im": im}


def random_clifford_t_toffoli(n, d, seed, K=3, p1=0.5, p3=0.25, name=None):
    """Random Clifford+T layers with three-qubit permutation gates: per layer
    each unused qubit gets, with probability p1, a gate from {H, S, T};
    otherwise, with probability p3 and two unused partners, a Toffoli or a
    Peres gate (itself as target), else CNOT or CZ with one partner."""
    rng = random.Random(seed)
    gates = []
    for layer in range(1, d + 1):
        order = list(range(n))
        rng.shuffle(order)
        used = set()
        for q in order:
            if q in used:
                continue
            free = [p for p in range(n) if p not in used and p != q]
            if rng.random() < p1 or not free:
                gates.append(gate1(layer, q, rng.choice(["H", "S", "T"])))
                used.add(q)
                continue
            if len(free) >= 2 and rng.random() < p3:
                c1, c2 = rng.sample(free, 2)
                gates.append((toffoli if rng.random() < 0.5 else peres)(layer, q, c1, c2))
                used.update([q, c1, c2])
                continue
            p = rng.choice(free)
            if rng.random() < 0.5:
                gates.append(cnot(layer, q, p))
            else:
                gates.append(cz(layer, min(q, p), max(q, p)))
            used.add(q)
            used.add(p)
    return circuit(name or "rctt_n%d_d%d_s%d" % (n, d, seed), n, d, K, gates, 0)


def mat_ch_tc():
    """Controlled Hadamard on qubits (target, control): H on the target when
    the control (second listed qubit) is 1; zeros neither absent nor a
    permutation pattern."""
    r = 1.0 / math.sqrt(2.0)
    return _mat([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, r, r], [0, 0, r, -r]])


def mat_cry_tc(theta):
    """Controlled rotated Hadamard of Eq. (HadT) on (target, control)."""
    c, s = math.cos(theta), math.sin(theta)
    return _mat([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, c, s], [0, 0, s, -c]])


def ch(layer, control, target):
    re, im = mat_ch_tc()
    return {"layer": layer, "qubits": [target, control], "kind": "CH", "re": re, "im": im}


def crh(layer, control, target, theta, kind="CRH"):
    re, im = mat_cry_tc(theta)
    return {"layer": layer, "qubits": [target, control], "kind": kind, "re": re, "im": im}


def random_clifford_t_ch(n, d, seed, K=3, p1=0.55, p_ch=0.4, name=None):
    """Random Clifford+T layers with controlled-Hadamard gates: per layer
    each unused qubit gets, with probability p1, a gate from {H, S, T},
    otherwise a partner and, with probability p_ch, a controlled Hadamard
    (itself as control), else CNOT or CZ."""
    rng = random.Random(seed)
    gates = []
    for layer in range(1, d + 1):
        order = list(range(n))
        rng.shuffle(order)
        used = set()
        for q in order:
            if q in used:
                continue
            free = [p for p in range(n) if p not in used and p != q]
            if rng.random() < p1 or not free:
                gates.append(gate1(layer, q, rng.choice(["H", "S", "T"])))
                used.add(q)
                continue
            p = rng.choice(free)
            r = rng.random()
            if r < p_ch:
                gates.append(ch(layer, q, p))
            elif r < p_ch + (1 - p_ch) / 2:
                gates.append(cnot(layer, q, p))
            else:
                gates.append(cz(layer, min(q, p), max(q, p)))
            used.add(q)
            used.add(p)
    return circuit(name or "rctch_n%d_d%d_s%d" % (n, d, seed), n, d, K, gates, 0)
