"""The oracle's own compile of a circuit into a p-bit lattice (test
infrastructure only; independent of the library's compiler).

Paper passages followed:
  * Eq. (UE): each gate entry U_{p,q} = exp(-E_{p,q}).  Its real part gives
    the magnitude |U| = exp(-Re E) and its imaginary part the phase
    exp(-i Im E) = U/|U|, stored here as an integer bin k with
    U/|U| = exp(2 pi i k / 2^K).
  * Sec. 2 one/two-qubit tables (rows = output state, columns = input state;
    two-qubit index s_{q0} + 2 s_{q1} as in Eq. (ET2)).
  * Appendix "zero elements": a diagonal gate keeps its input p-bit
    (s_out = s_in, Rz and the exchange gate J12), a permutation gate
    fixes its output as a Boolean function of its input (NOT: s_out = 1 -
    s_in; CNOT: s_1 XOR s_2).  Only gates without zero entries create new
    independent p-bits (g(d) of Sec. 2).
  * Fig. 2 / Eq. (weightedS): the sampler needs p_C proportional to |psi_C|;
    with hard zeros eliminated every assignment of the free p-bits is a
    valid path.

  * Appendix CCNOT: a three-qubit permutation gate is also deterministic
    (s_1 XOR (s_2 AND s_3) for the Toffoli), but not affine.
  * Appendix, general zero elements: a gate whose zeros are neither absent
    nor a permutation pattern (controlled-H, controlled rotations) gets
    e^(-J) in place of each zero for sampling (soft_J); such a gate then
    creates free p-bits like a gate without zeros.  The chain samples the
    law with e^(-J) weights and bins only paths that avoid every soft zero,
    which are exactly the paths of the circuit with their weights |psi_C|
    (conditioning), whatever J.

The lattice bit of layer l (0..d) and qubit q has index l*n + q.  Without
three-qubit gates every lattice bit is an affine GF(2) form of the free
bits: a constant XOR a set of free bits.  The cone of free bit b is the set
of lattice bits whose form contains b; flipping b flips exactly its cone.
With a non-affine permutation gate the circuit is `nonlinear`: the lattice
of a free-bit assignment is then found by evaluating the gates layer by
layer (`forward_lattice`), which is the definition in every case.
"""
from __future__ import annotations

import math

import numpy as np

ZERO_TOL = 1e-12
PHASE_TOL = 1e-9
MAG_RTOL = 1e-9


class CompileError(ValueError):
    pass


class OGate:
    """One gate with its magnitude / phase tables indexed out * 2^a + in."""

    def __init__(self, g, n, K, soft_J=None):
        self.layer = g.layer
        self.qubits = list(g.qubits)
        self.a = len(g.qubits)
        U = g.U
        dim = 2 ** self.a
        self.in_bits = [(g.layer - 1) * n + q for q in g.qubits]
        self.out_bits = [g.layer * n + q for q in g.qubits]
        self.mag = np.zeros(dim * dim)
        self.ph = np.full(dim * dim, -1, dtype=np.int64)
        nz = np.zeros((dim, dim), dtype=bool)
        for o in range(dim):
            for i in range(dim):
                re, im = float(U[o, i].real), float(U[o, i].imag)
                m = math.sqrt(re * re + im * im)
                if m <= ZERO_TOL:
                    continue
                nz[o, i] = True
                self.mag[o * dim + i] = m
                theta = math.atan2(im, re)
                step = 2.0 * math.pi / (2 ** K)
                k = int(round(theta / step))
                if abs(theta - k * step) > PHASE_TOL:
                    raise CompileError("phase off the 2pi/2^K grid")
                self.ph[o * dim + i] = k % (2 ** K)
        if nz.all():
            self.kind = "branch"
            self.perm = None
            if self.a > 2:
                raise CompileError("three-qubit gates must be permutations")
        elif (nz.sum(axis=0) == 1).all() and (nz.sum(axis=1) == 1).all():
            self.perm = [int(np.nonzero(nz[:, i])[0][0]) for i in range(dim)]
            self.kind = "copy" if self.perm == list(range(dim)) else "derived"
        elif soft_J is not None and self.a <= 2:
            self.kind = "branch"
            self.perm = None
        else:
            raise CompileError("gate with partial zero pattern")
        # sampling magnitudes: e^(-J) at the soft zeros of a gate that has
        # both zero and nonzero entries but no permutation pattern
        self.soft = np.zeros(dim * dim, dtype=bool)
        if self.kind == "branch" and not nz.all():
            self.soft = ~nz.ravel()
        self.mag_s = np.where(self.soft, math.exp(-soft_J) if soft_J is not None else 0.0, self.mag)
        mags = self.mag_s[self.mag_s > 0]
        self.const_mag = bool(mags.max() - mags.min() <= MAG_RTOL * mags.max())
        cols = [sum(self.mag[o * dim + i] for o in range(dim)) for i in range(dim)]
        self.col_sum = cols[0] if max(cols) - min(cols) <= MAG_RTOL * max(cols) else None

    @property
    def scope(self):
        return set(self.in_bits) | set(self.out_bits)

    def index(self, bits):
        """Table index of this gate for the lattice given as a bit array."""
        i = sum(int(bits[p]) << j for j, p in enumerate(self.in_bits))
        o = sum(int(bits[p]) << j for j, p in enumerate(self.out_bits))
        return o * (2 ** self.a) + i


def _xor(f1, f2):
    return (f1[0] ^ f2[0], f1[1] ^ f2[1])


class Compiled:
    pass


def compile_circuit(circ, soft_J=None):
    n, d, K = circ.n, circ.d, circ.K
    L = n * (d + 1)
    gates = [OGate(g, n, K, soft_J) for g in circ.gates]

    # affine forms (constant bit, frozenset of free bits) per lattice bit;
    # None once a bit depends on a non-affine gate
    nonlinear = False
    forms = [None] * L
    for q in range(n):
        forms[q] = ((circ.input >> q) & 1, frozenset())
    free_pos = []
    for layer in range(1, d + 1):
        lg = [g for g in gates if g.layer == layer]
        touched = {}
        for g in lg:
            for q in g.qubits:
                touched[q] = g
        # new free bits of this layer, numbered by ascending lattice index
        for q in range(n):
            g = touched.get(q)
            if g is not None and g.kind == "branch":
                b = len(free_pos)
                free_pos.append(layer * n + q)
                forms[layer * n + q] = (0, frozenset([b]))
        for q in range(n):
            if q not in touched:
                forms[layer * n + q] = forms[(layer - 1) * n + q]
        for g in lg:
            if g.kind == "branch":
                continue
            ins = [forms[p] for p in g.in_bits]
            dim = 2 ** g.a
            # output bit j as an affine function of the input bits:
            # out_j(in) = c_j XOR sum_t A_jt in_t, read off perm at 0 and e_t
            for j in range(g.a):
                c = (g.perm[0] >> j) & 1
                A = [((g.perm[1 << t] >> j) & 1) ^ c for t in range(g.a)]
                affine = True
                for i in range(dim):
                    want = (g.perm[i] >> j) & 1
                    got = c
                    for t in range(g.a):
                        got ^= A[t] & ((i >> t) & 1)
                    if want != got:
                        affine = False
                f = (c, frozenset())
                for t in range(g.a):
                    if A[t] and f is not None:
                        f = None if ins[t] is None else _xor(f, ins[t])
                if not affine:
                    nonlinear = True
                    f = None
                forms[g.out_bits[j]] = f
    h = len(free_pos)
    cone = [set() for _ in range(h)]
    if nonlinear:
        if not all(g.const_mag for g in gates):
            raise CompileError("non-affine gates need every gate magnitude constant")
        cone = None
    else:
        for p, (_, s) in enumerate(forms):
            for b in s:
                cone[b].add(p)

    # real-energy factors of each free bit: gates whose magnitude is not
    # constant and whose scope meets the cone, in gate order
    factors = []
    for b in range(h):
        factors.append([gi for gi, g in enumerate(gates)
                        if not g.const_mag and g.scope & cone[b]] if cone is not None else [])
    fscope = [set().union(*[gates[gi].scope for gi in factors[b]]) if factors[b] else set()
              for b in range(h)]

    # conflict graph and greedy colouring in ascending free-bit order
    colour = [0] * h
    for b in range(h):
        used = set()
        for b2 in range(b):
            if cone is not None and ((cone[b2] & fscope[b]) or (cone[b] & fscope[b2])):
                used.add(colour[b2])
        c = 0
        while c in used:
            c += 1
        colour[b] = c
    ncol = max(colour) + 1 if h else 0
    order = sorted(range(h), key=lambda b: (colour[b], b))

    Z = 1.0
    for g in gates:
        if g.col_sum is None:
            Z = None
            break
        Z *= g.col_sum

    out = Compiled()
    out.nonlinear = nonlinear
    out.circuit = circ
    out.n, out.d, out.K, out.L = n, d, K, L
    out.W = (L + 31) // 32
    out.gates = gates
    out.forms = forms
    out.free_pos = free_pos
    out.h = h
    out.cone = cone
    out.const = forward_lattice(out, [0] * h) if nonlinear else \
        np.array([forms[p][0] for p in range(L)], dtype=np.uint8)
    out.factors = factors
    out.colour = colour
    out.ncolours = ncol
    out.order = order
    out.Z = Z
    out.circuit = circ
    return out


def forward_lattice(comp, f):
    """Lattice bits for the free-bit assignment f, gate by gate in layer
    order: layer 0 is the input state, an idle qubit copies its bit, a gate
    without zero entries takes its outputs from the free bits (numbered by
    ascending lattice index), and a permutation gate maps its input bits to
    the output of its one nonzero entry (Appendix)."""
    n, d = comp.n, comp.d
    x = np.zeros(comp.L, dtype=np.uint8)
    for q in range(n):
        x[q] = (comp.circuit.input >> q) & 1
    slot = {p: b for b, p in enumerate(comp.free_pos)}
    for layer in range(1, d + 1):
        for q in range(n):
            x[layer * n + q] = x[(layer - 1) * n + q]
        for g in comp.gates:
            if g.layer != layer:
                continue
            if g.kind == "branch":
                for p in g.out_bits:
                    x[p] = f[slot[p]]
            else:
                i = sum(int(x[p]) << j for j, p in enumerate(g.in_bits))
                o = g.perm[i]
                for j, p in enumerate(g.out_bits):
                    x[p] = (o >> j) & 1
    return x


def lattice_from_free(comp, f):
    """Lattice bits for the free-bit assignment f (sequence of 0/1): the
    constant lattice with the cones of the set free bits flipped (affine
    circuits), else `forward_lattice`."""
    if comp.nonlinear:
        return forward_lattice(comp, f)
    x = comp.const.copy()
    for b in range(comp.h):
        if f[b]:
            for p in comp.cone[b]:
                x[p] ^= 1
    return x


def path_weight(comp, x):
    """(|psi_C|, phase bin) of the path given as lattice bits: the product
    of gate entries of Eq. (path); idle qubits contribute 1."""
    m = 1.0
    k = 0
    for g in comp.gates:
        idx = g.index(x)
        if g.mag[idx] == 0.0:
            return 0.0, 0
        m *= g.mag[idx]
        k += int(g.ph[idx])
    return m, k % (2 ** comp.K)


def violates(comp, x):
    """True if the path given as lattice bits meets a soft zero of a gate."""
    return any(g.soft[g.index(x)] for g in comp.gates)


def sampling_weight(comp, x):
    """Product of the sampling magnitudes (e^(-J) at soft zeros)."""
    m = 1.0
    for g in comp.gates:
        m *= g.mag_s[g.index(x)]
    return m


def alpha_of(comp, x):
    n, d = comp.n, comp.d
    return sum(int(x[d * n + q]) << q for q in range(n))


def enumerate_free(comp):
    """All 2^h paths: list of (free bits, lattice, |psi|, phase bin, alpha)."""
    res = []
    for v in range(2 ** comp.h):
        f = [(v >> b) & 1 for b in range(comp.h)]
        x = lattice_from_free(comp, f)
        m, k = path_weight(comp, x)
        res.append((f, x, m, k, alpha_of(comp, x)))
    return res


def pack_words(bits, W):
    w = np.zeros(W, dtype=np.uint32)
    for p, v in enumerate(bits):
        if v:
            w[p >> 5] |= np.uint32(1 << (p & 31))
    return w
