"""Host-side checks of the HIP library (no GPU): the C ABI loads and exports
every declared symbol, the library's circuit compile equals the oracle's
independent compile, error codes, and FP64 amplitude recovery."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import chain as och
from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from workloads import circuits as wc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2007_07379_amd", "libpbit.so")


@pytest.fixture(scope="module")
def pb():
    if not os.path.exists(LIB):
        from paper_2007_07379_amd import build
        build.build()
    from paper_2007_07379_amd import pbit
    return pbit


def test_every_declared_symbol_is_exported(pb):
    decl = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        txt = open(os.path.join(ROOT, "include", f)).read()
        decl |= set(re.findall(r"\b(pbit_[a-z0-9_]+)\s*\(", txt))
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = decl - exported
    assert not missing, missing
    assert {"pbit_compile_circuit", "pbit_gibbs_run", "pbit_mh_run", "pbit_amplitudes"} <= decl


# --- blob reader (layout of paper_2007_07379_amd/csrc/blob.h) -------------
H = dict(MAGIC=0, N=1, D=2, K=3, W=4, H=5, L=6, CID=7, NCOL=8, UNIFORM=9, AWORD=10, ASHIFT=11,
         PCONST=12, LINMASK=13, NQD=14, FW=15, OFF_CONST=16, OFF_FPOS=17, OFF_CONE=18, OFF_LIN=19,
         OFF_QD=20, OFF_COLIDX=21, OFF_COLENT=22, OFF_THRINFO=23, OFF_THRTAB=24, THR_TOTAL=25,
         HBITS=26, TOTAL=27, WS=28, NBLK=29, TOGW=30, OFF_TOG=31, NQG=32, OFF_QG=33, NRE=34, OFF_RE=35,
         NY=36, OFF_Y=37, NSOFT=38, OFF_SOFT=39)
MAX_FW = 8
THR_STRIDE = 14


class Blob:
    def __init__(self, b):
        self.b = b
        g = lambda k: int(b[H[k]])
        self.n, self.d, self.K, self.W, self.h = g("N"), g("D"), g("K"), g("W"), g("H")
        self.WS = g("WS")
        self.ncol = g("NCOL")
        self.uniform = g("UNIFORM")
        o = g("OFF_CONST")
        self.const = b[o:o + self.W]
        o = g("OFF_FPOS")
        self.fpos = [int(v) for v in b[o:o + self.h]]
        o = g("OFF_CONE")
        self.cone = b[o:o + self.h * self.WS].reshape(self.h, self.WS)[:, :self.W] if self.h else None
        o = g("OFF_LIN")
        self.lin = b[o:o + self.K * self.WS].reshape(self.K, self.WS)
        self.pconst = g("PCONST")
        self.qd = []
        o = g("OFF_QD")
        st = 2 + self.K * self.WS
        for q in range(g("NQD")):
            rec = b[o + q * st:o + (q + 1) * st]
            self.qd.append((int(rec[0]), rec[2:].reshape(self.K, self.WS)))
        self.qg = []
        o = g("OFF_QG")
        for _ in range(g("NQG")):
            t, m = int(b[o]), int(b[o + 1])
            o += 2
            items = []
            for _ in range(m):
                items.append((int(b[o]), b[o + 1:o + 1 + self.WS]))
                o += 1 + self.WS
            self.qg.append((t, items))
        ci, ce = g("OFF_COLIDX"), g("OFF_COLENT")
        self.colour = [None] * self.h
        for c in range(self.ncol):
            for k in range(MAX_FW):
                off, cnt = int(b[ci + (c * MAX_FW + k) * 2]), int(b[ci + (c * MAX_FW + k) * 2 + 1])
                for e in range(cnt):
                    ent = int(b[ce + off + e])
                    j, m = ent >> 4, ent & 15
                    for t in range(4):
                        if m >> t & 1:
                            assert self.colour[4 * j + t] is None
                            self.colour[4 * j + t] = c
        self.thr_off = g("OFF_THRINFO")
        self.tab_off = g("OFF_THRTAB")
        self.aword, self.ashift = g("AWORD"), g("ASHIFT")

    def threshold(self, bidx, x):
        if self.uniform:
            return 1 << 31
        rec = self.b[self.thr_off + bidx * THR_STRIDE:self.thr_off + (bidx + 1) * THR_STRIDE]
        toff, ns = int(rec[0]), int(rec[1])
        idx = 0
        for j in range(ns):
            p = int(rec[2 + j])
            idx |= ((int(x[p >> 5]) >> (p & 31)) & 1) << j
        return int(self.b[self.tab_off + toff + idx])

    def phase(self, x):
        xi = 0
        for w in range(self.W):
            xi |= int(x[w]) << (32 * w)
        acc = self.pconst
        for t in range(self.K):
            m = 0
            for w in range(self.W):
                m |= int(self.lin[t, w]) << (32 * w)
            acc += bin(xi & m).count("1") << t
        for delta, planes in self.qd:
            y = xi & (xi >> delta)
            for t in range(self.K):
                m = 0
                for w in range(self.W):
                    m |= int(planes[t, w]) << (32 * w)
                acc += bin(y & m).count("1") << t
        for t, items in self.qg:
            z = 0
            for delta, mk in items:
                m = 0
                for w in range(self.W):
                    m |= int(mk[w]) << (32 * w)
                assert z & m == 0 or True
                z |= (xi >> delta) & m
            acc += bin(xi & z).count("1") << t
        return acc % (1 << self.K)


def _cases():
    return [
        ("tiny", wc.tiny_ghz_t()),
        ("rct12", wc.workload_circuit("rct12")),
        ("brick20", wc.workload_circuit("brick20")),
        ("brick16", wc.workload_circuit("brick16")),
        ("rct_small", wc.random_clifford_t(5, 7, 77, K=3)),
        ("rhchain", wc.rotated_hadamard_chain(10, math.pi / 8, K=1)),
        ("rhchain3", wc.rotated_hadamard_chain(7, math.pi / 3, K=2)),
        ("rbrick", wc.rotated_brickwork(4, 6, 5, math.pi / 8, K=3)),
        ("hchain", wc.hadamard_chain(9, K=1)),
        ("rasym", wc.random_asymmetric(6, 10, 3, K=3)),
        # inputs beta != 0 (Eq. (U)): layer 0 clamped to beta
        ("tiny_b5", dict(wc.tiny_ghz_t(), input=5)),
        ("rct_small_b22", dict(wc.random_clifford_t(5, 7, 77, K=3), input=0b10110)),
        ("rhchain_b1", wc.rotated_hadamard_chain(10, math.pi / 8, K=1, input_state=1)),
        ("rbrick_b11", dict(wc.rotated_brickwork(4, 6, 5, math.pi / 8, K=3), input=0b1011)),
        ("rasym_b63", dict(wc.random_asymmetric(6, 10, 3, K=3), input=63)),
    ]


@pytest.mark.parametrize("name,c", _cases(), ids=[n for n, _ in _cases()])
def test_library_compile_equals_oracle(pb, name, c):
    lib_set = pb.CircuitSet(c)
    blob = Blob(lib_set.export(0))
    comp = ocomp.compile_circuit(oc.from_dict(c))
    info = lib_set.info(0)
    assert (blob.n, blob.d, blob.K, blob.W, blob.h) == (comp.n, comp.d, comp.K, comp.W, comp.h)
    assert blob.ncol == comp.ncolours
    assert bool(blob.uniform) == all(not f for f in comp.factors)
    assert np.array_equal(blob.const, ocomp.pack_words(comp.const, comp.W))
    assert blob.fpos == list(comp.free_pos)
    tables = och.Tables(comp)
    if comp.h:
        assert np.array_equal(blob.cone, tables.cone[:comp.h])
    assert blob.colour == list(comp.colour)
    assert (blob.aword * 32 + blob.ashift) == comp.d * comp.n
    if comp.Z is not None:
        assert info["has_exact_z"] == 1 and info["Z"] == pytest.approx(comp.Z, rel=1e-12)
    rng = np.random.default_rng(1)
    for trial in range(40):
        f = rng.integers(0, 2, size=comp.h)
        x = ocomp.lattice_from_free(comp, f)
        xw = ocomp.pack_words(x, comp.W)
        m, k = ocomp.path_weight(comp, x)
        assert blob.phase(xw) == k, (trial, name)
        for b in range(comp.h):
            assert blob.threshold(b, xw) == och.threshold(comp, b, xw, tables), (trial, b)


@pytest.mark.parametrize("seed", range(6))
def test_library_compile_with_toffoli_equals_oracle(pb, seed):
    """Circuits with Toffoli and Peres gates: the image's lattice of a free-bit
    assignment — constant words, the cones of the set free bits, then each
    derived AND variable in order, read off the lattice so far and its cone
    XORed in when 1 — equals the oracle's gate-by-gate lattice, and the
    image's phase polynomial gives the oracle's phase bin."""
    c = wc.random_clifford_t_toffoli(6, 8, 900 + seed, K=3, p3=0.5)
    lib_set = pb.CircuitSet(c)
    b = lib_set.export(0)
    blob = Blob(b)
    comp = ocomp.compile_circuit(oc.from_dict(c))
    assert comp.nonlinear and blob.uniform == 1
    assert (blob.h, blob.fpos) == (comp.h, list(comp.free_pos))
    ny, oy = int(b[H["NY"]]), int(b[H["OFF_Y"]])
    assert ny > 0
    st = 2 + blob.WS
    rng = np.random.default_rng(seed)
    for trial in range(60):
        f = rng.integers(0, 2, size=comp.h)
        x = np.array(blob.const, dtype=np.uint32)
        for bb in range(comp.h):
            if f[bb]:
                x ^= blob.cone[bb]
        for j in range(ny):
            p, q = int(b[oy + j * st]), int(b[oy + j * st + 1])
            if (x[p >> 5] >> (p & 31)) & (x[q >> 5] >> (q & 31)) & 1:
                x ^= b[oy + j * st + 2:oy + j * st + 2 + blob.W]
        want = ocomp.forward_lattice(comp, f)
        assert np.array_equal(x, ocomp.pack_words(want, comp.W)), trial
        assert blob.phase(x) == ocomp.path_weight(comp, want)[1], trial


@pytest.mark.parametrize("seed", [0, 2, 4, 6, 8])
def test_library_compile_with_soft_zeros_equals_oracle(pb, seed):
    """Controlled Hadamards as soft zeros (J = 2): free bits, cones,
    colouring and every threshold (the e^(-J) sampling law) equal the
    oracle's; the image's soft-zero records flag exactly the lattices the
    oracle calls violating, and on the others its phase polynomial (with
    the completed phases at the soft entries) gives the oracle's phase."""
    c = wc.random_clifford_t_ch(5, 7, 400 + seed, K=3)
    lib_set = pb.CircuitSet(c, soft_zero_J=2.0)
    b = lib_set.export(0)
    blob = Blob(b)
    comp = ocomp.compile_circuit(oc.from_dict(c), soft_J=2.0)
    assert (blob.h, blob.fpos, blob.colour) == (comp.h, list(comp.free_pos), list(comp.colour))
    assert blob.uniform == 0
    tables = och.Tables(comp)
    assert np.array_equal(blob.cone, tables.cone[:comp.h])
    ns, os_ = int(b[H["NSOFT"]]), int(b[H["OFF_SOFT"]])
    assert ns == sum(1 for g in comp.gates if g.soft.any())
    rng = np.random.default_rng(seed)
    seen = [0, 0]
    for trial in range(400):
        f = rng.integers(0, 2, size=comp.h)
        x = ocomp.lattice_from_free(comp, f)
        xw = ocomp.pack_words(x, comp.W)
        meets = False
        for g in range(ns):
            r = b[os_ + 5 * g:os_ + 5 * g + 5]
            idx = sum(int(x[int(r[j])]) << j for j in range(4))
            meets = meets or bool((int(r[4]) >> idx) & 1)
        v = ocomp.violates(comp, x)
        assert meets == v, trial
        seen[v] += 1
        if not v:
            assert blob.phase(xw) == ocomp.path_weight(comp, x)[1], trial
        for bb in range(comp.h):
            assert blob.threshold(bb, xw) == och.threshold(comp, bb, xw, tables), (trial, bb)
    assert seen[0] and seen[1]
    with pytest.raises(pb.PbitError):
        pb.CircuitSet(c)  # no soft_zero_J: refused


def test_toffoli_rejections(pb):
    """A zero-free three-qubit gate, a permutation with a phase, and a
    Toffoli beside a gate of non-constant magnitude are refused."""
    U = np.ones((8, 8)) / math.sqrt(8)
    g = {"layer": 1, "qubits": [0, 1, 2], "kind": "F3", "re": U.tolist(), "im": np.zeros((8, 8)).tolist()}
    assert _err(pb, wc.circuit("f3", 3, 1, 3, [g], 0)) == "UNSUPPORTED_GATE"
    re, im = wc.mat_perm3(wc.TOFFOLI_PERM)
    im = np.array(im)
    re = np.array(re)
    re[7, 6], im[7, 6] = 0.0, 1.0  # i instead of 1
    g = {"layer": 1, "qubits": [0, 1, 2], "kind": "T3", "re": re.tolist(), "im": im.tolist()}
    assert _err(pb, wc.circuit("t3", 3, 1, 2, [g], 0)) == "UNSUPPORTED_GATE"
    gs = [wc.gate1(1, 1, "RH", wc.mat_rh(math.pi / 8)), wc.toffoli(2, 0, 1, 2)]
    assert _err(pb, wc.circuit("nu", 3, 2, 1, gs, 0)) == "UNSUPPORTED_GATE"
    # an affine three-qubit permutation (a cyclic shift of the qubits) is fine
    # anywhere
    shift = [((i << 1) | (i >> 2)) & 7 for i in range(8)]
    re, im = wc.mat_perm3(shift)
    g = {"layer": 2, "qubits": [0, 1, 2], "kind": "ROT", "re": re, "im": im}
    s = pb.CircuitSet(wc.circuit("rot", 3, 2, 1, [wc.gate1(1, 1, "RH", wc.mat_rh(math.pi / 8)), g], 0))
    assert s.info(0)["uniform"] == 0


def _err(pb, c):
    with pytest.raises(pb.PbitError) as e:
        pb.CircuitSet(c)
    return e.value.name


def test_error_codes(pb):
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    U = np.eye(4, dtype=complex)
    U[np.ix_([2, 3], [2, 3])] = H
    ch = {"name": "ch", "n": 2, "d": 1, "K": 3, "input": 0, "matrices": {},
          "gates": [{"layer": 1, "qubits": [0, 1], "kind": "CH", "re": U.real.tolist(),
                     "im": U.imag.tolist()}]}
    assert _err(pb, ch) == "UNSUPPORTED_GATE"
    rz = wc.mat_rz(0.3)
    off = {"name": "off", "n": 1, "d": 1, "K": 3, "input": 0, "matrices": {},
           "gates": [{"layer": 1, "qubits": [0], "kind": "RZ", "re": rz[0], "im": rz[1]}]}
    assert _err(pb, off) == "PHASE_OFF_GRID"
    c = wc.hadamard_chain(2)
    c["gates"].append(dict(c["gates"][0]))
    assert _err(pb, c) == "INVALID_ARG"
    assert _err(pb, wc.hadamard_chain(1100, K=1)) == "TOO_LARGE"
    big = wc.brickwork(25, 2, 1)
    assert _err(pb, big) == "TOO_LARGE"


def test_amplitudes_match_oracle_estimator(pb):
    c = wc.random_clifford_t(4, 6, 5, K=3)
    s = pb.CircuitSet(c)
    comp = ocomp.compile_circuit(oc.from_dict(c))
    rng = np.random.default_rng(3)
    counts = rng.integers(0, 1000, size=(16, 8)).astype(np.uint64)
    amp, sre, sim = s.amplitudes(counts)
    a2, s2r, s2i = oest.amplitudes(counts, comp.Z)
    assert np.allclose(amp, a2, rtol=1e-12, atol=1e-14)
    assert np.allclose(sre, s2r, rtol=1e-9, atol=1e-15)
    assert np.allclose(sim, s2i, rtol=1e-9, atol=1e-15)
    l2, _, _ = s.amplitudes(counts, mode=pb.NORM_L2)
    assert np.allclose(l2, oest.amplitudes_l2(counts), rtol=1e-12, atol=1e-14)


def test_gibbs_argument_errors_before_device(pb):
    s = pb.CircuitSet(wc.tiny_ghz_t())
    with pytest.raises(pb.PbitError) as e:
        s.gibbs_run([1 << 20], 0, 1 << 13, d_hist=1)
    assert e.value.name == "COUNT_OVERFLOW"
    with pytest.raises(pb.PbitError) as e:
        s.gibbs_run([64], 0, 10, d_hist=None)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(pb.PbitError) as e:
        s.gibbs_run([64], 0, 10, d_hist=1, resume=True)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(pb.PbitError) as e:
        s.gibbs_run([64], 0, 10, d_hist=1, lanes_per_chain=3)
    assert e.value.name == "INVALID_ARG"


def test_launch_shape_rules(pb):
    """Static launch-shape rules: two lanes per chain for circuits whose
    conditionals are all 1/2 when the chains alone leave SIMDs with one wave;
    one lane for non-uniform circuits whatever is asked; the persistent tile
    queue for uniform circuits of a multi-circuit handle."""
    s = pb.CircuitSet(wc.workload_circuit("rct12"))
    sh = s.launch_shape([65536], 200, 10000)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["block"] == 1024 and sh["lanes_per_chain"] == 4
    assert sh["lds_hist"] == 1 and sh["lds_bytes"] <= 160 * 1024
    sh = s.launch_shape([65536], 200, 10000, specialize=1)
    assert sh["kernel"] == pb.KERNEL_TWO_LANE and sh["block"] == 512 and sh["toggle_tables"] == 1
    assert sh["lds_bytes"] <= 160 * 1024 and sh["sweeps_per_launch"] == 10200
    sh = s.launch_shape([65536], 200, 10000, lanes_per_chain=1, specialize=1)
    assert sh["kernel"] == pb.KERNEL_ONE_LANE and sh["block"] <= 256
    sh = s.launch_shape([65536], 200, 10000, lanes_per_chain=8)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lanes_per_chain"] == 8
    assert s.launch_shape([1000], 0, 50)["kernel"] == pb.KERNEL_TWO_LANE  # too small to compile for
    assert s.launch_shape([1000], 0, 50, specialize=2)["kernel"] == pb.KERNEL_SPECIALISED
    sh = s.launch_shape([1 << 20], 200, 1000, specialize=1)
    assert sh["kernel"] == pb.KERNEL_ONE_LANE
    sh = s.launch_shape([65536], 0, 100, lanes_per_chain=2, block_size=64, sweeps_per_launch=7)
    assert sh["kernel"] == pb.KERNEL_TWO_LANE and sh["block"] == 128 and sh["sweeps_per_launch"] == 7
    r = pb.CircuitSet(wc.rotated_hadamard_chain(10, math.pi / 8, K=1))
    assert r.launch_shape([1000], 0, 10, lanes_per_chain=2)["kernel"] == pb.KERNEL_ONE_LANE
    # the general kernel: two waves per 64 chains up to 32,768 chains (auto),
    # one lane per chain above or when asked
    sh = r.launch_shape([1000], 0, 10, specialize=2)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lanes_per_chain"] == 2 and sh["lds_hist"] in (0, 1)
    assert sh["block"] % 128 == 0
    sh = r.launch_shape([1000], 0, 10, specialize=2, lanes_per_chain=1)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lanes_per_chain"] == 1
    sh = r.launch_shape([65536], 0, 10, specialize=2)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lanes_per_chain"] == 1
    sh = r.launch_shape([1000], 0, 10, specialize=2, lanes_per_chain=2, block_size=64)
    assert sh["lanes_per_chain"] == 2 and sh["block"] == 128
    assert r.launch_shape([1000], 0, 10, specialize=1)["kernel"] == pb.KERNEL_ONE_LANE
    m = pb.CircuitSet([wc.tiny_ghz_t(), wc.rotated_hadamard_chain(6, math.pi / 8, K=1)])
    assert m.launch_shape([100, 100], 0, 10, idx=0)["kernel"] == pb.KERNEL_PERSISTENT
    assert m.launch_shape([100, 100], 0, 10, idx=1)["kernel"] == pb.KERNEL_ONE_LANE
    assert m.launch_shape([100, 100], 0, 10, idx=0, persistent=2)["kernel"] != pb.KERNEL_PERSISTENT
    with pytest.raises(pb.PbitError):
        m.launch_shape([100, 100], 0, 10, idx=2)
    # few free bits next to the samples of a workgroup: path counts in LDS
    sc = pb.CircuitSet(wc.random_clifford_t(16, 4, 24, K=3))
    h = sc.info(0)["h"]
    assert h <= 14
    sh = sc.launch_shape([4096], 100, 20000, specialize=2)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lds_hist"] == 2 and sh["block"] == 1024
    assert sh["lds_bytes"] >= 4 << h
    sh = sc.launch_shape([4096], 0, 2, specialize=2)  # too few samples per path
    assert sh["lds_hist"] != 2
    assert sc.launch_shape([4096], 0, 2, specialize=2, hist_mode=3)["lds_hist"] == 2
    assert sc.launch_shape([4096], 100, 20000, specialize=2, hist_mode=1)["lds_hist"] == 1
    assert sc.launch_shape([4096], 100, 20000, specialize=1, hist_mode=3)["kernel"] != pb.KERNEL_SPECIALISED
    # three-qubit products: one lane, toggle tables; the specialised kernel
    # splits sweeps over lanes as usual
    tt = pb.CircuitSet(wc.random_clifford_t_toffoli(12, 30, 13, K=3))
    sh = tt.launch_shape([65536], 0, 100, specialize=1)
    assert sh["kernel"] == pb.KERNEL_ONE_LANE and sh["toggle_tables"] == 1
    assert tt.launch_shape([65536], 0, 100, specialize=1, lanes_per_chain=2)["kernel"] == pb.KERNEL_ONE_LANE
    assert tt.launch_shape([4096], 0, 100, specialize=2, lanes_per_chain=4)["lanes_per_chain"] == 4
    # histograms beyond LDS, up to 2^20 bins, and sweeps short enough that
    # HBM atomics would bound them: bins stored as keys
    sw = pb.CircuitSet(wc.random_clifford_t(16, 17, 500, K=3))
    assert sw.info(0)["h"] <= 60
    sh = sw.launch_shape([122112], 200, 2000)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lds_hist"] == 3 and sh["block"] == 256
    assert sw.launch_shape([122112], 200, 2000, hist_mode=2)["lds_hist"] == 0
    # long sweeps (h = 102) hide the atomics
    b16 = pb.CircuitSet(wc.workload_circuit("brick16"))
    sh = b16.launch_shape([131072], 200, 2000)
    assert sh["kernel"] == pb.KERNEL_SPECIALISED and sh["lds_hist"] == 0
    assert b16.launch_shape([131072], 200, 2000, hist_mode=4)["lds_hist"] == 3
    assert s.launch_shape([65536], 200, 10000, hist_mode=4)["lds_hist"] == 3  # rct12, forced
    b20 = pb.CircuitSet(wc.workload_circuit("brick20"))
    assert b20.launch_shape([262144], 200, 2000)["lds_hist"] == 0  # long sweeps: HBM atomics
    assert b20.launch_shape([262144], 200, 2000, hist_mode=4)["lds_hist"] == 3  # 2^24 bins, 512 buckets
    big = pb.CircuitSet(wc.brickwork(22, 4, 1, K=4, kmax=3))  # 2^26 bins: beyond the key histogram
    assert big.launch_shape([1024], 0, 100, specialize=2, hist_mode=4)["lds_hist"] == 0


SPEC_CIRCUITS = [
    ("tiny", lambda: wc.tiny_ghz_t()),
    ("rct12", lambda: wc.workload_circuit("rct12")),
    ("brick20", lambda: wc.workload_circuit("brick20")),
    ("brick16", lambda: wc.workload_circuit("brick16")),
    ("hchain_odd", lambda: wc.hadamard_chain(33, K=1)),
    ("rct_w17", lambda: wc.random_clifford_t(16, 32, 1007, K=3)),
    ("rct_shallow", lambda: wc.random_clifford_t(16, 4, 24, K=3)),
    ("rctt", lambda: wc.random_clifford_t_toffoli(12, 30, 13, K=3)),
]


@pytest.mark.parametrize("name,mk", SPEC_CIRCUITS, ids=[c[0] for c in SPEC_CIRCUITS])
def test_specialised_source_compiles_for_gfx950(pb, name, mk, tmp_path):
    """The generated kernel of every uniform test circuit compiles offline for
    gfx950 without register spills: with the LDS histogram (where it fits) at
    1024 threads per workgroup (128 VGPRs) or else at 512 (256 VGPRs), the
    run-time fallback; without it at 256.  Circuits with h <= 14 also with the
    path counts in LDS, at 1024 or 512."""
    s = pb.CircuitSet(mk())
    info = s.info(0)
    modes = [(False, (256,))] + ([(True, (1024, 512))] if info["hist_bins"] * 4 <= 128 * 1024 else [])
    if info["h"] <= 14:
        modes.append((2, (1024, 512)))
    modes.append((3, (256,)))
    for lds, blocks in modes:
        for mb in blocks:
            vg, sc = _offline_compile(s, name, lds, mb, tmp_path)
            if sc == 0:
                break
        assert sc == 0, (name, lds, vg, sc)


def _offline_compile(s, name, lds, mb, tmp_path):
    src = s.specialised_source(0, lds_hist=lds, max_block=mb)
    assert "pbit_uniform_sweep" in src
    f = tmp_path / ("%s_%d_%d.hip" % (name, int(lds), mb))
    f.write_text(src)
    cmd = ["/opt/rocm/bin/hipcc", "-include", "hip/hip_runtime.h", "--offload-arch=gfx950", "-O3",
           "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
           "-c", str(f), "-o", str(f) + ".o", "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    vg = int(re.search(r"VGPRs: (\d+)", r.stderr).group(1))
    sc = int(re.search(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr).group(1))
    return vg, sc


GENERAL_CIRCUITS = [
    ("rhchain", lambda: pb_circ(wc.rotated_hadamard_chain(10, math.pi / 8, K=1)), 0.0),
    ("rbrick", lambda: pb_circ(wc.rotated_brickwork(4, 6, 5, math.pi / 8, K=3)), 0.0),
    ("rctch12", lambda: pb_circ(wc.workload_circuit("rctch12")), 4.0),
]


def pb_circ(c):
    return c


@pytest.mark.parametrize("name,mk,J", GENERAL_CIRCUITS, ids=[c[0] for c in GENERAL_CIRCUITS])
def test_general_source_compiles_for_gfx950(pb, name, mk, J, tmp_path):
    """Circuits with conditionals other than 1/2 get `pbit_general_sweep`
    (one lane per chain, colours unrolled); it compiles offline for gfx950
    without register spills, with the histogram in LDS or HBM; path counts
    and keys are refused."""
    s = pb.CircuitSet(mk(), soft_zero_J=J)
    for lds in (0, 1, 4, 5):  # one lane per chain, or two waves per 64 chains (+ 4)
        src = s.specialised_source(0, lds_hist=lds, max_block=256)
        assert "pbit_general_sweep" in src
        f = tmp_path / ("%s_%d.hip" % (name, lds))
        f.write_text(src)
        cmd = ["/opt/rocm/bin/hipcc", "-include", "hip/hip_runtime.h", "--offload-arch=gfx950", "-O3",
               "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
               "-c", str(f), "-o", str(f) + ".o", "-Rpass-analysis=kernel-resource-usage"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        assert int(re.search(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr).group(1)) == 0
    for kind in (2, 3):
        with pytest.raises(pb.PbitError) as e:
            s.specialised_source(0, lds_hist=kind, max_block=256)
        assert e.value.name == "MODE_UNAVAILABLE"


def test_shor_argument_errors_before_device(pb):
    """Column sampling: workspace size and every argument error are host
    checks (nothing is enqueued, no device needed)."""
    assert pb.shor_work_bytes(15, 7, 4, 1) == 32
    assert pb.shor_work_bytes(15, 7, 4, 250) == 8 * 256
    assert pb.shor_work_bytes(98743069, 10424, 27, 250) == 8 * 256
    for args in [(2, 1, 4, 10), (15, 1, 4, 10), (15, 15, 4, 10), (15, 7, 0, 10), (15, 7, 31, 10),
                 (15, 7, 4, 0), (15, 7, 4, (1 << 22) + 1), (1 << 31, 7, 4, 10)]:
        with pytest.raises(pb.PbitError) as e:
            pb.shor_work_bytes(*args)
        assert e.value.name == "INVALID_ARG", args
        with pytest.raises(pb.PbitError) as e:
            pb.shor_run(*args, d_P=1 << 20, d_work=1 << 20)
        assert e.value.name == "INVALID_ARG", args
    with pytest.raises(pb.PbitError) as e:
        pb.shor_run(15, 7, 4, 10, d_P=None, d_work=1 << 20)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(pb.PbitError) as e:
        pb.shor_run(15, 7, 4, 10, d_P=1 << 20, d_work=(1 << 20) + 4)
    assert e.value.name == "INVALID_ARG"
