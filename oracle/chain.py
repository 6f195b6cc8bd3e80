"""ctypes driver of the plain-C chain replay (test infrastructure only).

`gibbs` replays Fig. 2 steps 1-3 chain by chain from the oracle's own
compile (oracle/compile.py); see chain.c for the exact definition of an
update, a sweep and a sample.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chain.c")
LIB = os.path.join(HERE, "_oracle_chain.so")

TAG_GIBBS = 0


def build(force=False):
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC",
                               "-pthread", "-o", LIB + ".tmp", SRC, "-lm"])
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB)
        _lib.oracle_gibbs_run.restype = C.c_int
        _lib.oracle_philox4x32_10.restype = None
    return _lib


class _Run(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("d", C.c_int), ("K", C.c_int), ("L", C.c_int),
        ("W", C.c_int), ("h", C.c_int),
        ("const_words", C.c_void_p), ("free_pos", C.c_void_p), ("cone", C.c_void_p),
        ("G", C.c_int),
        ("arity", C.c_void_p), ("in_bits", C.c_void_p), ("out_bits", C.c_void_p),
        ("mag", C.c_void_p), ("ph", C.c_void_p),
        ("factor_off", C.c_void_p), ("factor_ids", C.c_void_p), ("order", C.c_void_p),
        ("seed", C.c_uint64), ("circuit_id", C.c_uint32), ("tag", C.c_uint32),
        ("chain_begin", C.c_uint32), ("chain_count", C.c_uint32),
        ("sweep_offset", C.c_uint32), ("burn_in", C.c_uint32), ("sweeps", C.c_uint32),
        ("init_state", C.c_void_p), ("out_state", C.c_void_p), ("hist", C.c_void_p),
    ]


def philox(ctr, key):
    """Philox4x32-10 block for counter ctr (4 x u32) and key (2 x u32)."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


class Tables:
    """The oracle compile flattened into the arrays chain.c reads."""

    def __init__(self, comp):
        from .compile import pack_words
        W, h = comp.W, comp.h
        self.comp = comp
        self.const_words = pack_words(comp.const, W)
        self.free_pos = np.array(comp.free_pos or [0], dtype=np.int32)
        cone = np.zeros((max(h, 1), W), dtype=np.uint32)
        for b in range(h):
            bits = np.zeros(comp.L, dtype=np.uint8)
            for p in comp.cone[b]:
                bits[p] = 1
            cone[b] = pack_words(bits, W)
        self.cone = cone
        G = len(comp.gates)
        self.G = G
        self.arity = np.array([g.a for g in comp.gates] or [0], dtype=np.int32)
        self.in_bits = np.zeros((max(G, 1), 2), dtype=np.int32)
        self.out_bits = np.zeros((max(G, 1), 2), dtype=np.int32)
        self.mag = np.zeros((max(G, 1), 16), dtype=np.float64)
        self.ph = np.zeros((max(G, 1), 16), dtype=np.int32)
        for gi, g in enumerate(comp.gates):
            self.in_bits[gi, :g.a] = g.in_bits
            self.out_bits[gi, :g.a] = g.out_bits
            m = len(g.mag)
            # the chain samples with e^(-J) at soft zeros; a soft zero's
            # phase entry is -1, which the replay reads as "do not bin"
            self.mag[gi, :m] = g.mag_s
            self.ph[gi, :m] = np.where(g.ph >= 0, g.ph, np.where(g.soft, -1, 0))
        off = [0]
        ids = []
        for b in range(h):
            ids += comp.factors[b]
            off.append(len(ids))
        self.factor_off = np.array(off, dtype=np.int32)
        self.factor_ids = np.array(ids or [0], dtype=np.int32)
        self.order = np.array(comp.order or [0], dtype=np.int32)


def _fill(r, comp, t):
    r.n, r.d, r.K, r.L, r.W, r.h = comp.n, comp.d, comp.K, comp.L, comp.W, comp.h
    r.const_words = t.const_words.ctypes.data
    r.free_pos = t.free_pos.ctypes.data
    r.cone = t.cone.ctypes.data
    r.G = t.G
    r.arity = t.arity.ctypes.data
    r.in_bits = t.in_bits.ctypes.data
    r.out_bits = t.out_bits.ctypes.data
    r.mag = t.mag.ctypes.data
    r.ph = t.ph.ctypes.data
    r.factor_off = t.factor_off.ctypes.data
    r.factor_ids = t.factor_ids.ctypes.data
    r.order = t.order.ctypes.data


def threshold(comp, b, x_words, tables=None):
    """The uint32 threshold of free bit b at lattice x (packed words)."""
    t = tables if tables is not None else Tables(comp)
    x = np.ascontiguousarray(x_words, dtype=np.uint32)
    r = _Run()
    _fill(r, comp, t)
    L = lib()
    L.oracle_threshold.restype = C.c_uint32
    return int(L.oracle_threshold(C.byref(r), int(b), C.c_void_p(x.ctypes.data)))


def gibbs(comp, chains, burn_in, sweeps, seed=0, circuit_id=0, chain_begin=0,
          sweep_offset=0, init_state=None, threads=1, tag=TAG_GIBBS, tables=None):
    """Replay `chains` chains (global indices chain_begin...).  Returns
    (final lattice words uint32[chains, W], histogram uint64[2^n, 2^K])."""
    if comp.nonlinear:
        return gibbs_forward(comp, chains, burn_in, sweeps, seed, circuit_id, chain_begin, sweep_offset,
                             init_state, tag)
    t = tables if tables is not None else Tables(comp)
    W = comp.W
    hist = np.zeros(1 << (comp.n + comp.K), dtype=np.uint64)
    out = np.zeros((chains, W), dtype=np.uint32)
    init = None
    if init_state is not None:
        init = np.ascontiguousarray(init_state, dtype=np.uint32).reshape(chains, W)
    keep = [t.const_words, t.free_pos, t.cone, t.arity, t.in_bits, t.out_bits, t.mag,
            t.ph, t.factor_off, t.factor_ids, t.order, hist, out, init]
    for a in keep:
        if a is not None:
            assert a.flags["C_CONTIGUOUS"]
    r = _Run()
    _fill(r, comp, t)
    r.seed = int(seed)
    r.circuit_id = int(circuit_id)
    r.tag = int(tag)
    r.chain_begin = int(chain_begin)
    r.chain_count = int(chains)
    r.sweep_offset = int(sweep_offset)
    r.burn_in = int(burn_in)
    r.sweeps = int(sweeps)
    r.init_state = init.ctypes.data if init is not None else None
    r.out_state = out.ctypes.data
    r.hist = hist.ctypes.data
    rc = lib().oracle_gibbs_run(C.byref(r), int(threads))
    if rc != 0:
        raise RuntimeError("oracle_gibbs_run failed")
    return out, hist.reshape(1 << comp.n, 1 << comp.K)


def gibbs_forward(comp, chains, burn_in, sweeps, seed=0, circuit_id=0, chain_begin=0, sweep_offset=0,
                  init_state=None, tag=TAG_GIBBS):
    """The chain of Fig. 2 steps 1-3 for circuits with non-affine gates
    (whose magnitudes are all constant, so every conditional is 1/2): a
    sweep redraws each free bit b as u < 2^31 from word b mod 4 of the
    Philox block at counter (sweep, b / 4, chain, circuit_id | tag << 16),
    the lattice of the new free bits is evaluated gate by gate, and each
    post-burn-in sweep bins (alpha, phase).  Plain Python."""
    from . import compile as ocomp
    W, h, K = comp.W, comp.h, comp.K
    hist = np.zeros(1 << (comp.n + K), dtype=np.uint64)
    out = np.zeros((chains, W), dtype=np.uint32)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    for lc in range(chains):
        chain = chain_begin + lc
        words = None if init_state is None else np.asarray(init_state, dtype=np.uint32).reshape(chains, W)[lc]
        for it in range(burn_in + sweeps):
            s = sweep_offset + it
            f = []
            for blk in range((h + 3) // 4):
                f.extend(int(u < (1 << 31)) for u in philox((s, blk, chain, circuit_id | (tag << 16)), key))
            x = ocomp.forward_lattice(comp, f[:h])
            if it >= burn_in:
                _, k = ocomp.path_weight(comp, x)
                hist[(ocomp.alpha_of(comp, x) << K) | k] += 1
            words = ocomp.pack_words(x, W)
        out[lc] = words if words is not None else ocomp.pack_words(comp.const, W)
    return out, hist.reshape(1 << comp.n, 1 << K)
