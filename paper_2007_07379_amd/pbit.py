"""Python binding of libpbit (argument marshalling only).

Every function mirrors one C entry point of include/pbit.h.  Device buffers
are passed as PyTorch tensors (their data_ptr()) or raw device addresses;
streams as torch.cuda.Stream or raw hipStream_t values.  All sampling work
runs in the HIP library: if libpbit.so is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbit.so")

PBIT_OK = 0
ERRORS = {
    -1: "INVALID_ARG", -2: "UNSUPPORTED_GATE", -3: "PHASE_OFF_GRID", -4: "TOO_LARGE",
    -5: "DEVICE", -6: "COUNT_OVERFLOW", -7: "OOM", -8: "MODE_UNAVAILABLE",
}
INIT_ZERO, INIT_RESUME = 0, 1
NORM_EXACT_Z, NORM_L2 = 0, 1


class PbitError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(status, "?"), status, msg))
        self.status = status
        self.name = ERRORS.get(status, "?")


class Gate(C.Structure):
    _fields_ = [("layer", C.c_uint32), ("arity", C.c_uint32), ("q", C.c_uint32 * 3),
                ("re", C.c_double * 64), ("im", C.c_double * 64)]


class CircuitDesc(C.Structure):
    _fields_ = [("n", C.c_uint32), ("d", C.c_uint32), ("gates", C.POINTER(Gate)),
                ("n_gates", C.c_uint32), ("input_state", C.c_uint64), ("K", C.c_uint32),
                ("zero_tol", C.c_double), ("phase_tol", C.c_double), ("circuit_id", C.c_uint32),
                ("soft_zero_J", C.c_double)]


class CircuitInfo(C.Structure):
    _fields_ = [("n", C.c_uint32), ("d", C.c_uint32), ("K", C.c_uint32), ("W", C.c_uint32),
                ("L", C.c_uint32), ("h", C.c_uint32), ("n_colours", C.c_uint32),
                ("uniform", C.c_uint32), ("n_gates", C.c_uint32), ("n_quad_offsets", C.c_uint32),
                ("hist_bins", C.c_uint32), ("circuit_id", C.c_uint32), ("has_exact_z", C.c_int32),
                ("Z", C.c_double), ("hist_offset", C.c_uint64)]


class GibbsCfg(C.Structure):
    _fields_ = [("chains", C.POINTER(C.c_uint32)), ("chain_begin", C.c_uint32),
                ("burn_in", C.c_uint32), ("sweeps", C.c_uint32), ("seed", C.c_uint64),
                ("sweep_offset", C.c_uint32), ("init", C.c_uint32),
                ("sweeps_per_launch", C.c_uint32), ("block_size", C.c_uint32),
                ("use_graph", C.c_uint32), ("hist_mode", C.c_uint32), ("toggle_mode", C.c_uint32),
                ("persistent", C.c_uint32), ("wg_per_cu", C.c_uint32), ("lanes_per_chain", C.c_uint32),
                ("specialize", C.c_uint32)]


class LaunchShape(C.Structure):
    _fields_ = [("kernel", C.c_uint32), ("block", C.c_uint32), ("lds_hist", C.c_uint32),
                ("toggle_tables", C.c_uint32), ("kernel_words", C.c_uint32), ("lds_bytes", C.c_uint32),
                ("sweeps_per_launch", C.c_uint64), ("lanes_per_chain", C.c_uint32), ("pad", C.c_uint32)]


KERNEL_ONE_LANE, KERNEL_TWO_LANE, KERNEL_PERSISTENT, KERNEL_SPECIALISED = 0, 1, 2, 3

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpbit.so is missing: run python -m paper_2007_07379_amd.build")
        L = C.CDLL(LIB_PATH)
        L.pbit_last_error.restype = C.c_char_p
        L.pbit_compile_circuit.argtypes = [C.POINTER(CircuitDesc), C.c_uint32, C.POINTER(C.c_void_p)]
        L.pbit_circuit_free.argtypes = [C.c_void_p]
        L.pbit_circuit_free.restype = None
        L.pbit_circuit_count.argtypes = [C.c_void_p]
        L.pbit_circuit_count.restype = C.c_uint32
        L.pbit_circuit_info_get.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(CircuitInfo)]
        L.pbit_circuit_export.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.POINTER(C.c_size_t)]
        L.pbit_gibbs_run.argtypes = [C.c_void_p, C.POINTER(GibbsCfg), C.c_void_p, C.c_void_p, C.c_void_p]
        L.pbit_amplitudes.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint64, C.c_int,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.pbit_sync.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _check(st):
    if st != PBIT_OK:
        raise PbitError(st, lib().pbit_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _gates_of(c):
    out = []
    for g in c["gates"]:
        m = g if "re" in g else c["matrices"][g["kind"]]
        re = np.asarray(m["re"], dtype=np.float64).ravel()
        im = np.asarray(m["im"], dtype=np.float64).ravel()
        G = Gate()
        G.layer = g["layer"]
        G.arity = len(g["qubits"])
        for j, q in enumerate(g["qubits"]):
            G.q[j] = q
        for i, v in enumerate(re):
            G.re[i] = v
        for i, v in enumerate(im):
            G.im[i] = v
        out.append(G)
    return out


class CircuitSet:
    """A compiled handle (pbit_circuit) over one or more circuits."""

    def __init__(self, circuits, circuit_ids=None, zero_tol=0.0, phase_tol=0.0, soft_zero_J=0.0):
        if isinstance(circuits, dict):
            circuits = [circuits]
        self.circuits = list(circuits)
        n = len(self.circuits)
        ids = list(circuit_ids) if circuit_ids is not None else list(range(n))
        descs = (CircuitDesc * n)()
        self._keep = []
        for i, c in enumerate(self.circuits):
            gl = _gates_of(c)
            arr = (Gate * max(len(gl), 1))(*gl)
            self._keep.append(arr)
            descs[i].n = c["n"]
            descs[i].d = c["d"]
            descs[i].gates = C.cast(arr, C.POINTER(Gate))
            descs[i].n_gates = len(gl)
            descs[i].input_state = c.get("input", 0)
            descs[i].K = c["K"]
            descs[i].zero_tol = zero_tol
            descs[i].phase_tol = phase_tol
            descs[i].circuit_id = ids[i]
            descs[i].soft_zero_J = soft_zero_J
        h = C.c_void_p()
        _check(lib().pbit_compile_circuit(descs, n, C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.pbit_circuit_free(h)
            self.handle = None

    def __len__(self):
        return int(lib().pbit_circuit_count(self.handle))

    def info(self, idx=0):
        i = CircuitInfo()
        _check(lib().pbit_circuit_info_get(self.handle, idx, C.byref(i)))
        return {f: getattr(i, f) for f, _ in CircuitInfo._fields_}

    def export(self, idx=0):
        n = C.c_size_t(0)
        _check(lib().pbit_circuit_export(self.handle, idx, None, C.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint32)
        _check(lib().pbit_circuit_export(self.handle, idx, buf.ctypes.data, C.byref(n)))
        return buf

    def state_words(self, chains):
        return sum(int(ch) * self.info(i)["W"] for i, ch in enumerate(chains))

    def hist_bins(self):
        last = self.info(len(self) - 1)
        return int(last["hist_offset"] + last["hist_bins"])

    def gibbs_run(self, chains, burn_in, sweeps, d_hist, d_state=None, seed=0, chain_begin=0,
                  sweep_offset=0, resume=False, sweeps_per_launch=0, block_size=0, use_graph=False,
                  hist_mode=0, toggle_mode=0, persistent=0, wg_per_cu=0, lanes_per_chain=0,
                  specialize=0, stream=None):
        if isinstance(chains, int):
            chains = [chains]
        arr = (C.c_uint32 * len(chains))(*[int(x) for x in chains])
        cfg = GibbsCfg()
        cfg.chains = C.cast(arr, C.POINTER(C.c_uint32))
        cfg.chain_begin = chain_begin
        cfg.burn_in = burn_in
        cfg.sweeps = sweeps
        cfg.seed = seed
        cfg.sweep_offset = sweep_offset
        cfg.init = INIT_RESUME if resume else INIT_ZERO
        cfg.sweeps_per_launch = sweeps_per_launch
        cfg.block_size = block_size
        cfg.use_graph = 1 if use_graph else 0
        cfg.hist_mode = hist_mode
        cfg.toggle_mode = toggle_mode
        cfg.persistent = persistent
        cfg.wg_per_cu = wg_per_cu
        cfg.lanes_per_chain = lanes_per_chain
        cfg.specialize = specialize
        _check(lib().pbit_gibbs_run(self.handle, C.byref(cfg), _ptr(d_state), _ptr(d_hist),
                                    _stream(stream)))

    def launch_shape(self, chains, burn_in, sweeps, idx=0, **kw):
        """Launch shape gibbs_run would use for circuit idx (same keyword
        fields as gibbs_run)."""
        if isinstance(chains, int):
            chains = [chains]
        arr = (C.c_uint32 * len(chains))(*[int(x) for x in chains])
        cfg = GibbsCfg()
        cfg.chains = C.cast(arr, C.POINTER(C.c_uint32))
        cfg.burn_in = burn_in
        cfg.sweeps = sweeps
        for k, v in kw.items():
            setattr(cfg, k, int(v))
        out = LaunchShape()
        L = lib()
        L.pbit_launch_shape_get.argtypes = [C.c_void_p, C.POINTER(GibbsCfg), C.c_uint32, C.POINTER(LaunchShape)]
        _check(L.pbit_launch_shape_get(self.handle, C.byref(cfg), idx, C.byref(out)))
        return {f: getattr(out, f) for f, _ in LaunchShape._fields_}

    def specialised_source(self, idx=0, lds_hist=True, max_block=None):
        """HIP source of the circuit-specialised sweep kernel of circuit idx."""
        if max_block is None:
            max_block = 1024 if lds_hist else 256  # lds_hist: 0/False, 1/True bins, 2 path counts
        L = lib()
        L.pbit_specialised_source.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_char_p,
                                              C.c_size_t, C.POINTER(C.c_size_t)]
        n = C.c_size_t(0)
        lh = int(lds_hist)
        _check(L.pbit_specialised_source(self.handle, idx, lh, max_block, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(L.pbit_specialised_source(self.handle, idx, lh, max_block, buf, n.value, C.byref(n)))
        return buf.value.decode()

    def autotune(self, chains, burn_in, sweeps, cache_path=None, persistent=0, stream=None):
        if isinstance(chains, int):
            chains = [chains]
        arr = (C.c_uint32 * len(chains))(*[int(x) for x in chains])
        cfg = GibbsCfg()
        cfg.chains = C.cast(arr, C.POINTER(C.c_uint32))
        cfg.burn_in = burn_in
        cfg.sweeps = sweeps
        cfg.persistent = persistent
        L = lib()
        L.pbit_autotune.argtypes = [C.c_void_p, C.POINTER(GibbsCfg), C.c_char_p, C.c_void_p]
        _check(L.pbit_autotune(self.handle, C.byref(cfg),
                               cache_path.encode() if cache_path else None, _stream(stream)))

    def amplitudes(self, counts, T=None, idx=0, mode=NORM_EXACT_Z):
        counts = np.ascontiguousarray(counts, dtype=np.uint64)
        T = int(counts.sum()) if T is None else int(T)
        na = 1 << self.info(idx)["n"]
        are = np.zeros(na)
        aim = np.zeros(na)
        sre = np.zeros(na)
        sim = np.zeros(na)
        _check(lib().pbit_amplitudes(self.handle, idx, counts.ctypes.data, T, mode, are.ctypes.data,
                                     aim.ctypes.data, sre.ctypes.data, sim.ctypes.data))
        return are + 1j * aim, sre, sim


def sync(stream=None):
    _check(lib().pbit_sync(_stream(stream)))


class MadeCfg(C.Structure):
    _fields_ = [("hidden", C.c_uint32), ("seed", C.c_uint64)]


class TrainCfg(C.Structure):
    _fields_ = [("batch", C.c_uint32), ("steps", C.c_uint32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


class MhCfg(C.Structure):
    _fields_ = [("chains", C.c_uint32), ("chain_begin", C.c_uint32), ("cycles", C.c_uint32),
                ("gibbs_per_mh", C.c_uint32), ("seed", C.c_uint64), ("step_offset", C.c_uint32),
                ("sweep_offset", C.c_uint32), ("init", C.c_uint32)]


def _made_sigs(L):
    V, P = C.c_void_p, C.c_uint64
    L.pbit_proposal_create.argtypes = [V, C.c_uint32, C.POINTER(MadeCfg), C.POINTER(V)]
    L.pbit_proposal_free.argtypes = [V]
    L.pbit_proposal_free.restype = None
    L.pbit_proposal_info.argtypes = [V, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(P)]
    L.pbit_proposal_set_params.argtypes = [V, V, P]
    L.pbit_proposal_get_params.argtypes = [V, V, P]
    L.pbit_proposal_logits.argtypes = [V, V, C.c_uint32, V, V]
    L.pbit_proposal_grad.argtypes = [V, V, C.c_uint32, V, C.POINTER(C.c_float), V]
    L.pbit_proposal_train.argtypes = [V, V, P, C.POINTER(TrainCfg), V, V]
    L.pbit_proposal_sample.argtypes = [V, C.c_uint32, C.c_uint32, P, C.c_uint32, V, V, V]
    L.pbit_proposal_sample_score.argtypes = [V, C.c_uint32, C.c_uint32, P, C.c_uint32, V, V, V, V, V]
    L.pbit_proposal_score.argtypes = [V, V, C.c_uint32, V, V]
    L.pbit_mh_run.argtypes = [V, V, C.POINTER(MhCfg), V, V, V, V]
    L.pbit_mh_run_static.argtypes = [V, V, C.POINTER(MhCfg), V, V, V, V]
    L.pbit_path_observables.argtypes = [V, C.c_uint32, V, C.c_uint32, V, V, V]
    L.pbit_log_eval.argtypes = [V, V, P, V]


class Proposal:
    """A learned MADE proposal (pbit_proposal) for circuit idx of a set."""

    def __init__(self, cset, idx=0, hidden=1024, seed=0):
        L = lib()
        _made_sigs(L)
        self.cset = cset
        cfg = MadeCfg(hidden, seed)
        h = C.c_void_p()
        _check(L.pbit_proposal_create(cset.handle, idx, C.byref(cfg), C.byref(h)))
        self.handle = h
        D, H, P = C.c_uint32(), C.c_uint32(), C.c_uint64()
        _check(L.pbit_proposal_info(h, C.byref(D), C.byref(H), C.byref(P)))
        self.D, self.H, self.n_params = D.value, H.value, P.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.pbit_proposal_free(h)
            self.handle = None

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().pbit_proposal_set_params(self.handle, a.ctypes.data, a.size))

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().pbit_proposal_get_params(self.handle, a.ctypes.data, a.size))
        return a

    def logits(self, d_states, n, d_logits, stream=None):
        _check(lib().pbit_proposal_logits(self.handle, _ptr(d_states), n, _ptr(d_logits), _stream(stream)))

    def grad(self, d_states, n, d_grad, stream=None):
        loss = C.c_float()
        _check(lib().pbit_proposal_grad(self.handle, _ptr(d_states), n, _ptr(d_grad), C.byref(loss),
                                        _stream(stream)))
        return loss.value

    def train(self, d_states, n_samples, batch, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              stream=None):
        cfg = TrainCfg(batch, steps, lr, beta1, beta2, eps)
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        _check(lib().pbit_proposal_train(self.handle, _ptr(d_states), n_samples, C.byref(cfg),
                                         losses.ctypes.data, _stream(stream)))
        return losses[:steps]

    def sample(self, n, d_out, d_logq, seed=0, step=0, chain_begin=0, stream=None):
        _check(lib().pbit_proposal_sample(self.handle, n, chain_begin, seed, step, _ptr(d_out),
                                          _ptr(d_logq), _stream(stream)))

    def score(self, d_states, n, d_logq, stream=None):
        _check(lib().pbit_proposal_score(self.handle, _ptr(d_states), n, _ptr(d_logq), _stream(stream)))

    def sample_score(self, n, d_out, d_logq, d_cur, d_logq_cur, seed=0, step=0, chain_begin=0, stream=None):
        """sample() into d_out / d_logq and score() of d_cur into d_logq_cur
        in one call (one pass over the network for small networks)."""
        _check(lib().pbit_proposal_sample_score(self.handle, n, chain_begin, seed, step, _ptr(d_out),
                                                _ptr(d_logq), _ptr(d_cur), _ptr(d_logq_cur), _stream(stream)))


def mh_run(cset, proposal, chains, cycles, d_state, d_hist, d_accepts=None, gibbs_per_mh=4, seed=0,
           step_offset=0, sweep_offset=0, resume=False, chain_begin=0, stream=None):
    cfg = MhCfg(chains, chain_begin, cycles, gibbs_per_mh, seed, step_offset, sweep_offset,
                INIT_RESUME if resume else INIT_ZERO)
    L = lib()
    _made_sigs(L)
    _check(L.pbit_mh_run(cset.handle, proposal.handle, C.byref(cfg), _ptr(d_state), _ptr(d_hist),
                         _ptr(d_accepts), _stream(stream)))


def mh_run_static(cset, proposal, chains, cycles, d_state, d_hist, d_accepts=None, gibbs_per_mh=4, seed=0,
                  step_offset=0, sweep_offset=0, resume=False, chain_begin=0, stream=None):
    """pbit_mh_run_static: mh_run with the proposals in the library's static
    device array (no allocation; at most 16 MiB of chains x (4 W + 16) bytes)."""
    cfg = MhCfg(chains, chain_begin, cycles, gibbs_per_mh, seed, step_offset, sweep_offset,
                INIT_RESUME if resume else INIT_ZERO)
    L = lib()
    _made_sigs(L)
    _check(L.pbit_mh_run_static(cset.handle, proposal.handle, C.byref(cfg), _ptr(d_state), _ptr(d_hist),
                                _ptr(d_accepts), _stream(stream)))


def path_observables(cset, d_state, chains, d_bin=None, d_logmag=None, idx=0, stream=None):
    """Per-chain histogram bin (alpha 2^K + phi, uint32) and ln|psi| over the
    gates of non-constant magnitude (float64) of word-major lattices."""
    L = lib()
    _made_sigs(L)
    _check(L.pbit_path_observables(cset.handle, idx, _ptr(d_state), chains, _ptr(d_bin), _ptr(d_logmag),
                                   _stream(stream)))


def log_eval(d_x, d_y, n, stream=None):
    """The library's FP64 logarithm of log q on n device doubles."""
    L = lib()
    _made_sigs(L)
    _check(L.pbit_log_eval(_ptr(d_x), _ptr(d_y), n, _stream(stream)))


class ShorCfg(C.Structure):
    _fields_ = [("N", C.c_uint64), ("a", C.c_uint64), ("n", C.c_uint32), ("T", C.c_uint32),
                ("seed", C.c_uint64)]


def _shor_sigs(L):
    L.pbit_shor_work_bytes.argtypes = [C.POINTER(ShorCfg), C.POINTER(C.c_size_t)]
    L.pbit_shor_run.argtypes = [C.POINTER(ShorCfg), C.c_void_p, C.c_void_p, C.c_void_p]


def shor_work_bytes(N, a, n, T, seed=0):
    """Device workspace bytes of shor_run."""
    L = lib()
    _shor_sigs(L)
    cfg = ShorCfg(N, a, n, T, seed)
    b = C.c_size_t(0)
    _check(L.pbit_shor_work_bytes(C.byref(cfg), C.byref(b)))
    return b.value


def shor_run(N, a, n, T, d_P, d_work, seed=0, stream=None):
    """Column sampling for the order of a mod N (pbit_shor_run): d_P gets
    2^n floats, d_work the T samples as (f << 32 | x) sorted by f, then x."""
    L = lib()
    _shor_sigs(L)
    cfg = ShorCfg(N, a, n, T, seed)
    _check(L.pbit_shor_run(C.byref(cfg), _ptr(d_P), _ptr(d_work), _stream(stream)))
