"""GPU parity of the Gibbs path (MI355X): final lattice words of every chain
and uint32 phase-bin counts must equal the CPU oracle's bit for bit on the
same Philox streams; at full workload sizes sampled chains are replayed by
the oracle one by one and the histogram is checked against the exact
amplitudes (4-sigma rule, TV of the path marginal)."""
import math
import os
import sys

import numpy as np
import pytest

from oracle import chain as och
from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from workloads import circuits as wc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_07379_amd import pbit
    return torch, pbit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(env, c, chains, burn_in, sweeps, seed=0, chain_begin=0, **kw):
    torch, pbit = env
    s = pbit.CircuitSet(c)
    info = s.info(0)
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    s.gibbs_run([chains], burn_in, sweeps, hist, state, seed=seed, chain_begin=chain_begin,
                stream=stream, **kw)
    torch.cuda.synchronize()
    W = info["W"]
    st = state.cpu().numpy().view(np.uint32).reshape(W, chains).T.copy()
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    return st, h, s


def oracle_run(c, chains, burn_in, sweeps, seed=0, chain_begin=0):
    comp = ocomp.compile_circuit(oc.from_dict(c))
    st, h = och.gibbs(comp, chains, burn_in, sweeps, seed=seed, chain_begin=chain_begin,
                      threads=os.cpu_count() or 8)
    return st, h, comp


CASES = [
    # name, circuit, chains, burn_in, sweeps, chain_begin
    ("tiny", lambda: wc.tiny_ghz_t(), 1024, 200, 2000, 0),
    ("rct12", lambda: wc.workload_circuit("rct12"), 1000, 20, 60, 4321),
    ("brick20", lambda: wc.workload_circuit("brick20"), 700, 10, 30, 0),
    ("brick16", lambda: wc.workload_circuit("brick16"), 513, 10, 40, 77),
    ("rhchain", lambda: wc.rotated_hadamard_chain(10, math.pi / 8, K=1), 999, 20, 300, 0),
    ("rbrick", lambda: wc.rotated_brickwork(5, 8, 3, math.pi / 7, K=3), 640, 20, 100, 9),
    ("hchain_odd", lambda: wc.hadamard_chain(33, K=1), 300, 5, 50, 0),
    ("rct_w17", lambda: wc.random_clifford_t(16, 32, 1007, K=3), 257, 5, 20, 0),
    ("rasym", lambda: wc.random_asymmetric(6, 10, 3, K=3), 777, 10, 40, 5),
    # inputs beta != 0 (Eq. (U)): layer 0 clamped to beta
    ("tiny_b5", lambda: dict(wc.tiny_ghz_t(), input=5), 1024, 200, 2000, 0),
    ("rct5_b22", lambda: dict(wc.random_clifford_t(5, 7, 77, K=3), input=0b10110), 600, 10, 50, 3),
    ("rbrick_b11", lambda: dict(wc.rotated_brickwork(5, 8, 3, math.pi / 7, K=3), input=0b01011), 640, 20, 100, 9),
]


MODES = {
    "tog": dict(toggle_mode=1, lanes_per_chain=1),
    "cone": dict(toggle_mode=2),
    # two lanes per chain (circuits whose conditionals are all 1/2; the
    # others run one lane per chain whatever is asked)
    "pair": dict(lanes_per_chain=2),
    "pair_ghist": dict(lanes_per_chain=2, hist_mode=2),
    # the circuit-specialised kernel (pbit_general_sweep for the circuits
    # with other conditionals), histogram in LDS or HBM, sweep groups
    "spec": dict(specialize=2, lanes_per_chain=1),
    "spec_ghist_groups": dict(specialize=2, lanes_per_chain=1, hist_mode=2, sweeps_per_launch=7),
    # two lanes per chain: sweeps split for uniform circuits; for the others
    # pbit_general_sweep in its two-wave form (each colour's bits split, flip
    # flags crossed through LDS)
    "spec_pair": dict(specialize=2, lanes_per_chain=2),
    "spec_pair_ghist_groups": dict(specialize=2, lanes_per_chain=2, hist_mode=2, sweeps_per_launch=7),
}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name,mk,chains,burn,sweeps,cb", CASES, ids=[c[0] for c in CASES])
def test_bit_exact_vs_oracle(env, name, mk, chains, burn, sweeps, cb, mode):
    c = mk()
    say("case", name, chains, burn, sweeps, cb, "mode", mode)
    st_g, h_g, _ = run_gpu(env, c, chains, burn, sweeps, seed=0x1234abcd5678 if not name.startswith("tiny") else 0,
                           chain_begin=cb, **MODES[mode])
    st_o, h_o, comp = oracle_run(c, chains, burn, sweeps, seed=0x1234abcd5678 if not name.startswith("tiny") else 0,
                                 chain_begin=cb)
    assert np.array_equal(st_g, st_o)
    assert np.array_equal(h_g, h_o)
    assert int(h_g.sum()) == chains * sweeps


def test_launch_shapes_and_graph_are_bit_identical(env):
    """Block sizes, sweep groups (state round-trips through HBM), global
    atomics vs LDS privatisation and hipGraph replay change nothing."""
    torch, pbit = env
    c = wc.random_clifford_t(8, 20, 5, K=3)
    ref_st, ref_h, _ = run_gpu(env, c, 2000, 7, 33)
    for kw in [dict(block_size=64), dict(block_size=128), dict(sweeps_per_launch=5),
               dict(hist_mode=2), dict(hist_mode=1, block_size=192), dict(toggle_mode=2),
               dict(toggle_mode=2, hist_mode=2, block_size=64), dict(lanes_per_chain=1),
               dict(lanes_per_chain=2, block_size=64), dict(lanes_per_chain=2, block_size=256),
               dict(lanes_per_chain=2, sweeps_per_launch=5), dict(lanes_per_chain=2, hist_mode=2)]:
        say("shape", kw)
        st, h, _ = run_gpu(env, c, 2000, 7, 33, **kw)
        assert np.array_equal(st, ref_st), kw
        assert np.array_equal(h, ref_h), kw
    # graph replay on a side stream, twice, eager work in between
    s = pbit.CircuitSet(c)
    info = s.info(0)
    stream = torch.cuda.Stream()
    for rep in range(6):
        lanes = 1 + rep % 2
        hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
        state = torch.zeros(2000 * info["W"], dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        s.gibbs_run([2000], 7, 33, hist, state, sweeps_per_launch=4, use_graph=True, stream=stream,
                    lanes_per_chain=lanes)
        stream.synchronize()
        h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(ref_h.shape)
        assert np.array_equal(h, ref_h), rep
        _ = torch.ones(1000, device="cuda").sum().item()


@pytest.mark.parametrize("lanes", [1, 2])
def test_resume_matches_uninterrupted(env, lanes):
    torch, pbit = env
    c = wc.workload_circuit("rct12")
    s = pbit.CircuitSet(c)
    info = s.info(0)
    ch = 512
    full_st, full_h, _ = run_gpu(env, c, ch, 10, 40, lanes_per_chain=1)
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(ch * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([ch], 10, 15, hist, state, lanes_per_chain=lanes)
    s.gibbs_run([ch], 0, 25, hist, state, sweep_offset=25, resume=True, lanes_per_chain=3 - lanes)
    torch.cuda.synchronize()
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], ch).T
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(full_h.shape)
    assert np.array_equal(st, full_st)
    assert np.array_equal(h, full_h)


def _full_run(env, name, spl=0):
    torch, pbit = env
    w = wc.WORKLOADS[name]
    c = wc.workload_circuit(name)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    chains, burn, sweeps = w["chains"], w["burn_in"], w["sweeps"]
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([chains], burn, sweeps, hist, state, sweeps_per_launch=spl)
    torch.cuda.synchronize()
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    return c, s, st, h, chains, burn, sweeps


GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_full_rct12_bit_exact_and_amplitudes(env):
    """Full random Clifford+T workload (65,536 chains x 10,000 sweeps after
    200 burn-in) in the launch the benchmark times: every one of the 4096 x 8
    uint64 counts equals the oracle's (tests/golden/rct12_full_hist.npz,
    written by tests/golden/make_rct12_full.py from the oracle alone) and the
    final lattice words of all chains hash to the oracle's SHA-256; sampled
    chains replayed by the oracle match word for word; the histogram passes
    the 4-sigma rule against the 2^12 statevector and the path-marginal TV is
    at the iid level and <= 0.01."""
    import hashlib
    import json
    c, s, st, h, chains, burn, sweeps = _full_run(env, "rct12")
    T = chains * sweeps
    assert int(h.sum()) == T
    gold_h = np.load(os.path.join(GOLD, "rct12_full_hist.npz"))["hist"]
    gold_s = json.load(open(os.path.join(GOLD, "rct12_full_state.json")))
    assert (gold_s["chains"], gold_s["burn_in"], gold_s["sweeps"]) == (chains, burn, sweeps)
    diff = np.argwhere(h != gold_h)
    say("rct12 full: counts differing from the oracle:", len(diff), diff[:5].tolist())
    assert len(diff) == 0
    assert np.array_equal(st[0], gold_s["first_chain"]) and np.array_equal(st[-1], gold_s["last_chain"])
    assert hashlib.sha256(np.ascontiguousarray(st, dtype="<u4").tobytes()).hexdigest() == gold_s["sha256"]
    comp = ocomp.compile_circuit(oc.from_dict(c))
    rng = np.random.default_rng(0)
    picks = [0, 1, 63, 64, chains - 1] + [int(v) for v in rng.integers(0, chains, size=3)]
    for ci in picks:
        so, _ = och.gibbs(comp, 1, burn, sweeps, seed=0, chain_begin=ci, threads=1)
        assert np.array_equal(st[ci], so[0]), ci
    circ = oc.from_dict(c)
    psi = exact.statevector(circ)
    pm, _ = exact.magnitude_marginal(circ)
    amp, sre, sim = s.amplitudes(h, T)
    ok, info = oest.z_gate(amp, sre, sim, psi)
    say("z-gate", info)
    assert ok, info
    tv = oest.tv_path(h, pm)
    say("TV_path", tv, "iid", oest.expected_iid_tv(pm, T))
    assert tv <= 0.01 and tv < 3 * oest.expected_iid_tv(pm, T)


def test_full_brick20_sampled_chains_and_amplitudes(env):
    """Full brickwork workload (n=20, d=24, K=4; 262,144 chains x 20,000
    sweeps after 200 burn-in, 5.2e9 samples into 2^24 bins in HBM), run as
    two resumed launches of < 2^32 samples each, as bench.py times it: sampled
    chains replayed by the oracle match bit for bit; the pooled histogram
    passes the 4-sigma rule against the 2^20 statevector and TV_path is at
    the iid level."""
    torch, pbit = env
    w = wc.WORKLOADS["brick20"]
    c = wc.workload_circuit("brick20")
    s = pbit.CircuitSet(c)
    info = s.info(0)
    chains, burn, sweeps = w["chains"], w["burn_in"], w["sweeps"]
    per = (2 ** 32 - 1) // chains
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    total = np.zeros(info["hist_bins"], dtype=np.uint64)
    done = 0
    while done < sweeps:
        n = min(per, sweeps - done)
        hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
        say("part", done, n)
        s.gibbs_run([chains], burn if done == 0 else 0, n, hist, state, seed=0,
                    sweep_offset=0 if done == 0 else burn + done, resume=done > 0)
        torch.cuda.synchronize()
        total += hist.cpu().numpy().view(np.uint32).astype(np.uint64)
        done += n
    h = total.reshape(1 << info["n"], 1 << info["K"])
    T = chains * sweeps
    assert int(h.sum()) == T
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
    comp = ocomp.compile_circuit(oc.from_dict(c))
    for ci in [0, 1, 12345, chains - 1]:
        so, _ = och.gibbs(comp, 1, burn, sweeps, seed=0, chain_begin=ci, threads=1)
        assert np.array_equal(st[ci], so[0]), ci
    circ = oc.from_dict(c)
    psi = exact.statevector(circ)
    pm, _ = exact.magnitude_marginal(circ)
    amp, sre, sim = s.amplitudes(h, T)
    ok, zinfo = oest.z_gate(amp, sre, sim, psi)
    say("z-gate", zinfo)
    assert ok, zinfo
    tv = oest.tv_path(h, pm)
    say("TV_path", tv, "iid", oest.expected_iid_tv(pm, T))
    assert tv <= 0.01 and tv < 3 * oest.expected_iid_tv(pm, T)


def test_brick20_chain_subset_bit_exact_in_the_benchmark_launch(env):
    """The brickwork workload (n=20, d=24, K=4) on its first 4,096 chains for
    the full 200 + 20,000 sweeps, in the benchmark's launch shape (the
    circuit-specialised kernel, one lane per chain, counts by HBM atomics
    into 2^24 bins) and cut at the benchmark's launch boundary (the sweeps
    split in two halves, the second resumed from the first's state): every
    count and every final lattice word equals the oracle's."""
    torch, pbit = env
    w = wc.WORKLOADS["brick20"]
    c = wc.workload_circuit("brick20")
    s = pbit.CircuitSet(c)
    info = s.info(0)
    chains, burn, sweeps = 4096, w["burn_in"], w["sweeps"]
    kw = dict(specialize=2, lanes_per_chain=1, hist_mode=2)
    sh = s.launch_shape([w["chains"]], burn, sweeps // 2)
    sh_sub = s.launch_shape([chains], burn, sweeps // 2, **kw)
    say("benchmark shape", sh, "subset shape", sh_sub)
    for k in ("kernel", "lanes_per_chain", "lds_hist", "block"):
        assert sh[k] == sh_sub[k], k
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    half = sweeps // 2
    s.gibbs_run([chains], burn, half, hist, state, seed=0, **kw)
    s.gibbs_run([chains], 0, sweeps - half, hist, state, seed=0, sweep_offset=burn + half, resume=True, **kw)
    torch.cuda.synchronize()
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
    say("oracle: brick20 chains [0, %d) x %d sweeps" % (chains, burn + sweeps))
    st_o, h_o, _ = oracle_run(c, chains, burn, sweeps)
    assert int(h.sum()) == chains * sweeps
    assert np.array_equal(st, st_o)
    diff = np.argwhere(h != h_o)
    say("counts differing:", len(diff))
    assert len(diff) == 0


def test_full_tiny_born_tv(env):
    c, s, st, h, chains, burn, sweeps = _full_run(env, "tiny")
    _, h_o, comp = oracle_run(c, chains, burn, sweeps)
    assert np.array_equal(h, h_o)
    psi = exact.statevector(oc.from_dict(c))
    amp, sre, sim = s.amplitudes(h)
    assert oest.tv_born(amp, psi) < 0.01
    ok, info = oest.z_gate(amp, sre, sim, psi)
    assert ok, info


@pytest.mark.parametrize("theta", [math.pi / 4, math.pi / 8, math.pi / 16, 3 * math.pi / 8])
def test_rotated_hadamard_prefactor_fig5(env, theta):
    """Fig. 5: d = 10 rotated Hadamards (Eq. (HadT)), weighted sampling.
    From the GPU counts, the samples that reach output alpha carry W = Z_alpha
    times their sign, so their spread is Z_alpha sqrt(1 - mean sign^2); it
    must match the exact Eq. (U30) prefactor of the oracle within 1 % of
    Z_alpha on both outputs."""
    c = wc.rotated_hadamard_chain(10, theta, K=1)
    chains, burn, sweeps = 65536, 100, 1000
    say("fig5 theta", theta)
    st, h, s = run_gpu(env, c, chains, burn, sweeps, seed=7)
    circ = oc.from_dict(c)
    _, Z = exact.magnitude_marginal(circ)
    T = chains * sweeps
    assert int(h.sum()) == T
    for a in (0, 1):
        na = float(h[a].sum())
        Za = Z * na / T
        m = (float(h[a, 0]) - float(h[a, 1])) / na
        est = Za * math.sqrt(max(1.0 - m * m, 0.0))
        want = exact.prefactor(circ, a, True)
        say("  output", a, "measured", est, "exact", want, "Z_alpha", Za)
        assert abs(est - want) <= 0.01 * Za, (a, est, want)


@pytest.mark.parametrize("first,second", [(1, 2), (2, 1)])
def test_general_kernel_resume_across_kernels(env, first, second):
    """A rotated-brickwork run (conditionals other than 1/2) resumed from
    the generic kernel into the specialised one and back equals the
    uninterrupted oracle run."""
    torch, pbit = env
    c = wc.rotated_brickwork(5, 8, 3, math.pi / 7, K=3)
    ch, burn, sweeps = 640, 7, 60
    st_o, h_o, _ = oracle_run(c, ch, burn, sweeps, seed=31)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(ch * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([ch], burn, 25, hist, state, seed=31, specialize=first)
    s.gibbs_run([ch], 0, sweeps - 25, hist, state, seed=31, sweep_offset=burn + 25, resume=True,
                specialize=second)
    torch.cuda.synchronize()
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], ch).T
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
    assert np.array_equal(st, st_o)
    assert np.array_equal(h, h_o)


@pytest.mark.parametrize("name,mk", [
    ("rct5_b22", lambda: dict(wc.random_clifford_t(5, 7, 77, K=3), input=0b10110)),
    ("rbrick", lambda: wc.rotated_brickwork(5, 8, 3, math.pi / 7, K=3)),
    ("rhchain_b1", lambda: wc.rotated_hadamard_chain(10, math.pi / 8, K=1, input_state=1)),
    ("rct12", lambda: wc.workload_circuit("rct12")),
])
def test_path_observables_match_oracle(env, name, mk):
    """pbit_path_observables on the chains' final lattices: the bin equals
    alpha 2^K + phi of the oracle's gate-by-gate path weight (Eq. (path)),
    and ln|psi| differs from the oracle's ln of the product of gate
    magnitudes by one constant for every path."""
    torch, pbit = env
    c = mk()
    chains = 777
    st, _, s = run_gpu(env, c, chains, 10, 3, seed=5)
    info = s.info(0)
    state = torch.from_numpy(st.T.copy().view(np.int32)).cuda().reshape(-1)
    d_bin = torch.zeros(chains, dtype=torch.int32, device="cuda")
    d_lm = torch.zeros(chains, dtype=torch.float64, device="cuda")
    pbit.path_observables(s, state, chains, d_bin, d_lm)
    torch.cuda.synchronize()
    bins = d_bin.cpu().numpy().view(np.uint32)
    lm = d_lm.cpu().numpy()
    comp = ocomp.compile_circuit(oc.from_dict(c))
    L = comp.n * (comp.d + 1)
    offs = []
    for ci in range(chains):
        x = np.array([(int(st[ci, p >> 5]) >> (p & 31)) & 1 for p in range(L)], dtype=np.int64)
        m, k = ocomp.path_weight(comp, x)
        assert m > 0.0, ci
        assert bins[ci] == (ocomp.alpha_of(comp, x) << comp.K) + k, ci
        offs.append(lm[ci] - math.log(m))
    offs = np.array(offs)
    assert np.max(np.abs(offs - offs[0])) <= 1e-12 * max(1.0, float(np.max(np.abs(lm))) + abs(offs[0])) * 64
    if info["uniform"]:
        assert np.all(lm == 0.0)
