"""GPU parity of the circuit-specialised sweep kernel (generated per circuit,
compiled at run time with hipRTC): for circuits whose conditionals are all
1/2, final lattice words and uint32 counts equal the CPU oracle's bit for
bit with 1, 2, 4 and 8 lanes per chain, LDS or HBM histograms, path counts
in LDS (circuits with few free bits), bins stored as keys and counted by the
key histogram, sweep groups that do not divide the lane count, hipGraph
replay, and runs resumed across the generic and the specialised kernels."""
import os
import sys

import numpy as np
import pytest

from oracle import chain as och
from oracle import circuit as oc
from oracle import compile as ocomp
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


CASES = [
    # name, circuit, chains, burn_in, sweeps, chain_begin
    ("tiny", lambda: wc.tiny_ghz_t(), 1024, 200, 2000, 0),
    ("rct12", lambda: wc.workload_circuit("rct12"), 1000, 20, 61, 4321),
    ("brick20", lambda: wc.workload_circuit("brick20"), 700, 10, 30, 0),
    ("brick16", lambda: wc.workload_circuit("brick16"), 513, 10, 43, 77),
    ("hchain_odd", lambda: wc.hadamard_chain(33, K=1), 300, 5, 50, 0),
    ("rct_w17", lambda: wc.random_clifford_t(16, 32, 1007, K=3), 257, 5, 21, 0),
    ("rasym", lambda: wc.random_asymmetric(6, 10, 3, K=3), 777, 10, 41, 5),
    ("rct_shallow", lambda: wc.random_clifford_t(16, 4, 24, K=3), 2000, 7, 300, 11),
    # inputs beta != 0 (Eq. (U)): layer 0 clamped to beta
    ("tiny_b5", lambda: dict(wc.tiny_ghz_t(), input=5), 1024, 200, 2000, 0),
    ("rct5_b22", lambda: dict(wc.random_clifford_t(5, 7, 77, K=3), input=0b10110), 600, 10, 51, 3),
    ("brick16_b", lambda: dict(wc.workload_circuit("brick16"), input=0xA5C3), 513, 10, 43, 77),
]

_oracle_cache = {}


def oracle(name, c, chains, burn, sweeps, seed, cb):
    key = (name, chains, burn, sweeps, seed, cb)
    if key not in _oracle_cache:
        comp = ocomp.compile_circuit(oc.from_dict(c))
        _oracle_cache[key] = och.gibbs(comp, chains, burn, sweeps, seed=seed, chain_begin=cb,
                                       threads=os.cpu_count() or 8)
    return _oracle_cache[key]


def run(env, s, chains, burn, sweeps, seed, cb, stream=None, **kw):
    torch, pbit = env
    info = s.info(0)
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([chains], burn, sweeps, hist, state, seed=seed, chain_begin=cb,
                stream=stream or torch.cuda.current_stream(), **kw)
    torch.cuda.synchronize()
    W = info["W"]
    st = state.cpu().numpy().view(np.uint32).reshape(W, chains).T.copy()
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    return st, h


@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
@pytest.mark.parametrize("name,mk,chains,burn,sweeps,cb", CASES, ids=[c[0] for c in CASES])
def test_specialised_bit_exact_vs_oracle(env, name, mk, chains, burn, sweeps, cb, lanes):
    torch, pbit = env
    c = mk()
    s = pbit.CircuitSet(c)
    seed = 0 if name == "tiny" else 0x1234abcd5678
    sh = s.launch_shape([chains], burn, sweeps, specialize=2, lanes_per_chain=lanes)
    assert sh["kernel"] == pbit.KERNEL_SPECIALISED and sh["lanes_per_chain"] == lanes
    st_o, h_o = oracle(name, c, chains, burn, sweeps, seed, cb)
    info = s.info(0)
    modes = [0, 2] + ([3] if info["h"] <= 14 else []) + ([4] if info["n"] + info["K"] <= 24 else [])
    if 3 in modes:
        assert s.launch_shape([chains], burn, sweeps, specialize=2, lanes_per_chain=lanes,
                              hist_mode=3)["lds_hist"] == 2
    for hm in modes:
        say("case", name, chains, burn, sweeps, cb, "lanes", lanes, "hist_mode", hm)
        st, h = run(env, s, chains, burn, sweeps, seed, cb, specialize=2, lanes_per_chain=lanes, hist_mode=hm)
        assert np.array_equal(st, st_o), hm
        assert np.array_equal(h, h_o), hm
        assert int(h.sum()) == chains * sweeps


@pytest.mark.parametrize("name", ["rct12", "rotated"])
def test_auto_rule_reuses_a_compiled_kernel(env, name):
    """A short run under the automatic rule takes the generic kernels until
    the handle holds a specialised kernel of the kind it needs (here compiled
    by a specialize=2 run), then that kernel; the counts and states are the
    generic kernels' bit for bit either way."""
    torch, pbit = env
    import math
    c = wc.workload_circuit("rct12") if name == "rct12" else wc.rotated_brickwork(6, 8, 3, math.pi / 7, K=3)
    s = pbit.CircuitSet(c)
    chains, burn, sweeps, seed = 3000, 5, 37, 99
    assert s.launch_shape([chains], burn, sweeps)["kernel"] != pbit.KERNEL_SPECIALISED
    st_g, h_g = run(env, s, chains, burn, sweeps, seed, 0, specialize=1)
    st_a, h_a = run(env, s, chains, burn, sweeps, seed, 0)  # auto, nothing compiled yet
    assert np.array_equal(st_a, st_g) and np.array_equal(h_a, h_g)
    run(env, s, chains, burn, sweeps, seed, 0, specialize=2)  # compiles the kernel
    sh = s.launch_shape([chains], burn, sweeps)
    say("auto after compile", name, sh)
    assert sh["kernel"] == pbit.KERNEL_SPECIALISED
    st_s, h_s = run(env, s, chains, burn, sweeps, seed, 0)
    assert np.array_equal(st_s, st_g) and np.array_equal(h_s, h_g)


def test_specialised_groups_graph_and_resume(env):
    torch, pbit = env
    c = wc.workload_circuit("rct12")
    chains, burn, sweeps, seed = 777, 9, 45, 3
    st_o, h_o = oracle("rct12", c, chains, burn, sweeps, seed, 0)
    s = pbit.CircuitSet(c)
    for kw in [dict(sweeps_per_launch=7, lanes_per_chain=4), dict(sweeps_per_launch=1, lanes_per_chain=8),
               dict(sweeps_per_launch=13, lanes_per_chain=2, hist_mode=2)]:
        say("groups", kw)
        st, h = run(env, s, chains, burn, sweeps, seed, 0, specialize=2, **kw)
        assert np.array_equal(st, st_o), kw
        assert np.array_equal(h, h_o), kw
    # graph replay on a side stream, eager work between replays
    info = s.info(0)
    side = torch.cuda.Stream()
    for rep in range(3):
        say("graph replay", rep)
        hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
        state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        s.gibbs_run([chains], burn, sweeps, hist, state, seed=seed, sweeps_per_launch=10, use_graph=True,
                    specialize=2, lanes_per_chain=4, stream=side)
        side.synchronize()
        st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
        h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
        assert np.array_equal(st, st_o), rep
        assert np.array_equal(h, h_o), rep
        _ = torch.ones(1000, device="cuda").sum().item()
    # resume across kernels: generic first, specialised after, and back
    for first, second in [(1, 2), (2, 1)]:
        say("resume", first, second)
        hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
        state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
        s.gibbs_run([chains], burn, 20, hist, state, seed=seed, specialize=first, lanes_per_chain=4 if first == 2 else 0)
        s.gibbs_run([chains], 0, sweeps - 20, hist, state, seed=seed, sweep_offset=burn + 20, resume=True,
                    specialize=second, lanes_per_chain=4 if second == 2 else 0)
        torch.cuda.synchronize()
        st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
        h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
        assert np.array_equal(st, st_o)
        assert np.array_equal(h, h_o)


def test_path_counts_groups_graph_and_resume(env):
    """Path counts in LDS with sweep groups (burn-in ending inside a group),
    graph replay and a resume from the generic kernel."""
    torch, pbit = env
    c = wc.random_clifford_t(16, 4, 24, K=3)
    chains, burn, sweeps, seed = 1500, 13, 90, 99
    st_o, h_o = oracle("rct_shallow", c, chains, burn, sweeps, seed, 0)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    for kw in [dict(sweeps_per_launch=7, lanes_per_chain=4), dict(sweeps_per_launch=1, lanes_per_chain=1),
               dict(sweeps_per_launch=40, lanes_per_chain=8)]:
        say("path counts, groups", kw)
        st, h = run(env, s, chains, burn, sweeps, seed, 0, specialize=2, hist_mode=3, **kw)
        assert np.array_equal(st, st_o), kw
        assert np.array_equal(h, h_o), kw
    side = torch.cuda.Stream()
    for rep in range(3):
        say("path counts, graph replay", rep)
        hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
        state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        s.gibbs_run([chains], burn, sweeps, hist, state, seed=seed, sweeps_per_launch=25, use_graph=True,
                    specialize=2, hist_mode=3, lanes_per_chain=2, stream=side)
        side.synchronize()
        st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
        h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
        assert np.array_equal(st, st_o), rep
        assert np.array_equal(h, h_o), rep
        _ = torch.ones(1000, device="cuda").sum().item()
    say("path counts, resume from the generic kernel")
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([chains], burn, 30, hist, state, seed=seed, specialize=1)
    s.gibbs_run([chains], 0, sweeps - 30, hist, state, seed=seed, sweep_offset=burn + 30, resume=True,
                specialize=2, hist_mode=3, lanes_per_chain=4)
    torch.cuda.synchronize()
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
    assert np.array_equal(st, st_o)
    assert np.array_equal(h, h_o)


def test_keys_groups_graph_and_resume(env):
    """Bins stored as keys (n + K = 19: 16 buckets of 2^15 bins) with sweep
    groups, burn-in ending inside a group, graph replay and a resume."""
    torch, pbit = env
    c = wc.workload_circuit("brick16")
    chains, burn, sweeps, seed = 600, 11, 37, 5
    st_o, h_o = oracle("brick16", c, chains, burn, sweeps, seed, 0)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    assert s.launch_shape([chains], burn, sweeps, specialize=2, hist_mode=4)["lds_hist"] == 3
    for kw in [dict(sweeps_per_launch=7, lanes_per_chain=4), dict(sweeps_per_launch=1, lanes_per_chain=1),
               dict(lanes_per_chain=8)]:
        say("keys, groups", kw)
        st, h = run(env, s, chains, burn, sweeps, seed, 0, specialize=2, hist_mode=4, **kw)
        assert np.array_equal(st, st_o), kw
        assert np.array_equal(h, h_o), kw
    side = torch.cuda.Stream()
    for rep in range(3):
        say("keys, graph replay", rep)
        hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
        state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        s.gibbs_run([chains], burn, sweeps, hist, state, seed=seed, sweeps_per_launch=9, use_graph=True,
                    specialize=2, hist_mode=4, lanes_per_chain=2, stream=side)
        side.synchronize()
        st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
        h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
        assert np.array_equal(st, st_o), rep
        assert np.array_equal(h, h_o), rep
        _ = torch.ones(1000, device="cuda").sum().item()
    say("keys, resume from the generic kernel")
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([chains], burn, 20, hist, state, seed=seed, specialize=1)
    s.gibbs_run([chains], 0, sweeps - 20, hist, state, seed=seed, sweep_offset=burn + 20, resume=True,
                specialize=2, hist_mode=4)
    torch.cuda.synchronize()
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(h_o.shape)
    assert np.array_equal(st, st_o)
    assert np.array_equal(h, h_o)


def test_keys_split_over_launches_at_full_size(env):
    """131,072 chains x 2,100 binned sweeps store more than the 2^28 keys one
    launch holds, so the run is split; states and counts equal those of HBM
    atomics (bit-exact against the oracle in the cases above), and chains
    sampled from the run replay exactly on the oracle."""
    torch, pbit = env
    c = wc.workload_circuit("brick16")
    chains, burn, sweeps, seed = 131072, 100, 2100, 17
    s = pbit.CircuitSet(c)
    assert chains * sweeps > (1 << 28)
    res = {}
    for hm in [2, 4]:
        say("brick16 full, hist_mode", hm)
        res[hm] = run(env, s, chains, burn, sweeps, seed, 0, specialize=2, hist_mode=hm)
    assert np.array_equal(res[2][0], res[4][0])
    assert np.array_equal(res[2][1], res[4][1])
    assert int(res[4][1].sum()) == chains * sweeps
    comp = ocomp.compile_circuit(oc.from_dict(c))
    for ch in [0, 77777, chains - 1]:
        say("oracle replay of chain", ch)
        st_o, _ = och.gibbs(comp, 1, burn, sweeps, seed=seed, chain_begin=ch, threads=1)
        assert np.array_equal(res[4][0][ch], st_o[0]), ch
