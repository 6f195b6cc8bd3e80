"""GPU checks of batched persistent launches: many circuits of uneven n, d
and chain counts in one launch per width class give exactly the states and
counts of separate runs (and of the oracle), also with sweep groups,
hipGraph replay and autotuned shapes; the full 256-circuit workload passes
the 4-sigma rule against every circuit's statevector."""
import json
import os
import sys
import tempfile

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


def small_set():
    rng = np.random.default_rng(0)
    circs, chains = [], []
    for i in range(14):
        n = int(rng.integers(2, 15))
        d = int(rng.integers(2, 34))
        c = wc.random_clifford_t(n, d, 500 + i, K=3)
        if i % 2:
            # inputs beta != 0 (Eq. (U)) on every other circuit
            c = dict(c, input=(0x5A5B >> (i % 5)) % (1 << n) or 1)
        circs.append(c)
        chains.append(int(rng.integers(1, 900)))
    # one non-uniform circuit rides along on the single-circuit path
    import math
    circs.append(wc.rotated_brickwork(3, 5, 1, math.pi / 7, K=3))
    chains.append(300)
    return circs, chains


def run_set(env, circs, chains, burn, sweeps, **kw):
    torch, pbit = env
    s = pbit.CircuitSet(circs)
    words = s.state_words(chains)
    hist = torch.zeros(s.hist_bins(), dtype=torch.int32, device="cuda")
    state = torch.zeros(max(words, 1), dtype=torch.int32, device="cuda")
    stream = kw.pop("stream", torch.cuda.current_stream())
    s.gibbs_run(chains, burn, sweeps, hist, state, seed=77, stream=stream, **kw)
    torch.cuda.synchronize()
    return s, state.cpu().numpy().view(np.uint32), hist.cpu().numpy().view(np.uint32)


def per_circuit(s, chains, st, hi):
    out = []
    so = 0
    for i, ch in enumerate(chains):
        inf = s.info(i)
        W = inf["W"]
        stt = st[so:so + ch * W].reshape(W, ch).T
        so += ch * W
        hh = hi[inf["hist_offset"]:inf["hist_offset"] + inf["hist_bins"]].astype(np.uint64)
        out.append((stt, hh.reshape(1 << inf["n"], 1 << inf["K"])))
    return out


def test_persistent_equals_separate_and_oracle(env):
    circs, chains = small_set()
    s1, st1, h1 = run_set(env, circs, chains, 5, 21, persistent=1)
    s2, st2, h2 = run_set(env, circs, chains, 5, 21, persistent=2)
    assert np.array_equal(st1, st2)
    assert np.array_equal(h1, h2)
    res = per_circuit(s1, chains, st1, h1)
    for i in [0, 3, 7, len(circs) - 1]:
        comp = ocomp.compile_circuit(oc.from_dict(circs[i]))
        so, ho = och.gibbs(comp, chains[i], 5, 21, seed=77, circuit_id=i, threads=os.cpu_count() or 8)
        assert np.array_equal(res[i][0], so), i
        assert np.array_equal(res[i][1], ho), i


def test_persistent_groups_graph_and_grid_shapes(env):
    torch, pbit = env
    circs, chains = small_set()
    _, st_ref, h_ref = run_set(env, circs, chains, 3, 17, persistent=1)
    for kw in [dict(persistent=1, sweeps_per_launch=4), dict(persistent=1, wg_per_cu=1),
               dict(persistent=1, wg_per_cu=8, hist_mode=2),
               dict(persistent=1, sweeps_per_launch=6, use_graph=True, stream=torch.cuda.Stream())]:
        say("shape", {k: v for k, v in kw.items() if k != "stream"})
        for rep in range(2 if kw.get("use_graph") else 1):
            _, st, h = run_set(env, circs, chains, 3, 17, **kw)
            assert np.array_equal(st, st_ref), (kw, rep)
            assert np.array_equal(h, h_ref), (kw, rep)


def test_specialised_members_of_a_batch(env):
    """specialize=2 takes the circuits with at least 512 chains out of the
    persistent launch into their own circuit-specialised launches (the
    non-uniform circuit, which never rides in the persistent launch, gets its
    specialised kernel too); states and counts are those of the plain
    persistent run, bit for bit, whatever histogram each specialised launch
    uses."""
    torch, pbit = env
    circs, chains = small_set()
    chains = [c * 3 for c in chains]
    _, st_ref, h_ref = run_set(env, circs, chains, 3, 17, persistent=1)
    s = pbit.CircuitSet(circs)
    kinds = [s.launch_shape(chains, 3, 17, idx=i, persistent=1, specialize=2)["kernel"] for i in range(len(circs))]
    say("kernels", kinds)
    assert pbit.KERNEL_SPECIALISED in kinds and pbit.KERNEL_PERSISTENT in kinds
    for i, k in enumerate(kinds):
        assert (k == pbit.KERNEL_SPECIALISED) == (chains[i] >= 512 or i == 14), (i, k, chains[i])
    for kw in [dict(persistent=1, specialize=2), dict(persistent=1, specialize=2, sweeps_per_launch=5),
               dict(persistent=1, specialize=2, hist_mode=3), dict(persistent=1, specialize=2, hist_mode=4)]:
        say("batch", kw)
        _, st, h = run_set(env, circs, chains, 3, 17, **kw)
        assert np.array_equal(st, st_ref), kw
        assert np.array_equal(h, h_ref), kw


def test_autotune_cache_and_identical_results(env):
    torch, pbit = env
    circs, chains = small_set()
    _, st_ref, h_ref = run_set(env, circs, chains, 3, 17, persistent=1)
    s = pbit.CircuitSet(circs)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        s.autotune(chains, 3, 17, cache_path=path, persistent=1)
        lines = open(path).read().strip().splitlines()
        assert len(lines) == 1 and json.loads(lines[0])["key"]
        s2 = pbit.CircuitSet(circs)
        s2.autotune(chains, 3, 17, cache_path=path, persistent=1)  # loads, no timing
        assert len(open(path).read().strip().splitlines()) == 1
        words = s2.state_words(chains)
        hist = torch.zeros(s2.hist_bins(), dtype=torch.int32, device="cuda")
        state = torch.zeros(words, dtype=torch.int32, device="cuda")
        s2.gibbs_run(chains, 3, 17, hist, state, seed=77, persistent=1)
        torch.cuda.synchronize()
        assert np.array_equal(state.cpu().numpy().view(np.uint32), st_ref)
        assert np.array_equal(hist.cpu().numpy().view(np.uint32), h_ref)


@pytest.mark.parametrize("specialize", [1, 0])
def test_full_batch256(env, specialize):
    """256 random Clifford+T circuits (n 4..16, d 4..32), 2^22 chains in
    total, 200 + 2000 sweeps: in one persistent launch per width class
    (specialize=1), or with every circuit of at least 1,024 chains on a
    launch of its own specialised kernel, compiled on host threads (auto: the
    run is long): pooled 4-sigma rule over every amplitude of every circuit,
    TV_path per circuit, sampled chains replayed by the oracle, and the
    cheapest members bit-exact in full."""
    torch, pbit = env
    data = json.load(open(os.path.join(wc.DATA_DIR, "batch256.json")))
    circs, chains = data["circuits"], data["chains"]
    assert sum(chains) == 1 << 22
    s = pbit.CircuitSet(circs)
    words = s.state_words(chains)
    hist = torch.zeros(s.hist_bins(), dtype=torch.int32, device="cuda")
    state = torch.zeros(words, dtype=torch.int32, device="cuda")
    kinds = [s.launch_shape(chains, 200, 2000, idx=i, persistent=1, specialize=specialize)["kernel"]
             for i in range(len(circs))]
    say("specialised launches", sum(k == pbit.KERNEL_SPECIALISED for k in kinds))
    assert (pbit.KERNEL_SPECIALISED in kinds) == (specialize == 0)
    s.gibbs_run(chains, 200, 2000, hist, state, seed=0, persistent=1, specialize=specialize)
    torch.cuda.synchronize()
    res = per_circuit(s, chains, state.cpu().numpy().view(np.uint32), hist.cpu().numpy().view(np.uint32))
    amps, sres, sims, psis = [], [], [], []
    worst_tv = 0.0
    for i, c in enumerate(circs):
        h = res[i][1]
        T = chains[i] * 2000
        assert int(h.sum()) == T
        circ = oc.from_dict(c)
        psi = exact.statevector(circ)
        pm, _ = exact.magnitude_marginal(circ)
        amp, sre, sim = s.amplitudes(h, T, idx=i)
        amps.append(amp), sres.append(sre), sims.append(sim), psis.append(psi)
        tv = oest.tv_path(h, pm)
        worst_tv = max(worst_tv, tv / max(oest.expected_iid_tv(pm, T), 1e-12))
    ok, info = oest.z_gate(np.concatenate(amps), np.concatenate(sres), np.concatenate(sims),
                           np.concatenate(psis))
    say("pooled z-gate", info, "worst TV / iid TV", worst_tv)
    assert ok, info
    assert worst_tv < 3.0
    for i in [0, 100, 255]:
        comp = ocomp.compile_circuit(oc.from_dict(circs[i]))
        for ci in [0, chains[i] - 1]:
            so, _ = och.gibbs(comp, 1, 200, 2000, seed=0, circuit_id=i, chain_begin=ci, threads=1)
            assert np.array_equal(res[i][0][ci], so[0]), (i, ci)
    # the circuits with the fewest chains x free bits, in full, as many as
    # 4e9 oracle updates allow (135 of the 256, a few seconds of host
    # threads): every count and every chain's final lattice equals the
    # oracle's
    cost = [chains[i] * s.info(i)["h"] * 2200 for i in range(len(circs))]
    cheap, tot = [], 0
    for i in sorted(range(len(circs)), key=lambda i: (cost[i], i)):
        if tot + cost[i] > 4e9 and len(cheap) >= 32:
            break
        cheap.append(i)
        tot += cost[i]
    say("bit-exact members", len(cheap), "oracle updates", tot)
    assert len(cheap) >= 32
    for i in cheap:
        comp = ocomp.compile_circuit(oc.from_dict(circs[i]))
        so, ho = och.gibbs(comp, chains[i], 200, 2000, seed=0, circuit_id=i, threads=os.cpu_count() or 8)
        assert np.array_equal(res[i][0], so), i
        assert np.array_equal(res[i][1], ho), i
