"""GPU parity of circuits with three-qubit permutation gates (the Appendix's
CCNOT, and the Peres gate): each sweep rebuilds the lattice from the free
bits' toggle rows and then the derived AND variables in layer order.  Final
lattice words and uint32 counts equal the oracle's (which evaluates every
lattice gate by gate) bit for bit, in the generic one-lane kernel, the
specialised kernel with every lane count and histogram placement, and a
persistent batch; per-bit cone toggles are refused."""
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


CASES = [
    # name, circuit, chains, burn_in, sweeps, chain_begin
    ("rctt_6x10", lambda: wc.random_clifford_t_toffoli(6, 10, 11, K=3), 300, 5, 20, 0),
    ("rctt_9x16", lambda: wc.random_clifford_t_toffoli(9, 16, 12, K=3), 200, 3, 15, 1000),
    ("rctt_12x30", lambda: wc.random_clifford_t_toffoli(12, 30, 13, K=3), 130, 2, 9, 77),
    ("peres_chain", lambda: wc.circuit("pc", 3, 6, 3, [wc.gate1(1, 0, "H"), wc.gate1(1, 1, "H"),
                                                       wc.gate1(1, 2, "H"), wc.peres(2, 0, 1, 2),
                                                       wc.gate1(3, 1, "T"), wc.toffoli(4, 2, 0, 1),
                                                       wc.gate1(5, 0, "H"), wc.peres(6, 1, 2, 0)], 0),
     200, 3, 40, 0),
]

_cache = {}


def oracle(name, c, chains, burn, sweeps, seed, cb):
    key = (name, chains, burn, sweeps, seed, cb)
    if key not in _cache:
        comp = ocomp.compile_circuit(oc.from_dict(c))
        assert comp.nonlinear
        _cache[key] = och.gibbs(comp, chains, burn, sweeps, seed=seed, chain_begin=cb)
    return _cache[key]


def run(env, s, chains, burn, sweeps, seed, cb, **kw):
    torch, pbit = env
    info = s.info(0)
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([chains], burn, sweeps, hist, state, seed=seed, chain_begin=cb,
                stream=torch.cuda.current_stream(), **kw)
    torch.cuda.synchronize()
    st = state.cpu().numpy().view(np.uint32).reshape(info["W"], chains).T.copy()
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    return st, h


@pytest.mark.parametrize("name,mk,chains,burn,sweeps,cb", CASES, ids=[c[0] for c in CASES])
def test_bit_exact_vs_oracle(env, name, mk, chains, burn, sweeps, cb):
    torch, pbit = env
    c = mk()
    s = pbit.CircuitSet(c)
    seed = 0x5eed
    st_o, h_o = oracle(name, c, chains, burn, sweeps, seed, cb)
    info = s.info(0)
    modes = [dict(specialize=1, hist_mode=1), dict(specialize=1, hist_mode=2),
             dict(specialize=1, sweeps_per_launch=4)]
    for lanes in (1, 2, 4, 8):
        modes.append(dict(specialize=2, lanes_per_chain=lanes))
        modes.append(dict(specialize=2, lanes_per_chain=lanes, hist_mode=2))
    if info["h"] <= 14:
        modes.append(dict(specialize=2, hist_mode=3))
    modes.append(dict(specialize=2, hist_mode=4, sweeps_per_launch=7))
    for kw in modes:
        say("case", name, kw)
        st, h = run(env, s, chains, burn, sweeps, seed, cb, **kw)
        assert np.array_equal(st, st_o), kw
        assert np.array_equal(h, h_o), kw
    with pytest.raises(pbit.PbitError) as e:
        run(env, s, chains, burn, sweeps, seed, cb, toggle_mode=2)
    assert e.value.name == "MODE_UNAVAILABLE"


def test_persistent_batch_with_toffoli(env):
    """A persistent launch holding circuits with and without three-qubit
    products equals the oracle circuit by circuit."""
    torch, pbit = env
    circs = [wc.random_clifford_t_toffoli(5, 8, 40 + i, K=3) for i in range(3)] + \
            [wc.random_clifford_t(5, 8, 50, K=3)]
    chains = [150, 70, 260, 90]
    s = pbit.CircuitSet(circs)
    words = s.state_words(chains)
    hist = torch.zeros(s.hist_bins(), dtype=torch.int32, device="cuda")
    state = torch.zeros(words, dtype=torch.int32, device="cuda")
    s.gibbs_run(chains, 2, 11, hist, state, seed=9, persistent=1, specialize=1,
                stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    st_all = state.cpu().numpy().view(np.uint32)
    h_all = hist.cpu().numpy().view(np.uint32).astype(np.uint64)
    so = ho = 0
    for i, c in enumerate(circs):
        info = s.info(i)
        assert s.launch_shape(chains, 2, 11, idx=i, persistent=1, specialize=1)["kernel"] == pbit.KERNEL_PERSISTENT
        comp = ocomp.compile_circuit(oc.from_dict(c))
        st_o, h_o = och.gibbs(comp, chains[i], 2, 11, seed=9, circuit_id=i)
        W = info["W"]
        st = st_all[so:so + chains[i] * W].reshape(W, chains[i]).T
        h = h_all[ho:ho + info["hist_bins"]].reshape(h_o.shape)
        assert np.array_equal(st, st_o), i
        assert np.array_equal(h, h_o), i
        so += chains[i] * W
        ho += info["hist_bins"]


def test_toffoli_amplitudes_4_sigma(env):
    """A larger run of a Toffoli circuit: amplitudes from the GPU counts pass
    the 4-sigma rule against the statevector and TV_path is at the i.i.d.
    level."""
    torch, pbit = env
    c = wc.random_clifford_t_toffoli(9, 16, 12, K=3)
    s = pbit.CircuitSet(c)
    chains, sweeps = 65536, 200
    st, h = run(env, s, chains, 10, sweeps, 21, 0)
    circ = oc.from_dict(c)
    psi = exact.statevector(circ)
    pm, _ = exact.magnitude_marginal(circ)
    amp, sre, sim = s.amplitudes(h)
    ok, info = oest.z_gate(amp, sre, sim, psi)
    assert ok, info
    T = chains * sweeps
    assert oest.tv_path(h, pm) < 3 * oest.expected_iid_tv(pm, T)


def test_full_rctt12_sampled_chains_and_amplitudes(env):
    """The benchmark's launch (rctt12: 65,536 chains x (200 + 10,000)
    sweeps, automatic shape): three chains replayed by the oracle end in the
    same lattice words; amplitudes pass the 4-sigma rule against the 2^12
    statevector; TV_path at the i.i.d. level."""
    torch, pbit = env
    w = wc.WORKLOADS["rctt12"]
    c = wc.workload_circuit("rctt12")
    chains, burn, sweeps = w["chains"], w["burn_in"], w["sweeps"]
    s = pbit.CircuitSet(c)
    say("rctt12 full run", s.launch_shape([chains], burn, sweeps))
    st, h = run(env, s, chains, burn, sweeps, 0, 0)
    comp = ocomp.compile_circuit(oc.from_dict(c))
    for ch in (0, 31337, chains - 1):
        say("oracle replay of chain", ch)
        st_o, _ = och.gibbs(comp, 1, burn, sweeps, seed=0, chain_begin=ch)
        assert np.array_equal(st[ch], st_o[0]), ch
    circ = oc.from_dict(c)
    psi = exact.statevector(circ)
    pm, _ = exact.magnitude_marginal(circ)
    amp, sre, sim = s.amplitudes(h)
    ok, info = oest.z_gate(amp, sre, sim, psi)
    assert ok, info
    assert oest.tv_path(h, pm) < 3 * oest.expected_iid_tv(pm, chains * sweeps)
