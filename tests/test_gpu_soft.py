"""GPU parity of soft zeros (Appendix: e^(-J) in place of the zeros of a
gate without a permutation pattern, e.g. the controlled Hadamard): chains
sample the e^(-J) law and bin only paths that avoid every soft zero.  Final
lattice words and uint32 counts equal the oracle's bit for bit in every
generic-kernel mode; amplitudes from the binned counts pass the 4-sigma
rule against the statevector; the learned proposal refuses such circuits."""
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


CASES = [
    # name, circuit, J, chains, burn_in, sweeps, chain_begin
    ("ch_4x6_J1", lambda: wc.random_clifford_t_ch(4, 6, 3, K=3), 1.0, 700, 10, 40, 0),
    ("ch_4x6_J3", lambda: wc.random_clifford_t_ch(4, 6, 3, K=3), 3.0, 500, 10, 40, 123),
    ("ch_6x10", lambda: wc.random_clifford_t_ch(6, 10, 400, K=3), 2.0, 300, 5, 30, 0),
    ("crh_chain", lambda: wc.circuit("crh", 2, 6, 2, [wc.gate1(1, 1, "H"), wc.crh(2, 1, 0, math.pi / 8, "CRH8"),
                                                      wc.gate1(3, 1, "H"), wc.crh(4, 1, 0, math.pi / 3, "CRH3"),
                                                      wc.gate1(5, 0, "H"), wc.ch(6, 0, 1)], 0),
     2.0, 600, 10, 50, 0),
    # threshold tables beyond 64 KiB: read from the image in device memory
    ("rctch12", lambda: wc.workload_circuit("rctch12"), 4.0, 300, 10, 25, 9),
]

MODES = [dict(toggle_mode=1, specialize=1), dict(toggle_mode=2), dict(toggle_mode=1, hist_mode=2, specialize=1),
         dict(toggle_mode=1, sweeps_per_launch=7, specialize=1), dict(toggle_mode=1, block_size=64, specialize=1),
         dict(specialize=2), dict(specialize=2, hist_mode=2, sweeps_per_launch=9),
         # the general kernel with one lane per chain and in its two-wave form
         dict(specialize=2, lanes_per_chain=1), dict(specialize=2, lanes_per_chain=2, block_size=128)]


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


@pytest.mark.parametrize("name,mk,J,chains,burn,sweeps,cb", CASES, ids=[c[0] for c in CASES])
def test_bit_exact_vs_oracle(env, name, mk, J, chains, burn, sweeps, cb):
    torch, pbit = env
    c = mk()
    s = pbit.CircuitSet(c, soft_zero_J=J)
    comp = ocomp.compile_circuit(oc.from_dict(c), soft_J=J)
    seed = 0xabc
    st_o, h_o = och.gibbs(comp, chains, burn, sweeps, seed=seed, chain_begin=cb, threads=os.cpu_count() or 8)
    assert 0 < int(h_o.sum()) < chains * sweeps
    for kw in MODES:
        say("case", name, kw)
        st, h = run(env, s, chains, burn, sweeps, seed, cb, **kw)
        assert np.array_equal(st, st_o), kw
        assert np.array_equal(h, h_o), kw


def test_soft_amplitudes_4_sigma(env):
    """65,536 chains on controlled-Hadamard circuits: the binned counts,
    normalised by the valid paths' mass and their own total, give
    amplitudes within the 4-sigma rule of the statevector."""
    torch, pbit = env
    for c, J in [(wc.random_clifford_t_ch(6, 10, 400, K=3), 2.0), (wc.random_clifford_t_ch(4, 6, 3, K=3), 1.0)]:
        s = pbit.CircuitSet(c, soft_zero_J=J)
        st, h = run(env, s, 65536, 20, 100, 5, 0)
        circ = oc.from_dict(c)
        psi = exact.statevector(circ)
        pm, Z = exact.magnitude_marginal(circ)
        T = int(h.sum())
        amp, sre, sim = oest.amplitudes(h, Z, T)
        ok, info = oest.z_gate(amp, sre, sim, psi)
        say("soft amplitudes", c["name"], "binned", T, info)
        assert ok, info


def test_proposal_refuses_soft_zeros(env):
    torch, pbit = env
    s = pbit.CircuitSet(wc.random_clifford_t_ch(4, 6, 3, K=3), soft_zero_J=2.0)
    with pytest.raises(pbit.PbitError) as e:
        pbit.Proposal(s, 0, hidden=64)
    assert e.value.name == "MODE_UNAVAILABLE"
