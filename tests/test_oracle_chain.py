"""Pins of the oracle's Gibbs replay and Philox to things other than the
oracle itself: exact path laws, closed forms and an independent Philox."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import ancestral
from oracle import chain as och
from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from workloads import circuits as wc

ROCRAND_PROBE = r"""
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>
int main(int argc, char** argv) {
  // args: seed counter0 counter1 counter2 counter3
  unsigned long long seed = strtoull(argv[1], 0, 0);
  unsigned long long c0 = strtoull(argv[2], 0, 0), c1 = strtoull(argv[3], 0, 0);
  unsigned long long c2 = strtoull(argv[4], 0, 0), c3 = strtoull(argv[5], 0, 0);
  unsigned long long subseq = c2 | (c3 << 32);
  unsigned long long offset = 4ull * (c0 | (c1 << 32));
  rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
  for (int i = 0; i < 4; ++i) printf("%u\n", e.next());
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not present")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    open(src, "w").write(ROCRAND_PROBE)
    subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include", "-o", exe, src],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_independent_rocrand(rocrand_probe):
    """The oracle's Philox4x32-10 equals rocRAND's independently written
    engine (host build of its header) at counters reachable through
    (subsequence, offset)."""
    rng = np.random.default_rng(7)
    # the offset argument is 4 * (c0 + 2^32 c1) < 2^64, so c1 < 2^30 here
    cases = [(0, (0, 0, 0, 0)), (0xFFFFFFFFFFFFFFFF, (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF))]
    for _ in range(6):
        seed = int(rng.integers(0, 2 ** 63))
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, size=4)]
        ctr[1] &= 0x3FFFFFFF
        cases.append((seed, tuple(ctr)))
    cases.append((0, (5, 3, 1023, 0)))
    for seed, ctr in cases:
        out = subprocess.check_output([rocrand_probe, str(seed)] + [str(c) for c in ctr]).split()
        want = [int(v) for v in out]
        got = och.philox(ctr, (seed & 0xFFFFFFFF, seed >> 32))
        assert got == want, (seed, ctr)


def test_philox_uniform_bits():
    """Every output bit is balanced over 4096 consecutive counters."""
    ones = np.zeros(128)
    N = 4096
    for i in range(N):
        o = och.philox((i, 0, 7, 0), (0, 0))
        for w in range(4):
            for b in range(32):
                ones[32 * w + b] += (o[w] >> b) & 1
    z = (ones - N / 2) / math.sqrt(N / 4)
    assert np.max(np.abs(z)) < 5.0


def _comp(c):
    return ocomp.compile_circuit(oc.from_dict(c))


def test_tiny_chain_support_and_amplitudes():
    """Config n=3 d=5: 1024 chains x 2000 sweeps after 200 burn-in.  Every
    sample lands on a valid (alpha, phase) bin, TV_path is at the iid level
    and the amplitudes pass the 4-sigma rule against the statevector."""
    c = wc.tiny_ghz_t()
    comp = _comp(c)
    _, hist = och.gibbs(comp, 1024, 200, 2000, seed=0, threads=8)
    T = 1024 * 2000
    assert int(hist.sum()) == T
    valid = {(0, 0), (2, 0), (5, 1), (7, 5)}
    nz = {(int(a), int(k)) for a, k in zip(*np.nonzero(hist))}
    assert nz == valid
    circ = oc.from_dict(c)
    psi = exact.statevector(circ)
    pm, Z = exact.magnitude_marginal(circ)
    amp, sre, sim = oest.amplitudes(hist, comp.Z)
    ok, info = oest.z_gate(amp, sre, sim, psi)
    assert ok, info
    tv = oest.tv_path(hist, pm)
    assert tv < 5 * oest.expected_iid_tv(pm, T)
    assert oest.tv_born(amp, psi) < 0.01


def test_chain_matches_ancestral_sampler():
    """Random Clifford+T n=4: the Gibbs output marginal and the forward
    ancestral sampler's agree (two-sample chi-square)."""
    c = wc.random_clifford_t(4, 8, 3, K=3)
    comp = _comp(c)
    _, hist = och.gibbs(comp, 512, 20, 200, seed=11, threads=8)
    anc = ancestral.sample(oc.from_dict(c), int(hist.sum()), seed=5)
    a = hist.sum(axis=1).astype(float)
    b = anc.sum(axis=1).astype(float)
    keep = (a + b) > 0
    _, p, _, _ = stats.chi2_contingency(np.stack([a[keep], b[keep]]))
    assert p > 1e-4


@pytest.mark.parametrize("theta", [math.pi / 8, math.pi / 3])
def test_nonuniform_chain_law(theta):
    """Rotated Hadamard chain (Eq. (HadT), non-uniform Re E, two colours):
    the final lattices of many independent chains follow the exact p_C of
    Eq. (weightedS) enumerated over all 2^h paths."""
    c = wc.rotated_hadamard_chain(6, theta, K=1)
    comp = _comp(c)
    assert comp.ncolours == 2
    chains = 40000
    states, _ = och.gibbs(comp, chains, 30, 1, seed=3, threads=8)
    paths = ocomp.enumerate_free(comp)
    probs = np.array([m for (_, _, m, _, _) in paths])
    probs /= probs.sum()
    idx = {}
    for i, (_, x, _, _, _) in enumerate(paths):
        idx[int(ocomp.pack_words(x, comp.W)[0])] = i
    obs = np.zeros(len(paths))
    for s in states[:, 0]:
        obs[idx[int(s)]] += 1
    exp_ = probs * chains
    keep = exp_ > 5
    chi2 = float(np.sum((obs[keep] - exp_[keep]) ** 2 / exp_[keep]))
    dof = int(keep.sum()) - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4


def test_resume_is_bit_exact():
    """A run split at a sweep boundary and resumed from the saved lattice
    reproduces the uninterrupted run (the Philox counter holds the sweep)."""
    c = wc.random_clifford_t(5, 10, 9, K=3)
    comp = _comp(c)
    s_full, h_full = och.gibbs(comp, 64, 10, 50, seed=42, threads=4)
    s1, h1 = och.gibbs(comp, 64, 10, 20, seed=42, threads=4)
    s2, h2 = och.gibbs(comp, 64, 0, 30, seed=42, sweep_offset=30, init_state=s1, threads=4)
    assert np.array_equal(s_full, s2)
    assert np.array_equal(h_full, h1 + h2)


def test_chain_index_independence():
    """Chains depend only on their global index: a sub-range replayed on
    its own equals the same chains inside a larger run."""
    comp = _comp(wc.random_clifford_t(4, 6, 2, K=3))
    s_all, _ = och.gibbs(comp, 100, 5, 7, seed=9, threads=3)
    s_sub, _ = och.gibbs(comp, 30, 5, 7, seed=9, chain_begin=40, threads=1)
    assert np.array_equal(s_all[40:70], s_sub)
