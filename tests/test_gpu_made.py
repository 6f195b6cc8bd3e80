"""GPU checks of the learned proposal (bf16 MFMA MADE) and of MH with it:
forward and gradients against the FP64 oracle MADE on the same bf16-rounded
weights, Adam against the closed-form update, the fused sampler (valid
paths, q bit-equal between sampler and scorer, distribution equal to q),
and exactness of the MH target (uniform proposal always accepted, a poor
proposal still converges to the exact path marginal)."""
import math
import sys

import numpy as np
import pytest
from scipy import stats

from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from oracle import made as omade
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


def bf16_round(a):
    """Round float32 values to bf16 (round to nearest even), as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def split(flat, D, H):
    o = 0
    out = []
    for shape in [(D, H), (H,), (H, H), (H,), (H, D), (D,)]:
        n = int(np.prod(shape))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape))
        o += n
    return out


def random_params(D, H, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    M1, M2, M3 = omade.masks(D, H)
    W1 = rng.normal(0, scale / math.sqrt(D), (D, H)) * M1
    W2 = rng.normal(0, scale / math.sqrt(H), (H, H)) * M2
    V = rng.normal(0, scale / math.sqrt(H), (H, D)) * M3
    b1 = rng.normal(0, 0.1, H)
    b2 = rng.normal(0, 0.1, H)
    c = rng.normal(0, 0.3, D)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, V.ravel(), c]).astype(np.float32)


def valid_paths(c, n, seed):
    """n random valid lattices (word-major W x n) and their bit rows."""
    comp = ocomp.compile_circuit(oc.from_dict(c))
    rng = np.random.default_rng(seed)
    X = np.zeros((n, comp.L), dtype=np.float64)
    words = np.zeros((comp.W, n), dtype=np.uint32)
    for b in range(n):
        f = rng.integers(0, 2, comp.h)
        x = ocomp.lattice_from_free(comp, f)
        X[b] = x
        words[:, b] = ocomp.pack_words(x, comp.W)
    return comp, X, words


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def oracle_params(flat, D, H):
    p = split(flat, D, H)
    # the GPU computes with bf16 weights (FP32 biases)
    return [bf16_round(p[0]), p[1], bf16_round(p[2]), p[3], bf16_round(p[4]), p[5]]


SMALL = lambda: wc.random_clifford_t(4, 6, 21, K=3)


@pytest.mark.parametrize("which,H", [("small", 64), ("brick16", 1024)])
def test_logits_match_oracle(env, which, H):
    torch, pbit = env
    c = SMALL() if which == "small" else wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H)
    D = q.D
    flat = random_params(D, H, 5)
    q.set_params(flat)
    n = 300
    comp, X, words = valid_paths(c, n, 1)
    d_states = to_dev(torch, words)
    d_logits = torch.zeros(n * D, dtype=torch.float32, device="cuda")
    q.logits(d_states, n, d_logits)
    torch.cuda.synchronize()
    Lg = d_logits.cpu().numpy().reshape(n, D).astype(np.float64)
    p = oracle_params(flat, D, H)
    Lo, (_, A1, H1, A2, H2) = omade.forward(p, X)
    # bound: bf16 rounding of the hidden activations, relative 2^-8 per term
    bound = 2.0 ** -7 * (np.abs(H2) @ np.abs(p[4]) + np.abs(H1) @ np.abs(p[2]) @ np.abs(p[4]) / 4) + 1e-4
    err = np.abs(Lg - Lo)
    say("max logit err", err.max(), "max bound", bound.max())
    assert np.all(err <= bound)


U_BF16 = 2.0 ** -8     # unit roundoff of bf16 (8 significant bits, round to nearest even)
SIGMA_ERR = 2.0 ** -20  # hardware exponential + reciprocal in the FP32 sigmoid, absolute


def acc32(K):
    """Worst-case relative error of a K-term FP32 accumulation (in any order)."""
    return (K + 1) * 2.0 ** -24


def error_bounds(p, X, free):
    """First-order per-element bounds on |GPU - FP64 oracle| for the logits
    and every gradient, propagated through the GPU's arithmetic: exact input
    bits and bf16 weights (the oracle uses the same), FP32 accumulation of
    every product (any order, split-K slices included), bf16 rounding of the
    stored activations H1, H2 and of the backward signals G3, G2, G1, the
    FP32 sigmoid, and the ReLU gates taken from the GPU's own activations
    (where |A| is within its error bound of 0 the gate may differ, and the
    whole pre-gate value is allowed as error there)."""
    W1, b1, W2, b2, V, c = p
    B, D = X.shape
    H = W1.shape[1]
    u = U_BF16
    M1, M2, M3 = omade.masks(D, H)
    aW1, aW2, aV = np.abs(W1), np.abs(W2), np.abs(V)
    L, (_, A1, H1, A2, H2) = omade.forward(p, X)
    eA1 = acc32(D) * (np.abs(X) @ aW1 + np.abs(b1))
    eH1 = eA1 + u * (np.abs(H1) + eA1)
    eA2 = eH1 @ aW2 + acc32(H) * ((np.abs(H1) + eH1) @ aW2 + np.abs(b2))
    eH2 = eA2 + u * (np.abs(H2) + eA2)
    eL = eH2 @ aV + acc32(H) * ((np.abs(H2) + eH2) @ aV + np.abs(c))
    f = free[None, :].astype(np.float64)
    sig = 1.0 / (1.0 + np.exp(-L))
    G3 = (sig - X) * f / B
    dG3 = f / B * (0.25 * eL + SIGMA_ERR)
    eG3 = dG3 + u * (np.abs(G3) + dG3)

    def wgrad(A, eA, G, eG, M):  # A^T G over the batch, masked
        aA, aG = np.abs(A) + eA, np.abs(G) + eG
        return (eA.T @ np.abs(G) + aA.T @ eG + acc32(B) * (aA.T @ aG)) * M

    def colsum(G, eG):
        return eG.sum(axis=0) + acc32(B) * (np.abs(G) + eG).sum(axis=0)

    def gated(T, eT, A, eA):  # bf16((T) * (A > 0)) with the gate of the GPU's A
        amb = np.abs(A) <= eA
        on = (A > 0) & ~amb
        d = np.where(on, eT, 0.0) + np.where(amb, np.abs(T) + eT, 0.0)
        return (T * (A > 0)), d + u * (np.abs(T) * (A > 0) + d)

    e = {}
    e["V"] = wgrad(H2, eH2, G3, eG3, M3)
    e["c"] = colsum(G3, eG3)
    T2 = G3 @ V.T
    eT2 = eG3 @ aV.T + acc32(D) * ((np.abs(G3) + eG3) @ aV.T)
    G2, eG2 = gated(T2, eT2, A2, eA2)
    e["W2"] = wgrad(H1, eH1, G2, eG2, M2)
    e["b2"] = colsum(G2, eG2)
    T1 = G2 @ W2.T
    eT1 = eG2 @ aW2.T + acc32(H) * ((np.abs(G2) + eG2) @ aW2.T)
    G1, eG1 = gated(T1, eT1, A1, eA1)
    e["W1"] = wgrad(X, np.zeros_like(X), G1, eG1, M1)
    e["b1"] = colsum(G1, eG1)
    return L, eL, e


@pytest.mark.parametrize("which,H,n", [("small", 64, 512), ("brick16", 1024, 4096)])
def test_grads_match_oracle_elementwise(env, which, H, n):
    """Every gradient element (W1, b1, W2, b2, V, c) against the FP64 oracle
    on the same bf16 weights, within the per-element bound propagated
    through the GPU's arithmetic (factor 1.5 for second-order terms);
    masked weights get exactly zero.  The brick16 case is the learned
    proposal's training shape (D = 400 positions, H = 1,024, batch 4,096):
    its weight gradients split the batch over K slices and its D = 400
    columns end in partial tiles."""
    torch, pbit = env
    c = SMALL() if which == "small" else wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H)
    D = q.D
    flat = random_params(D, H, 7)
    q.set_params(flat)
    comp, X, words = valid_paths(c, n, 2)
    d_states = to_dev(torch, words)
    d_grad = torch.zeros(q.n_params, dtype=torch.float32, device="cuda")
    loss = q.grad(d_states, n, d_grad)
    g_gpu = split(d_grad.cpu().numpy(), D, H)
    free = np.zeros(D, dtype=bool)
    free[comp.free_pos] = True
    p = oracle_params(flat, D, H)
    lo, g_or = omade.loss_and_grads(p, X, free)
    say("loss gpu", loss, "oracle", lo)
    assert abs(loss - lo) <= 2e-3 * abs(lo) + 1e-4
    _, _, bounds = error_bounds(p, X, free)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "V", "c"], g_gpu, g_or):
        err = np.abs(a - b)
        bd = 1.5 * bounds[name] + 1e-30
        ratio = err / bd
        worst = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        say(name, "max err", float(err.max()), "max err/bound", float(ratio.max()), "at", worst,
            "median err/bound", float(np.median(ratio)))
        assert np.all(err <= bd), name


def test_adam_step_matches_closed_form(env):
    torch, pbit = env
    c = SMALL()
    s = pbit.CircuitSet(c)
    H = 64
    q = pbit.Proposal(s, hidden=H)
    D = q.D
    flat = random_params(D, H, 9)
    q.set_params(flat)
    n = 256
    _, X, words = valid_paths(c, n, 3)
    d_states = to_dev(torch, words)
    d_grad = torch.zeros(q.n_params, dtype=torch.float32, device="cuda")
    q.grad(d_states, n, d_grad)
    g = d_grad.cpu().numpy().astype(np.float64)
    q.train(d_states, n, n, 1, lr=1e-3)
    after = q.get_params().astype(np.float64)
    want, _, _ = omade.adam_step(flat.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1)
    assert np.allclose(after, want, rtol=1e-5, atol=1e-7)


def test_training_is_deterministic(env):
    """On the learned proposal's training shape (D = 400, H = 1,024, batch
    4,096) a proposal's gradient is the same bits on every call, and so are
    the parameters after the same Adam steps from the same start (set_params
    resets the moments): the library products keep the kernel chosen on first
    use and every reduction has a fixed order."""
    torch, pbit = env
    c = wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    H = 1024
    q = pbit.Proposal(s, hidden=H)
    flat = random_params(q.D, H, 5)
    q.set_params(flat)
    n = 4096
    _, _, words = valid_paths(c, n, 8)
    d_states = to_dev(torch, words)
    grads = []
    for _ in range(2):
        d_grad = torch.zeros(q.n_params, dtype=torch.float32, device="cuda")
        q.grad(d_states, n, d_grad)
        torch.cuda.synchronize()
        grads.append(d_grad.cpu().numpy().copy())
    assert np.array_equal(grads[0].view(np.uint32), grads[1].view(np.uint32))
    after = []
    for _ in range(2):
        q.set_params(flat)
        losses = q.train(d_states, n, n, 3)
        after.append((q.get_params().copy(), losses.copy()))
    assert np.array_equal(after[0][0].view(np.uint32), after[1][0].view(np.uint32))
    assert np.array_equal(after[0][1].view(np.uint32), after[1][1].view(np.uint32))


@pytest.mark.parametrize("which,H", [("small", 64), ("brick16", 1024)])
def test_training_batches_unpacked_in_the_finalize(env, which, H):
    """A multi-step train call unpacks each later batch inside the previous
    step's finalize; one-step calls on the same batches (each a contiguous
    copy of the word-major columns) unpack on their own.  Parameters and
    losses agree bit for bit over batches that wrap past the end of the
    samples (1,000 samples, batches of 384 at 0, 384, 0, 384)."""
    torch, pbit = env
    c = SMALL() if which == "small" else wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    W = s.info(0)["W"]
    n, B, steps = 1000, 384, 4
    _, _, words = valid_paths(c, n, 21)
    d_states = to_dev(torch, words)
    flat = random_params(pbit.Proposal(s, hidden=H).D, H, 3)
    q = pbit.Proposal(s, hidden=H)
    q.set_params(flat)
    la = q.train(d_states, n, B, steps, lr=2e-3)
    r = pbit.Proposal(s, hidden=H)
    r.set_params(flat)
    lb = []
    cur = 0
    for _ in range(steps):
        if cur + B > n:
            cur = 0
        part = d_states.view(W, n)[:, cur:cur + B].contiguous().view(-1)
        lb.append(r.train(part, B, B, 1, lr=2e-3)[0])
        cur += B
    torch.cuda.synchronize()
    assert np.array_equal(np.asarray(la, dtype=np.float32).view(np.uint32),
                          np.asarray(lb, dtype=np.float32).view(np.uint32))
    assert np.array_equal(q.get_params().view(np.uint32), r.get_params().view(np.uint32))


@pytest.mark.parametrize("which,H", [("small", 64), ("small", 512), ("brick16", 1024)])
def test_adam_step_shadows_equal_a_refresh(env, which, H):
    """The Adam step writes the bf16 shadows (row-major and transposed) of the
    weights it updates; a second proposal given the same parameters builds
    its shadows with the separate shadow pass.  Logits, samples, their log q
    and the scores must agree bit for bit (D = 28 and 400: transposed rows
    padded past D)."""
    torch, pbit = env
    c = SMALL() if which == "small" else wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H, seed=4)
    D = q.D
    n = 1024
    _, _, words = valid_paths(c, n, 12)
    d_states = to_dev(torch, words)
    q.train(d_states, n, 512, 3, lr=3e-3)
    r = pbit.Proposal(s, hidden=H, seed=9)
    r.set_params(q.get_params())
    outs = []
    for p in (q, r):
        d_logits = torch.zeros(n * D, dtype=torch.float32, device="cuda")
        p.logits(d_states, n, d_logits)
        d_out, d_lq = _sample(env, p, 2048, seed=5)
        d_sc = torch.zeros(n, dtype=torch.float64, device="cuda")
        p.score(d_states, n, d_sc)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy().view(np.uint8) for t in (d_logits, d_out, d_lq, d_sc)])
    for a, b, name in zip(outs[0], outs[1], ("logits", "samples", "log q", "scores")):
        assert np.array_equal(a, b), name


def _rr_chain(d):
    """Two qubits driven by d two-qubit gates, each the Kronecker product of
    two rotated Hadamards (Eq. (HadT)) at different angles: zero-free, with
    three magnitudes, so every gate is a 16-entry real-energy record."""
    ra, _ = wc.mat_rh(math.pi / 5)
    rb, _ = wc.mat_rh(math.pi / 7)
    A = np.array(ra).reshape(2, 2)
    Bm = np.array(rb).reshape(2, 2)
    M = np.kron(Bm, A)  # row o0 + 2 o1, column i0 + 2 i1
    re = [float(v) for v in M.ravel()]
    gates = [{"layer": l, "qubits": [0, 1], "kind": "RR", "re": re, "im": [0.0] * 16} for l in range(1, d + 1)]
    return wc.circuit("rr_chain_d%d" % d, 2, d, 1, gates)


@pytest.mark.parametrize("which", ["rh48_pi5", "rr2_d12"])
def test_mh_accept_inside_the_sweep_kernel_equals_the_separate_accept(env, which):
    """Once the handle holds the circuit-specialised sweep kernel of a
    circuit with non-constant magnitudes (one lane per chain: more than
    32,768 chains), an MH cycle's accept runs inside its first sweep launch;
    the allocation-free run takes the separate accept kernel and the generic
    sweeps.  States, phase-bin counts and accept counters agree bit for bit
    over three cycles from the all-zero paths and two resumed ones (one-qubit
    records, whose tables the kernel selects from, and two-qubit ones, which
    it reads from arrays)."""
    torch, pbit = env
    # theta = pi / 5: every gate's magnitude varies (cos against sin), and a
    # near-uniform proposal still gets accepted often
    c = wc.rotated_hadamard_chain(48, math.pi / 5, K=1) if which == "rh48_pi5" else _rr_chain(12)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    W = info["W"]
    q = pbit.Proposal(s, hidden=128, seed=2)
    q.set_params(random_params(q.D, 128, 7, scale=0.05))
    n = 40000
    # compile the specialised kernel into the handle (a run of its own)
    h0 = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    s.gibbs_run([n], 0, 2, h0, torch.zeros(n * W, dtype=torch.int32, device="cuda"), seed=1, specialize=2)
    shape = s.launch_shape([n], 0, 4, init=1)
    assert shape["kernel"] == 3 and shape["lanes_per_chain"] == 1, shape

    def fresh():
        return (torch.zeros(n * W, dtype=torch.int32, device="cuda"),
                torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda"),
                torch.zeros(n, dtype=torch.int64, device="cuda"))

    st_a, h_a, acc_a = fresh()
    st_b, h_b, acc_b = fresh()
    pbit.mh_run(s, q, n, 3, st_a, h_a, acc_a, gibbs_per_mh=4, seed=11, chain_begin=5)
    pbit.mh_run_static(s, q, n, 3, st_b, h_b, acc_b, gibbs_per_mh=4, seed=11, chain_begin=5)
    pbit.mh_run(s, q, n, 2, st_a, h_a, acc_a, gibbs_per_mh=3, seed=11, chain_begin=5, step_offset=3,
                sweep_offset=12, resume=True)
    pbit.mh_run_static(s, q, n, 2, st_b, h_b, acc_b, gibbs_per_mh=3, seed=11, chain_begin=5, step_offset=3,
                       sweep_offset=12, resume=True)
    torch.cuda.synchronize()
    say("accepted", int(acc_a.sum()), "and", int(acc_b.sum()), "of", n * 5)
    assert torch.equal(acc_a, acc_b)
    assert torch.equal(h_a, h_b)
    assert torch.equal(st_a, st_b)
    assert int(acc_a.sum()) > 0
    assert int(h_a.to(torch.int64).sum()) == n * (3 * 5 + 2 * 4)


def _sample(env, q, n, seed=3, step=0):
    torch, pbit = env
    W = q.cset.info(0)["W"]
    d_out = torch.zeros(n * W, dtype=torch.int32, device="cuda")
    d_lq = torch.zeros(n, dtype=torch.float64, device="cuda")
    q.sample(n, d_out, d_lq, seed=seed, step=step)
    torch.cuda.synchronize()
    return d_out, d_lq


@pytest.mark.parametrize("which,H,n", [("small", 64, 4096), ("small", 512, 4096), ("brick16", 1024, 1024),
                                       ("small", 1152, 4096), ("brick16", 1024, 66536)])
def test_sampler_paths_valid_and_logq_bitwise(env, which, H, n):
    """Sampled paths are valid lattices; scoring them gives the sampler's log q
    bit for bit (H = 64: the fused kernel in score mode; 512, 1024: the wide
    sampler against the batched GEMMs and the logit replay; 1,152:
    made_sample_kernel against the batched GEMM forward).  66,536 paths: a
    full forward batch of 65,536 and a ragged one of 1,000."""
    torch, pbit = env
    c = SMALL() if which == "small" else wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H)
    q.set_params(random_params(q.D, H, 11, scale=2.0))
    d_out, d_lq = _sample(env, q, n)
    comp = ocomp.compile_circuit(oc.from_dict(c))
    words = d_out.cpu().numpy().view(np.uint32).reshape(comp.W, n)
    for b in range(0, n, max(1, n // 64)):
        x = np.array([(int(words[p >> 5, b]) >> (p & 31)) & 1 for p in range(comp.L)], dtype=np.uint8)
        f = [int(x[p]) for p in comp.free_pos]
        assert np.array_equal(x, ocomp.lattice_from_free(comp, f)), b
    d_lq2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    q.score(d_out, n, d_lq2)
    torch.cuda.synchronize()
    a, b = d_lq.cpu().numpy(), d_lq2.cpu().numpy()
    say("logq sample vs score max diff", np.abs(a - b).max())
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("which,H,n", [("small", 64, 3001), ("rh48", 128, 4099), ("small", 256, 2000),
                                        ("w4", 128, 2000), ("w8", 64, 1500), ("brick16", 1024, 1000),
                                        ("small", 1152, 1000)])
def test_sample_score_equals_separate_calls(env, which, H, n):
    """The MH step's fused pass (proposals drawn and the current paths scored
    in one kernel for small networks; the two calls in sequence otherwise)
    gives the separate calls' proposals and log q bit for bit, on a ragged
    chain count with a chain offset."""
    torch, pbit = env
    if which == "small":
        c = SMALL()
    elif which == "rh48":
        c = wc.rotated_hadamard_chain(48, math.pi / 64, K=1)
    elif which == "w4":
        c = wc.random_clifford_t(8, 12, 5, K=3)  # 104 lattice bits: 4 words
    elif which == "w8":
        c = wc.random_clifford_t(12, 20, 6, K=3)  # 252 lattice bits: 8 words
    else:
        c = wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H)
    q.set_params(random_params(q.D, H, 7, scale=2.0))
    W = s.info(0)["W"]
    d_cur, _ = _sample(env, q, n, seed=5, step=9)  # valid current paths
    z = lambda k, dt: torch.zeros(k, dtype=dt, device="cuda")
    d_out, d_lq, d_lqc = z(n * W, torch.int32), z(n, torch.float64), z(n, torch.float64)
    q.sample_score(n, d_out, d_lq, d_cur, d_lqc, seed=3, step=2, chain_begin=11)
    d_out2, d_lq2, d_lqc2 = z(n * W, torch.int32), z(n, torch.float64), z(n, torch.float64)
    q.sample(n, d_out2, d_lq2, seed=3, step=2, chain_begin=11)
    q.score(d_cur, n, d_lqc2)
    torch.cuda.synchronize()
    assert torch.equal(d_out, d_out2)
    assert np.array_equal(d_lq.cpu().numpy().view(np.uint64), d_lq2.cpu().numpy().view(np.uint64))
    assert np.array_equal(d_lqc.cpu().numpy().view(np.uint64), d_lqc2.cpu().numpy().view(np.uint64))
    assert np.isfinite(d_lqc.cpu().numpy()).all() and (d_lqc.cpu().numpy() < 0).all()


@pytest.mark.parametrize("which,H,n", [("small", 64, 4096), ("rh48", 128, 4099), ("small", 512, 2000),
                                        ("brick16", 1024, 1024), ("small", 1152, 2000)])
def test_sampler_logq_matches_oracle(env, which, H, n):
    """log q of sampled paths against the FP64 oracle's log q on the same
    bf16 weights, within the bound carried from the logits (|d log
    sigma(z) / dz| <= 1) plus the FP32 sigmoid and the 2^-32 quantisation of
    the threshold; H <= 256 runs the register-resident sampler, H = 512 and
    1,024 the wide sampler, H = 1,152 made_sample_kernel."""
    torch, pbit = env
    if which == "small":
        c = SMALL()
    elif which == "rh48":
        c = wc.rotated_hadamard_chain(48, math.pi / 64, K=1)
    else:
        c = wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H)
    flat = random_params(q.D, H, 19, scale=1.5)
    q.set_params(flat)
    d_out, d_lq = _sample(env, q, n, seed=23, step=4)
    comp = ocomp.compile_circuit(oc.from_dict(c))
    words = d_out.cpu().numpy().view(np.uint32).reshape(comp.W, n)
    X = np.array([[(int(words[pp >> 5, b]) >> (pp & 31)) & 1 for pp in range(comp.L)] for b in range(n)],
                 dtype=np.float64)
    free = np.zeros(comp.L, dtype=bool)
    free[comp.free_pos] = True
    p = oracle_params(flat, q.D, H)
    lq_o = omade.log_q(p, X, free)
    L, eL, _ = error_bounds(p, X, free)
    sig = 1.0 / (1.0 + np.exp(-L))
    qi = np.where(X > 0, sig, 1.0 - sig)
    bound = ((eL + SIGMA_ERR + 2.0 ** -31 / np.maximum(qi, 2.0 ** -32)) * free[None, :]).sum(axis=1)
    lq = d_lq.cpu().numpy()
    err = np.abs(lq - lq_o)
    say("log q max err", float(err.max()), "max err/bound", float((err / bound).max()))
    assert np.all(err <= 1.5 * bound)


@pytest.mark.parametrize("H", [64, 512, 1152])
def test_sampler_distribution_is_q(env, H):
    """The sampled path law is q: chi-square over all 2^h paths of a small
    circuit (H = 64: the register-resident sampler; H = 512: the wide
    sampler; H = 1,152: made_sample_kernel)."""
    torch, pbit = env
    c = wc.rotated_hadamard_chain(7, math.pi / 5, K=1)
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=H)
    flat = random_params(q.D, H, 13, scale=3.0)
    q.set_params(flat)
    comp = ocomp.compile_circuit(oc.from_dict(c))
    assert 3 <= comp.h <= 10
    n = 1 << 16
    d_out, _ = _sample(env, q, n, seed=17)
    words = d_out.cpu().numpy().view(np.uint32).reshape(comp.W, n)
    paths = ocomp.enumerate_free(comp)
    key = {tuple(ocomp.pack_words(x, comp.W)): i for i, (_, x, _, _, _) in enumerate(paths)}
    obs = np.zeros(len(paths))
    for b in range(n):
        obs[key[tuple(words[:, b])]] += 1
    free = np.zeros(comp.L, dtype=bool)
    free[comp.free_pos] = True
    X = np.array([x for (_, x, _, _, _) in paths], dtype=np.float64)
    qv = np.exp(omade.log_q(oracle_params(flat, q.D, H), X, free))
    assert qv.sum() == pytest.approx(1.0, abs=1e-9)
    exp_ = qv * n
    keep = exp_ > 5
    chi2 = float(np.sum((obs[keep] - exp_[keep]) ** 2 / exp_[keep]))
    p = stats.chi2.sf(chi2, int(keep.sum()) - 1)
    say("sampler chi2 p", p)
    assert p > 1e-4


def _mh(env, c, q, chains, cycles, gibbs=4, seed=0):
    torch, pbit = env
    s = q.cset
    info = s.info(0)
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    acc = torch.zeros(chains, dtype=torch.int64, device="cuda")
    pbit.mh_run(s, q, chains, cycles, state, hist, acc, gibbs_per_mh=gibbs, seed=seed)
    torch.cuda.synchronize()
    h = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    return h, acc.cpu().numpy()


def test_mh_uniform_proposal_always_accepts(env):
    torch, pbit = env
    c = wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=64)
    q.set_params(np.zeros(q.n_params, dtype=np.float32))
    chains, cycles = 512, 3
    h, acc = _mh(env, c, q, chains, cycles, gibbs=2)
    assert np.all(acc == cycles)
    assert int(h.sum()) == chains * cycles * 3


@pytest.mark.parametrize("theta,hidden", [(math.pi / 8, 64), (math.pi / 8, 512)])
def test_mh_poor_proposal_keeps_exact_target(env, theta, hidden):
    """Non-uniform target (rotated Hadamards + CNOT), proposal biased to
    P(1) = 0.3: MH + Gibbs still reproduce the exact output marginal (the
    current paths scored by the fused kernel at H = 64, by the GEMMs at
    H = 512)."""
    torch, pbit = env
    c = wc.rotated_brickwork(3, 6, 2, theta, K=3)
    s = pbit.CircuitSet(c)
    q = pbit.Proposal(s, hidden=hidden)
    flat = np.zeros(q.n_params, dtype=np.float32)
    flat[-q.D:] = math.log(0.3 / 0.7)
    q.set_params(flat)
    chains, cycles = 4096, 40
    h, acc = _mh(env, c, q, chains, cycles, gibbs=1, seed=5)
    circ = oc.from_dict(c)
    pm, _ = exact.magnitude_marginal(circ)
    T = int(h.sum())
    tv = oest.tv_path(h, pm)
    say("accept rate", acc.mean() / cycles, "TV", tv, "iid", oest.expected_iid_tv(pm, T))
    assert 0 < acc.mean() < cycles
    assert tv < 6 * oest.expected_iid_tv(pm, T) + 2e-3


def test_training_lowers_nll(env):
    torch, pbit = env
    c = wc.rotated_brickwork(3, 6, 2, math.pi / 8, K=3)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    chains = 8192
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device="cuda")
    s.gibbs_run([chains], 200, 1, hist, state, seed=1)
    q = pbit.Proposal(s, hidden=128, seed=3)
    losses = q.train(state, chains, 1024, 300, lr=3e-3)
    say("loss first", losses[:3], "last", losses[-3:])
    assert losses[-20:].mean() < 0.9 * losses[:5].mean()


def test_library_log_within_one_ulp(env):
    """The FP64 logarithm summed into log q against numpy's on 2^21
    arguments: every threshold probability T / 2^32 the samplers can form
    (T drawn uniformly and log-uniformly over [1, 2^32 - 1], and its
    complement), values around 1, and positive normal doubles over the whole
    exponent range.  The library's error is at most one ulp of the result,
    numpy's below one ulp, so the two differ by at most two."""
    torch, pbit = env
    rng = np.random.default_rng(5)
    m = 1 << 19
    T1 = rng.integers(1, 2 ** 32, size=m, dtype=np.uint64)
    T2 = np.floor(np.exp2(rng.uniform(0.0, 32.0, size=m))).astype(np.uint64).clip(1, 2 ** 32 - 1)
    x = np.concatenate([T1.astype(np.float64) * 2.0 ** -32, T2.astype(np.float64) * 2.0 ** -32,
                        (2.0 ** 32 - T2.astype(np.float64)) * 2.0 ** -32,
                        1.0 + rng.uniform(-0.3, 0.3, size=m // 2),
                        np.exp2(rng.uniform(-1020.0, 1020.0, size=m // 2))])
    x = x[x > 0]
    d_x = torch.from_numpy(x).cuda()
    d_y = torch.empty_like(d_x)
    pbit.log_eval(d_x, d_y, x.size)
    torch.cuda.synchronize()
    y = d_y.cpu().numpy()
    ref = np.log(x)
    ulp = np.spacing(np.abs(ref))
    err = np.abs(y - ref) / ulp
    say("log: %d arguments, max error %.3f ulp, mean %.3f" % (x.size, float(err.max()), float(err.mean())))
    assert np.all(np.isfinite(y))
    assert float(err.max()) <= 2.0
    assert np.all(y[x == 1.0] == 0.0)


def _tau_int(torch, series):
    """tau_int of a [steps, chains] float tensor on the GPU: chain-pooled
    autocovariance by FFT, Geyer's initial positive sequence; None for a
    constant series."""
    x = series - series.mean()
    S = x.shape[0]
    f = torch.fft.rfft(x, n=2 * S, dim=0)
    acov = torch.fft.irfft((f * f.conj()).real.sum(dim=1), n=2 * S)[:S] / (
        x.shape[1] * torch.arange(S, 0, -1, device=x.device, dtype=x.dtype))
    if not float(acov[0]) > 1e-12:
        return None
    rho = (acov / acov[0]).cpu().numpy()
    tau, k = -1.0, 0
    while 2 * k + 1 < S // 2:
        g = rho[2 * k] + rho[2 * k + 1]
        if g <= 0:
            break
        tau += 2 * g
        k += 1
    return float(tau)


def _observe(env, s, state, chains):
    """[n_obs, chains]: the output alpha as +-1, cos of the phase, ln|psi|."""
    torch, pbit = env
    d_bin = torch.empty(chains, dtype=torch.int32, device="cuda")
    d_lm = torch.empty(chains, dtype=torch.float64, device="cuda")
    pbit.path_observables(s, state, chains, d_bin, d_lm)
    b = d_bin.to(torch.int64)
    K = s.info(0)["K"]
    alpha, phi = b >> K, b & ((1 << K) - 1)
    return torch.stack([(1 - 2 * alpha).double(), torch.cos(phi.double() * (2 * math.pi / (1 << K))), d_lm])


def test_trained_proposal_beats_gibbs_and_the_untrained_proposal(env):
    """What the trained network gains (the rotated-Hadamard chain of Eq.
    (HadT), d = 48, theta = pi/128, whose path law makes single-site Gibbs
    slow): trained on Gibbs samples on the GPU, MH (1 MH step : 4 Gibbs
    sweeps) decorrelates at least 10 times faster per transition than plain
    Gibbs per sweep and at least 5 times faster than the same MH with the
    untrained (zero-weight, uniform) proposal, whose proposals are almost
    never accepted; long runs of all three keep TV_path <= 0.01."""
    torch, pbit = env
    c = wc.rotated_hadamard_chain(48, math.pi / 128, K=1)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    W = info["W"]
    tc, burn, G = 4096, 8192, 4
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    pm, _ = exact.magnitude_marginal(oc.from_dict(c))

    def series(advance, state, L):
        out = []
        for t in range(L):
            advance(t)
            out.append(_observe(env, s, state, tc).float())
        a = torch.stack(out)  # [L, n_obs, chains] on the GPU
        taus = [_tau_int(torch, a[:, o, :]) for o in range(a.shape[1])]
        return max(t for t in taus if t is not None), taus

    # plain Gibbs: one sweep per transition
    st = torch.zeros(tc * W, dtype=torch.int32, device="cuda")
    s.gibbs_run([tc], burn, 0, hist, st, seed=11)
    tau_g, taus_g = series(lambda t: s.gibbs_run([tc], 0, 1, hist, st, seed=11, sweep_offset=burn + t, resume=True),
                           st, 16384)
    say("Gibbs tau_int per sweep", tau_g, taus_g)
    # training set: independent chains after the burn-in
    ntrain = 1 << 18
    train = torch.zeros(ntrain * W, dtype=torch.int32, device="cuda")
    s.gibbs_run([ntrain], burn, 1, torch.zeros_like(hist), train, seed=7)
    trained = pbit.Proposal(s, hidden=128, seed=3)
    losses = trained.train(train, ntrain, 4096, 1500)
    say("loss", float(losses[:5].mean()), "->", float(losses[-20:].mean()))
    untrained = pbit.Proposal(s, hidden=128, seed=3)
    untrained.set_params(np.zeros(untrained.n_params, dtype=np.float32))

    def mh_tau(q, seed, L):
        st = torch.zeros(tc * W, dtype=torch.int32, device="cuda")
        s.gibbs_run([tc], burn, 0, hist, st, seed=seed)
        acc = torch.zeros(tc, dtype=torch.int64, device="cuda")

        def adv(t):
            cy, r = divmod(t, 1 + G)
            if r == 0:
                pbit.mh_run(s, q, tc, 1, st, hist, acc, gibbs_per_mh=0, seed=seed, step_offset=cy, resume=True)
            else:
                s.gibbs_run([tc], 0, 1, hist, st, seed=seed, sweep_offset=(1 << 30) + cy * G + r - 1, resume=True)
        tau, taus = series(adv, st, L)
        return tau, taus, float(acc.double().mean()) / ((L + G) // (1 + G))

    tau_m, taus_m, acc_m = mh_tau(trained, 12, 2048)
    tau_u, taus_u, acc_u = mh_tau(untrained, 13, 4096)
    say("MH trained: tau_int per transition", tau_m, taus_m, "accept", acc_m)
    say("MH untrained: tau_int per transition", tau_u, taus_u, "accept", acc_u)
    assert tau_m * 10 <= tau_g
    assert tau_m * 5 <= tau_u
    assert acc_m > 0.3 and acc_m > 20 * acc_u
    # long runs of 131,072 chains: TV of the output marginal
    chains, cycles = 131072, 100
    for name, run in [("gibbs", lambda h, st: s.gibbs_run([chains], 0, cycles * (1 + G), h, st, seed=1,
                                                          sweep_offset=burn, resume=True)),
                      ("mh", lambda h, st: pbit.mh_run(s, trained, chains, cycles, st, h, None, gibbs_per_mh=G,
                                                       seed=2, resume=True))]:
        st = torch.zeros(chains * W, dtype=torch.int32, device="cuda")
        h = torch.zeros_like(hist)
        s.gibbs_run([chains], burn, 0, h, st, seed=1)
        run(h, st)
        torch.cuda.synchronize()
        hh = h.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
        tv = oest.tv_path(hh, pm)
        say(name, "TV_path", tv, "samples", int(hh.sum()))
        assert tv <= 0.01
