"""Benchmark of the Gibbs hot path on one MI355X.

A step is one full pbit_gibbs_run of the workload (every chain: burn-in +
binned sweeps, phase polynomial, histogram), inputs resident in HBM.  Prints
one JSON line with the p-bit update rate, the roofline of the sampling
kernel (algorithmic integer-VALU ops over the kernel time measured with HIP
events on the launch stream), and the CPU oracle timed on the host cores on
a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload brick20]

With the defaults the line also carries tau_int and effective samples/s of
plain Gibbs on the workload, and a learned-proposal comparison (MADE trained
on the GPU, 1 MH : 4 Gibbs against plain Gibbs) on a rotated-Hadamard chain.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = full-rate 32-bit VALU
# lane-operations per second.  v_mad_u64_u32, v_bitop3_b32, v_alignbit_b32
# and v_bcnt_u32_b32 all issue at full rate on gfx950 (measured: 0.24
# wave64 instructions per SIMD per cycle for an independent stream of
# v_mad_u64_u32, against 0.25 for a full-rate instruction).
VALU_PEAK = 256 * 4 * 16 * 2.4e9
# Philox4x32-10 per block: 10 rounds x (2 32x32->64 multiplies + 2
# three-input XORs) = 40 slots; a block serves 4 updates.  The blocks of one
# sweep differ only in the counter word that carries the block index (the
# sweep, chain and circuit words are shared), so the first three rounds are
# partly common to all blocks of a sweep: 6 slots of them are needed once per
# sweep (5) or once per chain (1), leaving 34 slots per block.
PHILOX_SLOTS_PER_BLOCK = 34
PHILOX_SLOTS_PER_SWEEP = 5
UPDATE_FIXED_SLOTS = 1  # the threshold compare u < T

HDR = dict(N=1, D=2, K=3, W=4, H=5, LINMASK=13, NQD=14, OFF_CONE=18, OFF_LIN=19, OFF_QD=20, WS=28,
           NQG=32, OFF_QG=33, NY=36, OFF_Y=37, UNIFORM=9, OFF_THRINFO=23)


def algorithmic_ops(blob):
    """VALU lane-slots the method needs per sweep (all updates of one chain)
    and per sample, counted at the minimum a direct implementation needs:
    one Philox block per four updates (34 slots once the rounds that the
    blocks of a sweep share are counted once, 5 slots, per sweep), one
    compare per update, one XOR per nonzero
    cone word for the expected half of the updates that flip; per sample two
    slots (AND, popcount) per nonzero linear phase-plane word, two (funnel
    shift, AND/OR) per nonzero quadratic mask word plus two per word of each
    quadratic popcount, and three for the output index and the bin; per
    derived AND variable of a three-qubit gate, four plus one per nonzero
    word of its cone, per sweep; per update of a circuit with conditionals
    other than 1/2, two per scope bit of its threshold table (extract and
    place) and one for the table read."""
    g = lambda k: int(blob[HDR[k]])
    h, W, WS, K = g("H"), g("W"), g("WS"), g("K")
    cone = blob[g("OFF_CONE"):g("OFF_CONE") + h * WS].reshape(h, WS)[:, :W]
    nnz = int(np.count_nonzero(cone))
    nblk = (h + 3) // 4
    per_sweep = nblk * PHILOX_SLOTS_PER_BLOCK + PHILOX_SLOTS_PER_SWEEP + h * UPDATE_FIXED_SLOTS + 0.5 * nnz
    lin = blob[g("OFF_LIN"):g("OFF_LIN") + K * WS].reshape(K, WS)[:, :W]
    per_sample = 2 * int(np.count_nonzero(lin))
    o = g("OFF_QD")
    st = 2 + K * WS
    for q in range(g("NQD")):
        planes = blob[o + q * st + 2:o + (q + 1) * st].reshape(K, WS)[:, :W]
        used = int(np.count_nonzero(planes.any(axis=0)))
        per_sample += 2 * used + 2 * int(np.count_nonzero(planes))
    o = g("OFF_QG")
    for _ in range(g("NQG")):
        m = int(blob[o + 1])
        o += 2
        union = np.zeros(W, dtype=bool)
        for _ in range(m):
            mk = blob[o + 1:o + 1 + W]
            per_sample += 2 * int(np.count_nonzero(mk))
            union |= mk != 0
            o += 1 + WS
        per_sample += 2 * int(np.count_nonzero(union))
    per_sample += 3  # alpha funnel shift + mask, histogram index
    if not g("UNIFORM"):
        ot = g("OFF_THRINFO")
        for b in range(h):
            per_sweep += 2 * int(blob[ot + b * 14 + 1]) + 1
    # three-qubit products: per derived variable, two shifts, a three-input
    # AND with 1 and the negation to a mask (4), then one three-input
    # AND-XOR per nonzero word of its cone
    ny, oy = g("NY"), g("OFF_Y")
    for j in range(ny):
        rec = blob[oy + j * (2 + WS):oy + (j + 1) * (2 + WS)]
        per_sweep += 4 + int(np.count_nonzero(rec[2:2 + W]))
    return per_sweep, per_sample, nnz


def cpu_baseline(c, h, burn, sweeps, chains_sample, soft_J=None):
    from oracle import chain as och
    from oracle import circuit as oc
    from oracle import compile as ocomp
    comp = ocomp.compile_circuit(oc.from_dict(c), soft_J=soft_J)
    threads = os.cpu_count() or 1
    if comp.nonlinear:
        # the gate-by-gate replay is plain Python on one core: a few chains
        threads = 1
        chains_sample = 2
        sweeps = min(sweeps, 2000)
    t0 = time.perf_counter()
    och.gibbs(comp, chains_sample, burn, sweeps, seed=0, threads=threads)
    dt = time.perf_counter() - t0
    ups = chains_sample * (burn + sweeps) * h / dt
    return {"value": ups, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d chains x (%d + %d) sweeps of the same circuit (first chains of the "
                      "workload), %.1f s" % (chains_sample, burn, sweeps, dt)}


def path_observables(torch, pbit, s, state, info, chains, masks):
    """Observables of every chain's current path for tau_int ([n_obs,
    chains] float64): +-1 parity characters of the output alpha for each
    mask, cos and sin of the phase 2 pi phi / 2^K, and ln|psi| (gates of
    non-constant magnitude), from the library's pbit_path_observables."""
    d_bin = torch.empty(chains, dtype=torch.int32, device=state.device)
    d_lm = torch.empty(chains, dtype=torch.float64, device=state.device)
    pbit.path_observables(s, state, chains, d_bin, d_lm, stream=torch.cuda.current_stream())
    K, n = info["K"], info["n"]
    b = d_bin.to(torch.int64) & 0xFFFFFFFF
    alpha, phi = b >> K, b & ((1 << K) - 1)
    out = []
    for m in masks:
        v = alpha & m
        par = torch.zeros_like(v)
        for q in range(n):
            par ^= (v >> q) & 1
        out.append((1 - 2 * par).to(torch.float64))
    ang = phi.to(torch.float64) * (2.0 * 3.141592653589793 / (1 << K))
    out += [torch.cos(ang), torch.sin(ang), d_lm]
    return torch.stack(out)


def observable_names(masks):
    return ["parity(alpha & %#x)" % m for m in masks] + ["cos phi", "sin phi", "ln|psi|"]


def magnitude_marginal(c):
    """Exact output law of the sampled path measure (p_C proportional to
    |psi_C|): the circuit run on beta with every gate matrix replaced by its
    entrywise modulus, normalised.  Used only to report TV_path."""
    n = c["n"]
    v = np.zeros(1 << n)
    v[c.get("input", 0)] = 1.0
    v = v.reshape([2] * n)
    for g in sorted(c["gates"], key=lambda g: (g["layer"], min(g["qubits"]))):
        m = g if "re" in g else c["matrices"][g["kind"]]
        U = np.abs(np.array(m["re"], dtype=np.float64) + 1j * np.array(m["im"], dtype=np.float64))
        qs = list(g["qubits"])
        a = len(qs)
        Ut = U.reshape([2] * (2 * a))
        axes = [n - 1 - q for q in reversed(qs)]
        v = np.moveaxis(np.tensordot(Ut, v, axes=(list(range(a, 2 * a)), axes)), list(range(a)), axes)
    v = v.reshape(-1)
    return v / v.sum()


def tv_path(hist, pm):
    emp = hist.sum(axis=1).astype(np.float64)
    return 0.5 * float(np.abs(emp / emp.sum() - pm).sum())


def _rh(theta):
    return lambda wc: wc.rotated_hadamard_chain(48, theta, K=1)


PI = 3.141592653589793
MH_WORKLOADS = {
    # chains: population timed for s/transition and binned for TV; tau_chains:
    # chains whose output series gives tau_int; burn_in in sweeps
    "brick16": dict(circuit=lambda wc: wc.workload_circuit("brick16"), chains=131072, burn_in=200, hidden=1024,
                    train=1 << 20, train_steps=2560, batch=4096, long_cycles=400, tau_chains=4096),
    "rhchain48": dict(circuit=_rh(PI / 64), chains=131072, burn_in=2000, hidden=128, train=1 << 18,
                      train_steps=1500, batch=4096, long_cycles=200, tau_chains=4096),
}
for _k in (16, 32, 128, 256, 512):
    MH_WORKLOADS["rhchain48_pi%d" % _k] = dict(MH_WORKLOADS["rhchain48"], circuit=_rh(PI / _k),
                                                burn_in=max(2000, _k * _k // 2))


def tau_of_series(torch, ser):
    """tau_int of a [steps, chains] series: chain-pooled autocovariance by
    FFT, Geyer's initial positive sequence.  None for a constant series."""
    x = ser - ser.mean()
    S = x.shape[0]
    f = torch.fft.rfft(x, n=2 * S, dim=0)
    acov = torch.fft.irfft((f * f.conj()).real.sum(dim=1), n=2 * S)[:S] / (x.shape[1] * torch.arange(
        S, 0, -1, device=x.device, dtype=x.dtype))
    if not float(acov[0]) > 1e-12 * max(1.0, float((ser * ser).mean())):
        return None
    rho = (acov / acov[0]).cpu().numpy()
    tau = -1.0
    k = 0
    while 2 * k + 1 < S // 2:
        g = rho[2 * k] + rho[2 * k + 1]
        if g <= 0:
            break
        tau += 2 * g
        k += 1
    return float(tau)


def adaptive_tau(torch, advance, observe, min_len=512, max_len=65536):
    """Runs `advance` (one transition of the tau population) and records
    `observe` ([n_obs, chains]) until the series is at least 50 times the
    largest tau_int over the observables long (or max_len); returns (tau_int
    of the slowest observable, per-observable taus, series length)."""
    buf = []
    L = min_len
    while True:
        while len(buf) < L:
            advance(len(buf))
            buf.append(observe().to(torch.float32))
        ser = torch.stack(buf)  # [S, n_obs, chains]
        taus = [tau_of_series(torch, ser[:, o, :]) for o in range(ser.shape[1])]
        tau = max(t for t in taus if t is not None)
        if L >= 50 * tau or L >= max_len:
            return tau, taus, L
        L *= 2


def mh_compare(args, name, hidden=0):
    """ESS per second of plain Gibbs against the learned-proposal MH (1 MH
    step : gibbs_per_mh Gibbs sweeps) on the same GPU.  tau_int is the
    largest over the observables (output parities, cos/sin of the phase,
    ln|psi|) of a population of tau_chains chains, recorded until it is 50
    tau_int long; time per transition and TV_path come from long runs of the
    full population."""
    import torch
    from paper_2007_07379_amd import pbit
    from workloads import circuits as wc

    cfg = MH_WORKLOADS[name]
    chains, burn, hidden = cfg["chains"], cfg["burn_in"], hidden or cfg["hidden"]
    long_cycles, tc = cfg["long_cycles"], cfg["tau_chains"]
    G = args.gibbs_per_mh
    c = cfg["circuit"](wc)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    W, h = info["W"], info["h"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rng = np.random.default_rng(0)
    masks = sorted({int(m) for m in rng.integers(1, 1 << info["n"], size=16)}) if info["n"] > 1 else [1]
    pm = magnitude_marginal(c)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def observe(st, n):
        return lambda: path_observables(torch, pbit, s, st, info, n, masks)

    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device=dev)

    # --- plain Gibbs ---------------------------------------------------------
    # tau population: burn-in, then one sweep per transition
    st_t = torch.zeros(tc * W, dtype=torch.int32, device=dev)
    s.gibbs_run([tc], burn, 0, hist, st_t, seed=11, stream=stream)
    tau_g, taus_g, len_g = adaptive_tau(
        torch, lambda t: s.gibbs_run([tc], 0, 1, hist, st_t, seed=11, sweep_offset=burn + t, resume=True,
                                     stream=stream), observe(st_t, tc))
    # full population: burn-in, then a long timed run binned for TV
    state = torch.zeros(chains * W, dtype=torch.int32, device=dev)
    s.gibbs_run([chains], burn, 0, hist, state, seed=1, stream=stream)
    start = state.clone()
    n_long = long_cycles * (1 + G)
    # untimed warm-up of the same launch (a run this long may use the kernel
    # generated for the circuit, compiled on first use)
    warm = state.clone()
    s.gibbs_run([chains], 0, n_long, hist, warm, seed=1, sweep_offset=burn, resume=True, stream=stream)
    del warm
    hist.zero_()
    e0, e1 = ev(), ev()
    torch.cuda.synchronize()
    e0.record(stream)
    s.gibbs_run([chains], 0, n_long, hist, state, seed=1, sweep_offset=burn, resume=True, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_g = e0.elapsed_time(e1) / 1e3 / n_long  # seconds per sweep
    hist_g = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    tv_g = tv_path(hist_g, pm)
    ess_g = chains / (tau_g * t_g)

    # --- training the proposal on Gibbs samples ------------------------------
    ntrain = cfg["train"]
    train = torch.zeros(ntrain * W, dtype=torch.int32, device=dev)
    th = torch.zeros(info["hist_bins"], dtype=torch.int32, device=dev)
    s.gibbs_run([ntrain], burn, 1, th, train, seed=7, stream=stream)
    q = pbit.Proposal(s, hidden=hidden, seed=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = q.train(train, ntrain, cfg["batch"], cfg["train_steps"], lr=args.lr, stream=stream)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del train, th

    # --- MH + Gibbs ------------------------------------------------------------
    st_t = torch.zeros(tc * W, dtype=torch.int32, device=dev)
    s.gibbs_run([tc], burn, 0, hist, st_t, seed=12, stream=stream)
    acc = torch.zeros(tc, dtype=torch.int64, device=dev)

    def mh_advance(t):
        cy, r = divmod(t, 1 + G)
        if r == 0:
            pbit.mh_run(s, q, tc, 1, st_t, hist, acc, gibbs_per_mh=0, seed=12, step_offset=cy, resume=True,
                        stream=stream)
        else:
            s.gibbs_run([tc], 0, 1, hist, st_t, seed=12, sweep_offset=(1 << 30) + cy * G + r - 1, resume=True,
                        stream=stream)

    tau_m, taus_m, len_m = adaptive_tau(torch, mh_advance, observe(st_t, tc))
    acc_rate = float(acc.double().mean().item()) / ((len_m + G) // (1 + G))
    state = start.clone()
    hist.zero_()
    e0, e1 = ev(), ev()
    torch.cuda.synchronize()
    e0.record(stream)
    pbit.mh_run(s, q, chains, long_cycles, state, hist, None, gibbs_per_mh=G, seed=2, resume=True, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_m = e0.elapsed_time(e1) / 1e3 / n_long  # seconds per transition
    hist_m = hist.cpu().numpy().view(np.uint32).astype(np.uint64).reshape(1 << info["n"], 1 << info["K"])
    tv_m = tv_path(hist_m, pm)
    ess_m = chains / (tau_m * t_m)
    names = observable_names(masks)
    return {
        "workload": "%s: n=%d d=%d, h=%d free p-bits, %d chains, MADE hidden %d, 1 MH : %d Gibbs"
                    % (name, info["n"], info["d"], h, chains, hidden, G),
        "observables": "tau_int is the largest over: %s (constant ones skipped)" % ", ".join(names),
        "gibbs": {"tau_int_sweeps": tau_g, "tau_per_observable": dict(zip(names, taus_g)), "tau_series": len_g,
                  "s_per_sweep": t_g, "ess_per_s": ess_g, "tv_path": tv_g, "tv_samples": chains * n_long},
        "mh": {"tau_int_transitions": tau_m, "tau_per_observable": dict(zip(names, taus_m)), "tau_series": len_m,
               "s_per_transition": t_m, "ess_per_s": ess_m, "tv_path": tv_m, "tv_samples": chains * n_long,
               "accept_rate": acc_rate},
        "train": {"samples": ntrain, "steps": cfg["train_steps"], "batch": cfg["batch"], "seconds": t_train,
                  "loss_first": float(losses[0]), "loss_last": float(losses[-20:].mean())},
        "ess_ratio_mh_over_gibbs": ess_m / ess_g,
        "tv_ok": bool(tv_g <= 0.01 and tv_m <= 0.01),
    }


def mh_mode(args):
    out = mh_compare(args, args.workload, args.hidden)
    out["metric"] = "effective samples/s (TV<=0.01), Gibbs vs learned-proposal MH"
    print(json.dumps(out))


def masked_weight_counts(D, H):
    """Unmasked weights of the three products of a D-position, H-wide MADE
    (degrees as in the network definition)."""
    din = np.arange(1, D + 1)
    dh = 1 + (np.arange(H) * (D - 1)) // H
    dout = np.arange(D)
    return (int((din[:, None] <= dh[None, :]).sum()), int((dh[:, None] <= dh[None, :]).sum()),
            int((dh[:, None] <= dout[None, :]).sum()))


def sample_mode(args):
    """The learned proposal's MH-step network work on its own: drawing
    `chains` proposals (pbit_proposal_sample) and scoring the chains' current
    paths (pbit_proposal_score), as one MH step of pbit_mh_run does, at the
    workload's network shape.  The MFMA roofline counts one masked forward
    (2 FLOP per unmasked weight) per path drawn or scored."""
    import torch
    from paper_2007_07379_amd import pbit
    from workloads import circuits as wc
    cfg = MH_WORKLOADS[args.workload]
    c = cfg["circuit"](wc)
    s = pbit.CircuitSet(c)
    info = s.info(0)
    H = args.hidden or cfg["hidden"]
    n = cfg["chains"]
    q = pbit.Proposal(s, hidden=H, seed=3)
    D, W = q.D, info["W"]
    stream = torch.cuda.current_stream()
    out = torch.zeros(n * W, dtype=torch.int32, device="cuda")
    lq = torch.zeros(n, dtype=torch.float64, device="cuda")
    cur = torch.zeros(n * W, dtype=torch.int32, device="cuda")
    lqc = torch.zeros(n, dtype=torch.float64, device="cuda")
    q.sample(n, cur, lqc, seed=1, step=0, stream=stream)  # valid current paths
    for _ in range(max(args.warmup, 1)):
        q.sample(n, out, lq, seed=2, step=1, stream=stream)
        q.score(cur, n, lqc, stream=stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for i in range(args.steps):
        ev[i][0].record(stream)
        q.sample(n, out, lq, seed=2, step=2 + i, stream=stream)
        ev[i][1].record(stream)
        q.score(cur, n, lqc, stream=stream)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    t_s = float(np.mean([e[0].elapsed_time(e[1]) for e in ev])) / 1e3
    t_c = float(np.mean([e[1].elapsed_time(e[2]) for e in ev])) / 1e3
    n1, n2, n3 = masked_weight_counts(D, H)
    flops = 2.0 * (n1 + n2 + n3) * n
    print(json.dumps({
        "metric": "proposals/s (MADE sampler)", "value": n / t_s, "unit": "proposals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": (t_s + t_c) * 1e3, "higher_is_better": True,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "%s network: D=%d positions, two masked hidden layers of %d, %d chains (h=%d free)"
                               % (args.workload, D, H, n, info["h"])},
        "sample_ms": t_s * 1e3, "score_ms": t_c * 1e3,
        "roofline_sample": {"bound": "mfma", "achieved": flops / t_s / 1e12, "peak": BF16_PEAK / 1e12,
                            "unit": "TFLOP/s", "frac": flops / t_s / BF16_PEAK, "traffic": None,
                            "flops_per_proposal": 2.0 * (n1 + n2 + n3)},
        "roofline_score": {"bound": "mfma", "achieved": flops / t_c / 1e12, "peak": BF16_PEAK / 1e12,
                           "unit": "TFLOP/s", "frac": flops / t_c / BF16_PEAK, "traffic": None},
    }))


def gibbs_ess(torch, pbit, s, info, c, chains, sweeps, step_s, hist_total, tau_chains=4096):
    """tau_int of plain Gibbs on the timed workload (largest over the output
    parities, cos/sin of the phase and ln|psi| of tau_chains chains after
    the burn-in) and the effective samples per second of the timed run."""
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(0)
    masks = sorted({int(m) for m in rng.integers(1, 1 << info["n"], size=16)}) if info["n"] > 1 else [1]
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    st = torch.zeros(tau_chains * info["W"], dtype=torch.int32, device="cuda")
    burn = 200
    s.gibbs_run([tau_chains], burn, 0, hist, st, seed=21, stream=stream)
    tau, taus, L = adaptive_tau(
        torch, lambda t: s.gibbs_run([tau_chains], 0, 1, hist, st, seed=21, sweep_offset=burn + t, resume=True,
                                     stream=stream, specialize=1),
        lambda: path_observables(torch, pbit, s, st, info, tau_chains, masks), min_len=256)
    names = observable_names(masks)
    out = {"tau_int_sweeps": tau, "tau_per_observable": dict(zip(names, taus)), "tau_series": L,
           "tau_chains": tau_chains, "ess_per_s": chains * sweeps / tau / step_s,
           "observables": "largest tau_int over %d output parities, cos and sin of the phase, ln|psi| "
                          "(constant observables skipped)" % len(masks)}
    if info["n"] <= 22:
        out["tv_path"] = tv_path(hist_total, magnitude_marginal(c))
    return out


BF16_PEAK = 2.5e15  # MI355X dense bf16 MFMA FLOP/s


def train_mode(args):
    """MADE training throughput on the brick16 network (D = 400 lattice
    positions of the n=16, d=24 brickwork circuit, two masked hidden layers
    of 1024, batch 4096): Adam steps per second and the MFMA roofline of the
    masked products (forward, weight gradients, input gradients of the
    hidden layers), counting only unmasked weights."""
    import torch
    from paper_2007_07379_amd import pbit
    from workloads import circuits as wc
    c = wc.workload_circuit("brick16")
    s = pbit.CircuitSet(c)
    info = s.info(0)
    H, batch, steps, ntrain = 1024, 4096, max(args.steps, 1) * 40, 1 << 16
    train = torch.zeros(ntrain * info["W"], dtype=torch.int32, device="cuda")
    hist = torch.zeros(info["hist_bins"], dtype=torch.int32, device="cuda")
    s.gibbs_run([ntrain], 200, 1, hist, train, seed=7)
    q = pbit.Proposal(s, hidden=H, seed=3)
    D = q.D
    q.train(train, ntrain, batch, 5, lr=args.lr)  # warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    q.train(train, ntrain, batch, steps, lr=args.lr, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    # unmasked weights (degrees as in the network definition)
    n1, n2, n3 = masked_weight_counts(D, H)
    # forward (3 products), weight gradients (3), input gradients of the two
    # hidden layers (2): 2 FLOP per multiply-add
    flops_step = 2 * batch * (3 * (n1 + n2 + n3) - n1)
    achieved = flops_step * steps / dt
    print(json.dumps({
        "metric": "MADE training steps/s", "value": steps / dt, "unit": "steps/s", "n_gpus": 1,
        "steps": steps, "ms_per_step": dt / steps * 1e3, "higher_is_better": True, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "MADE D=%d, two masked hidden layers of %d, batch %d, Adam (brick16 paths)"
                               % (D, H, batch)},
        "samples_per_s": batch * steps / dt,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": BF16_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / BF16_PEAK, "traffic": None,
                     "flops_per_step": flops_step, "dense_flops_per_step": 2 * batch * (3 * (2 * D * H + H * H) - D * H)},
    }))


# Period finding by column sampling (Sec. 5): the paper's 27-bit example
# (250 column samples) and Table 1's 20-bit case (order 479,568; T = 2 r
# samples), with the paper's wall times on one laptop core in MATLAB
SHOR_WORKLOADS = {
    "shor27": dict(N=98743069, a=10424, n=27, T=250, paper_s=5923.0, paper="about 5,923 s"),
    "shor20": dict(N=961307, a=5, n=20, T=2 * 479568, paper_s=32 * 3600.0, paper="32 hours"),
}
# VALU instructions of one term exp(-2 pi i k x / 2^n) in shor_column_kernel:
# 32-bit multiply, conversion, scale, hardware cosine and sine, two adds; each
# issues at full rate on gfx950 (the kernel sustains more than 4 terms per
# SIMD per 4 cycles' worth of these, so none can be quarter rate)
SHOR_SLOTS_PER_TERM = 7


def shor_mode(args):
    """Column sampling for the order of a mod N (shor27: 10424 mod 98743069,
    n = 27, 250 samples; shor20: 5 mod 961307, n = 20, T = 2 r): one
    pbit_shor_run per step, P over all 2^n outputs."""
    import torch
    from paper_2007_07379_amd import pbit
    w = SHOR_WORKLOADS[args.workload]
    N, a, n, T = w["N"], w["a"], w["n"], w["T"]
    stream = torch.cuda.current_stream()
    P = torch.empty(1 << n, dtype=torch.float32, device="cuda")
    work = torch.empty(pbit.shor_work_bytes(N, a, n, T) // 8, dtype=torch.int64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        pbit.shor_run(N, a, n, T, P, work, seed=0, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        pbit.shor_run(N, a, n, T, P, work, seed=i, stream=stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    kernel_s = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev])) / 1e3
    terms = T * float(1 << n)
    slots = terms * SHOR_SLOTS_PER_TERM
    out = {
        "metric": "column-sampling wall time (Sec. 5)", "value": wall, "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": wall / w["paper_s"],
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: period finding by column sampling, N=%d, a=%d, n=%d first-register p-bits, "
                               "%d column samples, P over all 2^%d outputs" % (args.workload, N, a, n, T, n)},
        "terms_per_s": terms / kernel_s,
        "roofline": {"bound": "alu", "achieved": slots / kernel_s / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "Tslot-op/s", "frac": slots / kernel_s / VALU_PEAK, "traffic": None,
                     "kernel": "shor_column_kernel (+ shor_prepare_kernel)", "kernel_ms": kernel_s * 1e3,
                     "slots_per_term": SHOR_SLOTS_PER_TERM},
        "baseline_note": "vs_baseline divides by the paper's %s for the same workload on one laptop "
                         "core in MATLAB (other hardware and software: context)" % w["paper"],
    }
    if not args.no_cpu:
        from oracle import shor as oshor
        xs = oshor.draws(n, T, 0)
        ks = list(range(0, 1 << n, (1 << n) // max(1, min(1 << n, (1 << 23) // T))))
        t0 = time.perf_counter()
        oshor.column_probs(N, a, n, xs, ks=ks)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": dt * (1 << n) / len(ks), "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": "%d of the 2^%d outputs (x %d samples) in %.1f s, scaled to all"
                                         % (len(ks), n, T, dt)}
    print(json.dumps(out))


def copy_mode(args):
    """One plain device-to-device copy of known size, the reference point that
    scales the FETCH_SIZE / WRITE_SIZE hardware counters to bytes."""
    import torch
    n = args.copy_mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    assert bool((b == 1).all())
    print(json.dumps({"copy_bytes": 4 * n, "read_kib": 4 * n / 1024, "write_kib": 4 * n / 1024}))


def source_digest(*names):
    import hashlib
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2007_07379_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# HBM traffic per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE passes over
# `bench.py --steps 1 --warmup 0 --no-cpu`, scaled by the same counters read
# for a 256 MiB device copy (FETCH_SIZE reads 0.5 of the copy's bytes on this
# part, WRITE_SIZE 1.0).  Keyed by kernel, workload and a digest of the kernel
# sources: a figure is reported only while the sources it was taken on are
# unchanged.
MEASURED_TRAFFIC = {
    # (kernel, workload): (source digest, sources, read bytes, written bytes)
    ("pbit_uniform_sweep (generated for the circuit, 4 lanes per chain)", "rct12"):
        ("9a34a822711a64ac", ('jit.cpp', 'jit.h', 'compile.cpp', 'blob.h'), 131.75 * 1024 * 2, 36864 * 1024 * 1),
    ("gibbs_pair_kernel<16>", "rct12"): ("1cc1ef522bb50502", ('gibbs_pair.hip', 'philox.h', 'blob.h', 'gibbs.h'), 157.5 * 1024 * 2, 36864 * 1024 * 1),
    # the 2^24-bin histogram's atomics, 32 bytes each (profiles/pbit_uniform_sweep_brick20_pmc.md)
    ("pbit_uniform_sweep (generated for the circuit, 1 lanes per chain)", "brick20"):
        ("9a34a822711a64ac", ('jit.cpp', 'jit.h', 'compile.cpp', 'blob.h'), 171.938 * 1024 * 2, 8.19354e7 * 1024 * 1),
}


def measured_traffic(kernel, workload):
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    digest, srcs, rd, wr = rec
    if source_digest(*srcs) != digest:
        return None
    return rd + wr


def batch_mode(args):
    """256 random Clifford+T circuits (n 4..16, d 4..32, chains proportional
    to 2^n, 2^22 in total), 200 + 2000 sweeps, one persistent launch per
    lattice-width class."""
    import torch
    from paper_2007_07379_amd import pbit
    from workloads import circuits as wc
    data = json.load(open(os.path.join(wc.DATA_DIR, "batch256.json")))
    circs, chains = data["circuits"], data["chains"]
    burn, sweeps = 200, 2000
    s = pbit.CircuitSet(circs)
    infos = [s.info(i) for i in range(len(circs))]
    updates = sum(ch * (burn + sweeps) * inf["h"] for ch, inf in zip(chains, infos))
    ops = 0.0
    for i, ch in enumerate(chains):
        ps, pa, _ = algorithmic_ops(s.export(i))
        ops += ch * ((burn + sweeps) * ps + sweeps * pa)
    # the run is captured once into a hipGraph (on a stream of its own: a
    # graph needs a non-null stream) and replayed by the timed steps
    stream = torch.cuda.Stream()
    hist = torch.zeros(s.hist_bins(), dtype=torch.int32, device="cuda")
    state = torch.zeros(s.state_words(chains), dtype=torch.int32, device="cuda")
    kw = dict(persistent=1, specialize=args.specialize, use_graph=not args.no_graph)
    kinds = [s.launch_shape(chains, burn, sweeps, idx=i, **kw)["kernel"] for i in range(len(circs))]
    n_spec = sum(1 for k in kinds if k == pbit.KERNEL_SPECIALISED)
    t0 = time.perf_counter()
    # the first run compiles the specialised kernels (on host threads) and
    # captures the graph
    s.gibbs_run(chains, burn, sweeps, hist, state, seed=0, stream=stream, **kw)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    for _ in range(max(args.warmup, 1) - 1):
        s.gibbs_run(chains, burn, sweeps, hist, state, seed=0, stream=stream, **kw)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        s.gibbs_run(chains, burn, sweeps, hist, state, seed=0, stream=stream, **kw)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3
    ms_per_step = wall / args.steps * 1e3
    out = {
        "metric": "p-bit updates/s", "value": updates / (ms_per_step / 1e3), "unit": "updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batch256: 256 random Clifford+T circuits, n 4..16, d 4..32, %d chains "
                               "in total (proportional to 2^n), %d burn-in + %d sweeps, persistent launch"
                               % (sum(chains), burn, sweeps)},
        "samples_per_s": sum(chains) * sweeps / (ms_per_step / 1e3),
        "roofline": {"bound": "alu", "achieved": ops / kernel_s / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "Tslot-op/s", "frac": ops / kernel_s / VALU_PEAK, "traffic": None,
                     "kernel": ("batched_kernel (width classes)" if not n_spec else
                                "pbit_uniform_sweep for %d circuits on launches of their own + batched_kernel "
                                "for the rest" % n_spec),
                     "kernel_ms": kernel_s * 1e3},
        "warmup_s": t_warm,
        "first_run_s": t_first,
        "specialised_circuits": n_spec,
        "graph": bool(kw["use_graph"]),
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="brick20")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=0,
                    help="chains of the oracle's timed sample (0: about 10^10 updates, 10-20 s of host cores)")
    ap.add_argument("--no-ess", action="store_true", help="gibbs mode: skip tau_int / ESS and the MH comparison")
    ap.add_argument("--mh-workload", default="rhchain48_pi256",
                    help="gibbs mode: workload of the learned-proposal comparison ('' to skip)")
    ap.add_argument("--mode", default="gibbs", choices=["gibbs", "mh", "copy", "train", "shor", "sample"])
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--specialize", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--no-graph", action="store_true", help="batch256: enqueue each run instead of a graph replay")
    ap.add_argument("--hist-mode", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="histogram placement (pbit_gibbs_cfg.hist_mode), gibbs mode")
    ap.add_argument("--gibbs-per-mh", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--hidden", type=int, default=0, help="mh mode: MADE width (0: the workload's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: chains are independent, so N GPUs would each run "
              "their own share of them; no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    if args.mode == "copy":
        copy_mode(args)
        return
    if args.mode == "train":
        train_mode(args)
        return
    # the modes with workloads of their own take their default when
    # --workload was left at the Gibbs default, and refuse unknown names
    def mode_workload(table, default):
        if args.workload == ap.get_default("workload"):
            args.workload = default
        elif args.workload not in table:
            ap.error("--mode %s: unknown workload %r (one of: %s)" % (args.mode, args.workload, ", ".join(table)))

    if args.mode == "shor":
        mode_workload(SHOR_WORKLOADS, "shor27")
        shor_mode(args)
        return
    if args.mode == "sample":
        mode_workload(MH_WORKLOADS, "brick16")
        sample_mode(args)
        return
    if args.mode == "mh":
        mode_workload(MH_WORKLOADS, "brick16")
        mh_mode(args)
        return
    if args.workload == "batch256":
        batch_mode(args)
        return

    import torch
    from paper_2007_07379_amd import pbit
    from workloads import circuits as wc

    w = wc.WORKLOADS[args.workload]
    c = wc.workload_circuit(args.workload)
    chains, burn, sweeps = w["chains"], w["burn_in"], w["sweeps"]
    soft_J = w.get("soft_J", 0.0)
    s = pbit.CircuitSet(c, soft_zero_J=soft_J)
    info = s.info(0)
    h = info["h"]
    blob = s.export(0)
    per_sweep, per_sample, nnz = algorithmic_ops(blob)

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    # uint32 counts: a run whose chains x sweeps reaches 2^32 is cut into
    # equal parts (the chain state carries over), each with its own
    # histogram; the first part also runs the burn-in
    per_part = (2 ** 32 - 1) // chains
    n_parts = -(-sweeps // per_part)
    parts = []
    done = 0
    for k in range(n_parts):
        n = (sweeps - done) // (n_parts - k)
        parts.append((burn if done == 0 else 0, n, 0 if done == 0 else burn + done))
        done += n
    hists = [torch.zeros(info["hist_bins"], dtype=torch.int32, device=dev) for _ in parts]
    state = torch.zeros(chains * info["W"], dtype=torch.int32, device=dev)

    def run_parts():
        for (b, n, off), hh in zip(parts, hists):
            s.gibbs_run([chains], b, n, hh, state, seed=0, sweep_offset=off, resume=off > 0, stream=stream,
                        hist_mode=args.hist_mode)

    def step():
        for hh in hists:
            hh.zero_()
        run_parts()

    shape = s.launch_shape([chains], parts[0][0], parts[0][1], hist_mode=args.hist_mode)
    kname = {pbit.KERNEL_ONE_LANE: "gibbs_kernel<%d,%s>" % (shape["kernel_words"],
                                                          "true" if info["uniform"] else "false"),
             pbit.KERNEL_TWO_LANE: "gibbs_pair_kernel<%d>" % shape["kernel_words"],
             pbit.KERNEL_PERSISTENT: "batched_kernel",
             pbit.KERNEL_SPECIALISED: ("pbit_uniform_sweep (generated for the circuit, %d lanes per chain)"
                                       % shape["lanes_per_chain"]) if info["uniform"] else
                                      "pbit_general_sweep (generated for the circuit, one lane per chain)"}[shape["kernel"]]
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        run_parts()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # samples binned by one run (fewer than chains x sweeps with soft zeros)
    step()
    torch.cuda.synchronize()
    binned = float(sum(int(hh.to(torch.int64).sum().item()) & 0xFFFFFFFFFFFF for hh in hists))
    hist_total = sum(hh.cpu().numpy().view(np.uint32).astype(np.uint64) for hh in hists).reshape(
        1 << info["n"], 1 << info["K"])
    kms = [a.elapsed_time(b) for a, b in ev]
    kernel_s = float(np.mean(kms)) / 1e3
    ms_per_step = wall / args.steps * 1e3
    updates = chains * (burn + sweeps) * h
    value = updates / (ms_per_step / 1e3)
    ops = chains * ((burn + sweeps) * per_sweep + sweeps * per_sample)
    achieved = ops / kernel_s
    out = {
        "metric": "p-bit updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %s, n=%d d=%d K=%d, %d chains x (%d burn-in + %d) sweeps, h=%d free p-bits"
                        % (args.workload, c.get("name", ""), info["n"], info["d"], info["K"], chains,
                           burn, sweeps, h),
            "chains": chains, "sweeps": sweeps, "burn_in": burn, "free_bits": h,
            "soft_zero_J": soft_J,
        },
        "samples_per_s": chains * sweeps / (ms_per_step / 1e3),
        "binned_samples_per_s": binned / (ms_per_step / 1e3),
        "lattice_bit_updates_per_s": value * info["L"] / max(h, 1),
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK / 1e12,
            "unit": "Tslot-op/s",
            "frac": achieved / VALU_PEAK,
            "traffic": measured_traffic(kname, args.workload),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
            "kernel": kname,
            "kernel_ms": kernel_s * 1e3,
            "launches_per_step": len(parts),
            "kernel_ms_per_launch": kernel_s * 1e3 / len(parts),
            "launch": {k: shape[k] for k in ("block", "lds_hist", "lanes_per_chain", "lds_bytes",
                                             "sweeps_per_launch")},
            "ops_per_update": per_sweep / max(h, 1),
            "ops_per_sample": per_sample,
        },
    }
    if not args.no_ess:
        out["ess"] = gibbs_ess(torch, pbit, s, info, c, chains, sweeps, ms_per_step / 1e3, hist_total)
        if args.mh_workload:
            # the learned proposal where it pays: a rotated-Hadamard chain whose
            # path law is strongly correlated (every conditional of the
            # uniform workloads is 1/2, so Gibbs is already i.i.d. there)
            out["learned_proposal"] = mh_compare(args, args.mh_workload)
    if not args.no_cpu:
        cc = args.cpu_chains or max(64, min(chains, int(1e10 / ((burn + sweeps) * max(h, 1)))))
        out["cpu_baseline"] = cpu_baseline(c, h, burn, sweeps, cc, soft_J or None)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
