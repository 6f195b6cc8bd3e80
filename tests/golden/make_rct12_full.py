"""Writes the expected result of the full random Clifford+T run (n=12,
d=40, K=3; 65,536 chains x (200 burn-in + 10,000) sweeps, Philox seed 0,
circuit id 0) from the CPU oracle alone:

  rct12_full_hist.npz   uint64[4096, 8] phase-bin counts
  rct12_full_state.json SHA-256 of the final lattice words, uint32[65536, 16]
                        little-endian, chain-major

    python tests/golden/make_rct12_full.py [threads]

Only `oracle/` and the committed circuit are used; the GPU path is not.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import chain as och  # noqa: E402
from oracle import circuit as oc  # noqa: E402
from oracle import compile as ocomp  # noqa: E402
from workloads import circuits as wc  # noqa: E402

CHAINS, BURN, SWEEPS, SEED = 65536, 200, 10000, 0


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 8)
    c = wc.workload_circuit("rct12")
    comp = ocomp.compile_circuit(oc.from_dict(c))
    t0 = time.time()
    st, h = och.gibbs(comp, CHAINS, BURN, SWEEPS, seed=SEED, threads=threads)
    dt = time.time() - t0
    assert int(h.sum()) == CHAINS * SWEEPS
    np.savez_compressed(os.path.join(HERE, "rct12_full_hist.npz"), hist=h.astype(np.uint64))
    digest = hashlib.sha256(np.ascontiguousarray(st, dtype="<u4").tobytes()).hexdigest()
    meta = {
        "what": "final lattice words of the full rct12 run, written by the CPU oracle",
        "circuit": "workloads/data/rct12.json", "chains": CHAINS, "burn_in": BURN, "sweeps": SWEEPS,
        "seed": SEED, "circuit_id": 0, "W": int(comp.W), "h": int(comp.h),
        "layout": "uint32[chains, W] little-endian, chain-major",
        "sha256": digest,
        "first_chain": [int(v) for v in st[0]], "last_chain": [int(v) for v in st[-1]],
    }
    with open(os.path.join(HERE, "rct12_full_state.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print("rct12 full: %.1f s on %d threads, %.3g updates/s" % (dt, threads, CHAINS * (BURN + SWEEPS) * comp.h / dt))


if __name__ == "__main__":
    main()
