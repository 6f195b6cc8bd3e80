"""CPU oracle for Feynman-path sampling on the p-bit Boltzmann machine.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
path (no kernels, headers, helpers, tables or pre/post-processing); the two
meet only through the seeded circuit generators in `workloads/`.

Everything here is plain and slow on purpose, in FP64, each function citing
the passage of the paper it follows:

  exact.py      statevector of Eq. (U), brute-force Feynman-path sum of
                Eq. (path), the magnitude circuit and Z of Eq. (weightedS)
  compile.py    gate energies Eq. (UE) as magnitude / phase-bin tables,
                the Appendix's exact elimination of zero entries (copy / XOR
                / NOT / CCNOT) or e^(-J) soft zeros, free p-bits, cones,
                real-energy factors,
                colouring; the lattice of a free-bit assignment evaluated
                gate by gate (three-qubit permutation gates)
  chain.c       Philox4x32-10 and the Gibbs chain of Fig. 2 steps 1-3,
  chain.py      replayed chain by chain (plain C, loaded through ctypes;
                circuits with non-affine gates in plain Python)
  estimator.py  Eqs. (U343), (U23), (U26), (U30): amplitudes, sigma, TV
  ancestral.py  an independent exact sampler of p_C (layer-by-layer)
  made.py       FP64 MADE forward / backward / Adam (the learned proposal)
  shor.py       period finding by column sampling (Sec. 5, Fig. 7) and the
                circuit of Fig. 6 built from matrices

Pins that tie each part to the paper rather than to itself live in
tests/test_oracle_*.py; none of the functions above is unpinned.  The
estimator's exact-Z and L2 legs and its sigma are pinned at exact
expectation against the statevector and the closed forms of Eq. (stdT)
(tests/test_oracle_estimator.py).  `chain.philox` has no published
known-answer vectors in reach; it is checked against an independent host
build of rocRAND's Philox4x32-10 engine when hipcc is present
(tests/test_oracle_chain.py).
"""
