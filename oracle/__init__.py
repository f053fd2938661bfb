"""Plain FP64 CPU oracle for the state-vector gate engine.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls,
links or executes this package; only the test suite, the smoke check and the
CPU-baseline leg of the benchmark do.  It shares no code with the GPU path:
gate matrices, pair loops, norms, the two-byte codec and the entangling-gate
decomposition are all written out here independently, from the paper
(Willsch et al., "Benchmarking Supercomputers with the Juelich Universal
Quantum Computer Simulator", arXiv:1912.03243) and textbook definitions.

Modules
  gates          textbook 2x2 / 4x4 gate matrices
  statevector    Eq. (1) pair update, controlled and k-qubit gates, norm,
                 amplitudes, circuit runner
  dense          brute-force 2^n x 2^n embeddings (n <= 10), used to pin the
                 pair loops
  observables    single-qubit expectation values <Q_alpha(i)> (Section 3)
  enc2           reference two-byte block codec (bit-exact target for the GPU)
  decomposition  CZ decomposition Eq. (2) and branch sum Eq. (3) (Section 4)

Every floating-point result is FP64 except the two-byte codec, whose format
is defined in FP32.
"""
from . import gates, statevector, dense, observables, enc2, decomposition  # noqa: F401
