"""CPU oracle for the data-parallel GKR prover (TEST INFRASTRUCTURE ONLY).

A plain, slow, big-integer implementation of what the GPU path computes:
forward evaluation of a layered add/mul circuit, the Fiat-Shamir transcript,
the two-phase linear-time (Libra-style) GKR sumcheck prover and the verifier.
Field elements are Python ints reduced mod the BN254 scalar-field prime.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package. The product path never calls it and shares no code
with it; the two meet only through the seeded generator in `gkr_synth`.

Parity status: pinned. Field laws, the SHA-256 transcript (hashlib and the
FIPS 180-4 vectors), eq/MLE identities, brute-force hypercube sums of every
round polynomial on tiny circuits, the per-round invariant g_j(0)+g_j(1) =
claim, verifier acceptance and tamper rejection pin each part; see the tests.
"""
from . import field, mle, transcript, circuit, prover, verifier, general, goldilocks  # noqa: F401
