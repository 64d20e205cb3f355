"""CPU oracle for the SubQuad hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the GPU path computes:
3-mer shingling and MinHash signatures, LSH banding into candidate pairs, Smith-Waterman
(Gotoh) local alignment scores, and the per-pair gated fusion forward and backward.
Floating point is float64. Each function cites the passage of the paper (arXiv 2602.17330)
it follows; where the paper is silent the reading taken is stated in the docstring.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may import
anything from this package. It shares no code with the GPU path (the ``synth`` input
generators aside) and never imports it.

Parity status: every function here is pinned by CPU tests against values fixed by the
mathematics (brute force on tiny inputs, closed forms, textbook special cases, published
generator outputs, invariants); see ``tests/test_oracle_*.py``.
"""
from . import edit, gate, graph, lsh, minhash, proto, rmt, sw  # noqa: F401
