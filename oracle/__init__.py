"""CPU oracle for the vector-set search hot path (test infrastructure).

This package is test infrastructure, not product code: only the test
suite, the smoke check of the entry module and the benchmark's CPU
baseline may import it.  It shares no code with the HIP library and never
imports it.

Everything here is a plain, slow, float64 (or exact integer) rendering of
what the paper defines, written so each step can be checked against the
text by eye:

  prng       splitmix64 and the random sparse projection (Def. 7's W)
  flyhash    projection + winner-take-all codes (Def. 7, Alg. 1)
  sketch     count and binary Bloom filters (Defs. 8 and 10, Algs. 3, 5)
  filter     query sketches, top-A positions, first and second filter
             (Alg. 6, filtering steps)
  hausdorff  Hausdorff distance and the two comparison measures
             (Def. 4, Sec. 3.2)
  search     the whole cascade search and exact brute force
             (Alg. 6 end to end, Def. 5)
  index      literal inverted index and max-heap forms (Def. 9, Alg. 4,
             and the heap of Alg. 6), used only to cross-check `filter`
  lowp       the precision form of the re-rank: bfloat16 / OCP E4M3
             quantisation, approximate Hausdorff values, and the exact
             re-check of candidates within a margin of the k-th
  learned    the learned projection (two-layer network before the
             winner-take-all) and its triplet training objective with
             gradients
  biovss     the full-scan search of Alg. 2: Hausdorff distance over
             Hamming distances of the codes for every set, the first c,
             then the exact re-rank

Parity status: every function is pinned by tests under tests/ (worked
examples printed in the paper, closed forms, invariants, brute force on
tiny inputs).  `prng.projection_rows` follows a construction the paper
leaves open (it only says W is random); it is pinned by a published
splitmix64 test vector and by distribution invariants.
"""
from . import prng, flyhash, sketch, filter, hausdorff, search, index, lowp, learned, biovss  # noqa: F401
