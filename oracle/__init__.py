"""Plain FP64 CPU oracle of IterativeCUR (Pritchard, Park, Nakatsukasa, Martinsson,
"Fast Rank Adaptive CUR via a Recycled Small Sketch", arXiv 2509.21963).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite
(`tests/`), the smoke check in `__graft_entry__.py` and the `cpu_baseline` leg of
`bench.py` may import it.  The HIP library under `paper_2509_21963_amd/` never calls,
links or imports anything here, and nothing here imports the HIP library: the two
share no code.  The only thing both sides consume is the seeded input generator
module `paper_2509_21963_amd/workloads.py`, which holds none of the method's
arithmetic.

Modules
  rng      counter-based random numbers for the sketch operator G (Philox4x32-10,
           Box-Muller, BF16 rounding, sparse-sign sampling by Floyd's algorithm)
  lupp     textbook right-looking LU with partial pivoting, returning pivot order
  icur     the sketch G A, the IterativeCUR loop of Alg. 1, exact residual norms,
           the Schur-complement and recurrence identities, the risk-aware threshold

Every function cites the passage of the paper it follows.  Everything is FP64 unless a
docstring says otherwise.
"""
