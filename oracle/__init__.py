"""FP64 CPU oracle for MACH (Tsourakakis, "MACH: Fast Randomized Tensor
Decompositions").

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import or call anything under `oracle/`.
The product path (`paper_0909_4969_amd`) never does, and the oracle imports
nothing from it: the two share no code.  The only module both sides use is
`synth` (seeded input generators, none of the method's arithmetic).

Contents
  philox.py  Philox4x32-10 counter-based generator (the per-entry coin).
  mach.py    sampling (the MACH coin toss and 1/p rescale), matricization,
             n-mode products, HOSVD (Alg. 1), HOOI sweeps (Alg. 2), core,
             fit and the comparison metrics.
  segments.py  the per-mode orderings of the kept entries (plain sorts).

Parity status per function is listed in each module header.  Every function
is pinned by a `-m "not gpu"` test to something other than itself (published
vectors, closed forms, invariants, a different library routine, brute force),
except where the header says "parity unpinned".
"""
