"""Oracle for the sample-sort hot path.  TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU code that the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in this package.  It shares no code, header, table or helper with
the GPU library (``paper_1410_6754_amd``) and imports nothing from it; the
only thing both sides share are the seeded input generators, which hold none
of the method's arithmetic.

Contents
  sort      the whole-sort definition: textbook top-down stable mergesort
            (C, ``mergesort.c``), a pure-Python twin, and brute force over all
            permutations for tiny inputs.
  rng       SplitMix64 (Steele, Lea and Flood, 2014), the counter-based
            generator that both sides implement independently for sampling.
  steps     step models of one level (sample, splitters, classification with
            equality buckets, histogram, scan, stable partition, bucket
            grouping) and of the all-pairs-rank base case.
  checkers  independent output checks: sortedness, permutation, gather,
            stability, multiset fingerprint.
  rlm       RLM-sort (Section 5): multisequence selection (Section 4.1),
            the simultaneous selections of one level, and the whole
            recurse-last multiway mergesort on small inputs.

Every function cites the passage of the paper it follows.  Parity status of
each function is listed in its docstring; the only function without a pin is
``steps.imbalance_ok`` ("parity unpinned": the load-balance lemma of Section 6
is probabilistic).
"""

from . import checkers, rlm, rng, steps  # noqa: F401
from .sort import (  # noqa: F401
    KEY_F32,
    KEY_U32,
    KEY_U64,
    brute_force_perm,
    key_dtype,
    ord_keys,
    oracle_sort,
    oracle_sort_perm,
    oracle_sort_perm_parallel,
    py_mergesort_perm,
)
