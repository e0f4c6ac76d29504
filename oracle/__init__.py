"""CPU oracle for the MAG multiple-pattern-matching scan.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import, call or run anything in this package.
It is slow on purpose, shares no code with the HIP library, and never imports
it.

* ``oracle.match``  - the plain definition of the problem (Section 1):
  every ``(i, id)`` with ``T[i..i+m) == P_id``, from C (``occ.c``): a brute
  force double loop and a chained-hash matcher.
* ``oracle.method`` - the filter's intermediate objects written from their
  definitions (Sections 2-3): alphabet maps (per byte, and on whole q-grams
  through a 64-bit hash whose constants are a reading: the paper names no
  hash), the fixed parameter heuristic,
  superimposed q-gram classes, the Shift-Or mask table and the set of
  candidate windows, plus the class-density estimate of Section 2.
* ``oracle.mlp``    - float64 forward/backward/Adam of the parameter-selector
  MLP (no counterpart in the paper; pinned by finite differences).
* ``oracle.selector`` - the selector's pattern-set features and its grid of
  candidate (q, k, sigma') triples (pinned by hand-computed small cases).
"""
