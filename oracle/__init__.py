"""CPU oracle for fast fermion sampling (FFS).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes anything in this package; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark do.  The oracle shares no code with the
HIP path: it is plain numpy in float64/complex128 plus a pure-Python Philox.

Modules
  philox   -- Philox4x32-10 and the two maps the sampler draws from it.
  sampler  -- the sampler itself: per-sample random column order (Eq. (2)),
              conditional weights |u^T h|^2 (Eq. (3)), inverse-CDF draw.
  brute    -- brute-force enumerators (Eq. (1) law, exact law of the sampler).
  dpp      -- DPP front end of the applications section: dual
              eigendecomposition, eigenvector selection (lambda/(lambda+1),
              fixed-size k-DPP).
  jastrow  -- Slater-Jastrow reweighting (SI S-5): log J^2, reweighted
              densities and double occupancy, brute-force exact values.
  metropolis -- the Metropolis conditional update of SI S-7 (large L).

Every function cites the passage of the paper it follows.  Parity status:
all functions are pinned by tests/test_oracle_pins.py,
tests/test_oracle_dpp.py, tests/test_oracle_jastrow.py and
tests/test_oracle_metropolis.py; none is
"parity unpinned".
"""
