"""Plain FP64 CPU oracle for the incremental SVD engine -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  The GPU engine
never calls it and shares no code with it; the only common dependency is the
seeded input generator ``synth`` (inputs only, none of the method).

Contents, each following the paper step by step in FP64:
* ``svd``      -- own one-sided Jacobi full SVD (C, ``jacobi.c``) and TruncatedSVD
* ``brand``    -- Algorithms A1 (row append), A2 (column append), A3 (rank-1)
* ``metrics``  -- N_t recurrences, EVR, E_inc / E_opt / gap / ratio, principal angles
* ``policies`` -- periodic, error-threshold, angle-threshold, adaptive rank
* ``engine``   -- the engine loop of Algorithm 1 with policy evaluation
* ``finance``  -- causal de-meaning, low-rank covariances, portfolio volatility and
                  the covariance / risk errors of the finance study (Section 5)

Pins (tests/test_oracle_*.py): LAPACK's SVD via numpy on random, graded,
rank-deficient inputs and the 2x2 closed form; Eckart-Young; untruncated
appends equal the SVD of the appended matrix; truncated appends equal the
truncated SVD of [A_hat; x^T]; the rank-1 projection identity; N_t against
the direct sum; closed-form principal angles and scipy's subspace_angles;
invariants (ratio >= 1, 0 <= EVR <= 1, orthonormality) along a full
500x50 -> 1500x50 stream.
"""
