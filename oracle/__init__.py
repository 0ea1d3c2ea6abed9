"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of what the parametric
matmul path computes, written from the paper and pinned by the tests under
``tests/`` against values the paper prints, closed forms and brute force:

* ``matmul``        -- the matrix product (C, double / wrapping uint32);
* ``comprehensive`` -- the comprehensive-optimization algorithm (Algorithms 1
                       and 2, Section 3) over polynomial constraint systems,
                       with brute-force consistency over finite domains;
* ``enumerate``     -- a brute-force enumerator of the matmul family's
                       resource constraints over machine and parameter grids;
* ``mlp``           -- the cost-model network in float64 (forward, backward,
                       mean-squared error, Adam).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it.
"""
