"""CPU FP64 oracle for the Inverse Fast Multipole Method (Ambikasaran & Darve).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constants with the HIP library.

Contents (each function cites the passage of the paper it follows):

* ``geometry``   -- uniform quadtree, Morton (Z) order, neighbour and
                    interaction lists (Section 4.2, table of cluster lists;
                    Section 2.2 for the Z ordering).
* ``chebyshev``  -- Chebyshev interpolation nodes, Lagrange basis, child to
                    parent transfer maps (Section 5: 8 nodes per dimension in
                    the paper; the order p is an input here).
* ``kernels``    -- kernel functions K(r) of the configurations.
* ``fmm_matrix`` -- the FMM matrix A~ written out densely from its definition
                    (Section 2.2), an FMM matrix-vector product, and the
                    diagonal rule.
* ``householder``-- plain Householder QR, with and without column pivoting.
* ``ifmm``       -- the IFMM itself: extended sparse system (Section 4.1),
                    elimination with on-the-fly compression (Algorithm 1),
                    back substitution (Algorithm 2), and FP64 iterative
                    refinement with the FMM product.

Pins: ``tests/test_oracle_*.py`` check every function here against closed
forms, brute force and exact identities (see each test's docstring).
"""
