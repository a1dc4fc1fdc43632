"""CPU oracle for phi-functions of Kronecker sums -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct FP64 implementation of what the
phiks method of Caliari, Cassini and Zivcovich computes (arXiv 2210.07667).  It
exists to check the GPU library.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does, and the
oracle imports nothing from the product package (it shares no kernels, headers,
helpers, tables or constant generators with it).  Inputs come from the neutral
``workloads`` module.

Contents (each function cites the passage it follows):

* ``gll``     -- Gauss-Lobatto-Legendre nodes/weights on [0, 1] (Section 3.3).
* ``tensor``  -- mu-mode product by explicit loops (``loops.c``, plain C compiled
                 with gcc), Tucker operator, vec layout (Section 2, Lemma 1).
* ``expm``    -- small-matrix exponential by scaled Taylor series + squaring
                 (plain definition of exp; the paper uses a Pade variant).
* ``bound``   -- numerical-range rectangle, quadrature remainder and the (s, q)
                 planner (Section 3.3, estimate (CPestimate)).
* ``phiks``   -- the two algorithms: phi-functions on one vector
                 (eqs. integrandsimul / simul) and linear combinations
                 (eqs. integrandcomb / comb), with multi-scale outputs.
* ``brute``   -- exact references for pins: assembled K, the augmented-matrix
                 exponential of Section 2 (AMH Theorem 2.1), scalar closed forms.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(tests/test_oracle_*.py) against something other than itself; none is
"parity unpinned".
"""
