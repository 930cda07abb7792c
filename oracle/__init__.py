"""CPU oracle for multistage mixed precision iterative refinement (MSIR).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links it, and this package never imports the product.

The oracle is a plain, slow, readable restatement of the method of Oktay and
Carson, "Multistage Mixed Precision Iterative Refinement" (arXiv 2107.06200):

* ``fmt``      unit roundoffs (Table 3) and round-to-nearest-even into each format
* ``dd``       double-double arithmetic standing in for quadruple precision
* ``scaling``  power-of-two equilibration before a half-precision LU (Sec. 2.1.2)
* ``lu``       LU with partial pivoting whose stored factors live in u_f (Alg. 4 init)
* ``solve``    substitution with the factors in u_f or in a higher precision
* ``ops``      residual and matrix-vector products in a named precision
* ``gmres``    left-preconditioned GMRES used by SGMRES-IR (Alg. 3) and GMRES-IR (Alg. 2)
* ``msir``     the multistage controller (Alg. 4 with the criteria of Sec. 2.1.1)
* ``metrics``  forward, normwise and componentwise backward errors (Sec. 2, eqs. for ferr/nbe/cbe)
* ``bounds``   the condition-number limits of Sec. 2.2 / Table 4

Every floating-point operation whose precision the method fixes is emulated in
float64 followed by an explicit rounding to the target format (exact for
+, -, *, / and sqrt whenever the wide format has at least 2p+2 bits), or by an
explicitly exact construction (fp32 fused multiply-add, double-double).
"""
