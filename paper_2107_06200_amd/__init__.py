"""MSIR on MI355X: multistage mixed precision iterative refinement for dense Ax=b.

The solver itself lives in the HIP library ``libmsir.so`` (built from
``csrc/``); ``paper_2107_06200_amd.msir`` is its thin ctypes binding.
``paper_2107_06200_amd.workloads`` builds the seeded synthetic inputs.
Importing this package does not load the library.
"""
