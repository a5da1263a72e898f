"""CPU FP64 oracle for the batched ALB eigensolves — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy/SciPy implementations of what the GPU
path computes.  Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does.  It
shares no code with the GPU library: its only common dependency is the seeded
input generator (``workloads``), which holds no solver arithmetic.

Modules
-------
planewave   local Kohn-Sham Hamiltonian H^{Q_k} on a periodic plane-wave grid
            (Eq. (1), LocalKS) and its dense form for tiny grids
lobpcg      LOBPCG (Algorithm 1) with the Teter preconditioner (Eq. (3))
chebyshev   Chebyshev filter and filtered subspace iteration (Algorithm 2,
            applied to H^{Q_k}), spectral bounds by Lanczos
alb         restriction to E_k and SVD orthonormalisation (ALB construction,
            "Generating ALB functions" subsection); subspace angles
band_energy band energy through the Chebyshev filter and its adjoint gradient

Pins: every function is checked in ``tests/test_oracle.py`` against closed
forms, brute force, invariants or an independent library routine.  No part of
the oracle is "parity unpinned".
"""
