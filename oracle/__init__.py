"""CPU FP64 oracle for the ESP reciprocal-space path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

Contents (each function cites the passage of the paper it follows):

* ``pswf``       -- the order-zero prolate spheroidal wave function, its
                    eigenvalue, integral and derivative (Appendix A.1).
* ``splitting``  -- the PSWF kernel split N^c / F^c, F_N, the Fourier kernel
                    and the mode-wise pressure kernel (Sec. 3.1-3.2).
* ``lattice``    -- cell algebra, structure factors over a box of integer
                    modes, and periodic neighbour pairs (library primitives
                    wrapped so that a reader can check them by eye).
* ``ewald``      -- classical Gaussian Ewald summation converged to ~1e-12,
                    the exact Coulomb reference (Sec. 2.1).
* ``esp_direct`` -- ESP with explicit structure-factor sums (Sec. 3), which
                    isolates the splitting truncation.
* ``esp_grid``   -- the four-step gridded ESP (Sec. 4.1-4.3, Algorithm 1)
                    plus the analytic-differentiation force path (App. C),
                    written plainly with a full complex FFT.

Parity status: every function is pinned by at least one test under
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
