"""Plain FP64 CPU oracle for the FFT convolution scheme with weakly singular kernels.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
execute this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU path.

It computes, slowly and plainly, what the paper defines (Tiwari, Pandey, Paul,
Anand, "Fast accurate approximation of convolutions with weakly singular
kernel and its applications"):

* ``fft``        -- its own mixed-radix DFT/FFT and a naive DFT (library-free).
* ``moments``    -- kernel moments ghat(k) (Section 2.2): closed forms for the
                    log and Helmholtz kernels, an independent Gauss-Jacobi /
                    Gauss-Legendre quadrature for power kernels.
* ``scheme``     -- the discrete operator A_n (Section 2.1, eq. An) and its
                    quadrature-weight form (eqs. quad, quad_wts).
* ``smoothing``  -- Fourier smoothing of jump densities (Section 2.4).
* ``ls``         -- the Lippmann-Schwinger Nystrom system (Section 3.3,
                    eq. descretls): matvec, dense solve, restarted GMRES.
* ``metrics``    -- the relative error and observed order (eqs. rel-err,
                    ord-conv).

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, high-precision quadrature, brute force or invariants; see the
module headers for the pins.
"""
