"""CPU oracle for the Gauss-Chebyshev bilateral filter (Ghosh & Chaudhury, 2016).

TEST INFRASTRUCTURE ONLY. Nothing in the GPU library imports, links or runs
anything in this package; only the tests, the smoke check and the CPU baseline
leg of the benchmark do. It shares no code with the GPU library.

Contents, each a plain FP64 statement of what the paper computes:

* ``coeffs``   -- the Chebyshev fit of exp on [-mu, mu] (Section III-A and
                  III-B: nodes, eq. 16 rescaled, recursion eq. 12-13, eq. 19),
                  computed in mpmath and rounded to FP64; Taylor coefficients
                  of the Gauss-polynomial filter (Section II).
* ``filters``  -- numpy FP64: the direct bilateral filter (eq. 1), the
                  truncated spatial Gaussian (eq. 7), the Gauss-Chebyshev
                  filter in the paper's order and notation (eqs. 6-10 with the
                  centring of eq. 17), and a pair-wise form that plugs the
                  approximate kernel (eq. 4) straight into eq. (1).
* ``adjoint``  -- FP64 gradients of the Gauss-Chebyshev filter output with
                  respect to the image and sigma_r (not in the paper).
* ``native``   -- ctypes binding of ``c/oracle.c``: the same direct and
                  Gauss-Chebyshev filters in plain C (FP64, OpenMP over rows)
                  for crops of large images.
"""
