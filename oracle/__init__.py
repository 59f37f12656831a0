"""CPU oracle for total least squares by Rayleigh quotient iteration.

TEST INFRASTRUCTURE ONLY. Nothing in the library path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it. It shares no code with the GPU
path; the two meet only through the seeded inputs of ``tlsgen``.

Contents (every routine cites the passage of Oktay & Carson, "Mixed
Precision Rayleigh Quotient Iteration for Total Least Squares Problems",
that it follows):

* ``exact``        the TLS solution by its definitions: SVD of [A, b]
                   (Section 1), the same in mpmath at 50 digits, and the
                   secular equation derived from the Newton system (eq. 2).
* ``rqi``          textbook RQI (Algorithm 1), PCGTLS (Algorithm 3) and
                   RQI-PCGTLS / RQI-PCGTLS-MP (Algorithms 2 and 4) in plain
                   NumPy, with the psi stopping rule (eq. 4).
* ``polish``       Rayleigh quotient and residuals in extended precision
                   (x86 80-bit long double), standing in for the paper's
                   quadruple-precision error evaluation (Section 4).
* ``certify``      a-posteriori certificates of a computed (sigma, x).
* ``constraints``  the precision constraints of Section 3.1 from exact
                   singular values.
* ``lowprec``      simulated low-precision scaled Cholesky factor
                   (Section 3.1, two-sided diagonal scaling).
* ``mlp``          float64 forward, backward and Adam for the warm-start
                   network (project addition, not in the paper).
* ``costmodel``    the operation-count model of Section 3.2.

Parity status of each routine is recorded in its module docstring.
"""
