"""Plain FP64 CPU oracle of the QPAT Jacobian / priorconditioned-LSQR path.

TEST INFRASTRUCTURE ONLY. Nothing in the product library imports, calls or
links this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the GPU path: the only
common dependency is the seeded input generator ``qpat_inputs``, which holds
none of the method's arithmetic.

Each function follows the paper (Hannukainen, Hyvonen, Majander, Tarvainen,
"Efficient inclusion of total variation type priors in quantitative
photoacoustic tomography") and cites the passage it writes out:

* ``fem``      -- P1 FEM of the diffusion approximation (Sec. 2, eq. (2.1);
                  the weak form and the load matrices G(1), G(2) of the
                  Appendix), element integrals by a degree-3 quadrature rule.
* ``solve``    -- K^{-1} by a sparse direct factorisation or by Jacobi-PCG.
* ``jacobian`` -- J s and J^T t exactly as the Appendix writes them, with G(1)
                  and G(2) formed as sparse matrices.
* ``prior``    -- Perona-Malik c_u, M(u), M_delta (Sec. 3 eq. (3.7);
                  Sec. 4 eqs. (4.3), (4.5), (4.8)).
* ``plsqr``    -- priorconditioned LSQR (Sec. 4, eq. (4.10) and Algorithm 1
                  step 3), Paige-Saunders recurrences applied to A L^{-1}.
* ``driver``   -- Algorithm 1 with fixed outer/inner counts.
"""
from . import fem, solve, jacobian, prior, plsqr, driver  # noqa: F401
