"""FP64 CPU oracle for the MLMC sample-solve path -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path (the
HIP library and its Python binding) never does, and the two share no code.
The only thing both sides use is the seeded input module ``mlmc_inputs``,
which holds no arithmetic of the method.

Contents (each function cites the passage of Dodwell et al., "Multilevel
Monte Carlo Simulations of Composite Structures with Uncertain
Manufacturing Defects", that it follows):

* ``mesh``     -- uniformly refined structured quadrilateral meshes
                  (Section 2.3, uniform refinement ``h_l = 2^-l h_0``).
* ``material`` -- orthotropic ply stiffness and its rotation by the fibre
                  angle (Section 3.1, rotated constitutive matrices).
* ``kl``       -- covariance operators and their truncated Karhunen-Loeve
                  expansion (Section 3.1, Eqs. covarianceFunction, inftyKL).
* ``strip``    -- Q1 stiffness assembly, Dirichlet lifting, Jacobi-PCG and
                  direct solves, fibre-stress QoI (Section 3.1, Eq.
                  matrixinplane and the integration-point maximum over the
                  central region).
* ``mlmc``     -- MC/MLMC estimators, optimal sample numbers, bias and
                  variance estimates, Algorithm 1, the biased trinomial
                  estimator (Section 2).
* ``plate``    -- classical laminate theory and the Reissner-Mindlin
                  buckling eigenproblem (Section 4.1, Eqs. CLTABD,
                  momentequil, MomentWeakForm, matrixeig).
* ``sr``       -- selective refinement, Algorithm 2 (Section 2.4).

Everything is float64.  Functions whose result has no independent pin say
"parity unpinned" in their docstring.
"""
