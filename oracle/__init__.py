"""Plain, slow FP64 CPU oracle for multilevel Monte-Carlo estimation of tr(A^-1).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes anything in this package; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark call it.  It shares no code with the GPU
path: the only module both sides use is ``workloads`` (seeded synthetic input
generators, which hold none of the method's arithmetic).

Every function states the passage of Frommer, Nasr Khalil and Ramirez-Hidalgo,
"A Multilevel Approach to Variance Reduction in the Stochastic Estimation of
the Trace of a Matrix" (arXiv 2108.11281) that it follows.  Where the paper is
silent or garbled, the reading taken is stated next to the code.

Modules
  philox     Philox4x64-10 counter RNG and the probe distributions (Sec. 3)
  operators  2D Poisson (Example 4.1), Wilson-like 2-spin U(1) (Example 4.3),
             3D 7-point variable coefficient diffusion
  hierarchy  orthonormal aggregation P, R = P^H, Galerkin A_{l+1} = R A_l P
             (Sec. 4.1, Remark 4.3)
  mlmc       exact per-sample level differences, direct coarsest trace
             (Remark 4.2), the MLMC estimator and its accuracy control (Sec. 2,
             Sec. 5), plain Hutchinson (eq. plain_tr_estimate)
  nn         learned-smoother convolution network forward/backward in FP64
"""
