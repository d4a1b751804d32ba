"""Plain CPU FP64 oracle for H2 construction from Hessian-vector products.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything under this package: only the test suite, the smoke entry point
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP library (no kernels, headers, helpers, tables or constants); the only module
both sides use is the seeded input generator, which holds none of the method's
arithmetic.

Every function follows the paper's statement of the method (arXiv 2003.10173,
"Hierarchical Matrix Approximations of Hessians Arising in Inverse Problems
Governed by PDEs"), step by step, in float64, with numpy/LAPACK routines as the
only library primitives (matmul, QR, SVD, eigvalsh).  Where the paper is silent
the reading taken is stated in the docstring of the function that takes it.

Modules
  rng       counter-based Gaussian stream (splitmix64 + Box-Muller)
  tree      KD cluster tree and admissibility block lists (Sec. 2, Sec. 3.1)
  h2        H2 container, HGEMV (Sec. 3.2 four-stage product), dense expansion
  peel      randomized peeling + recompression into strong H2 (Sec. 3.2, 3.3)
  ns        power-iteration norms (Sec. 3.2) and Newton-Schulz (Appendix A, Alg. 1-3)
  hessians  the synthetic Hessian-vector products of the workloads
"""
