"""Plain, slow FP64 CPU oracle for the spectral IMEX timestep and its discrete adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle follows the paper ("Fast automated adjoints for spectral PDE solvers",
Skene & Burns) directly:

* transforms are explicit dense matrices, and their adjoints are the Hermitian
  transposes of those matrices (Methods, "Spectral transforms");
* every linear system is assembled densely and solved by a dense LU with partial
  pivoting; adjoint solves reuse the same factors (Methods, "Linear system solves");
* the IMEX Runge-Kutta and multistep schemes and their adjoints are written out
  stage by stage (Supplementary, "Initial value problems");
* the gradient follows the adjoint-state method (adjoint state equation and the
  efficient-gradient identity).

It shares no code with the GPU path.
"""
