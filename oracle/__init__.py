"""FP64 CPU oracle for the FR/CPR Jacobian-free implicit solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or call anything in this package.
The product path (the HIP library and its Python binding) never imports it,
and this package imports nothing from the product.

Plain, slow, obviously-correct numpy implementations of what the method
computes, each function citing the passage of Wang & Yu, "A comparative study
of implicit Jacobian-free Rosenbrock-Wanner, ESDIRK and BDF methods for
unsteady flow simulation with high-order flux reconstruction formulations"
(arXiv:1904.04825) that it follows.

Array layout (shared input/output convention, not shared code):
U[v, e, k] with v in (rho, rho u, rho v, E), e = ey*nx + ex, k = b*(P+1) + a
where a indexes the xi (reference-x) solution point and b the eta one.
"""
