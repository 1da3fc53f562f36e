"""CPU oracle for the two-level fully discrete Method of Local Corrections.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its Python
binding) may import, call or link anything in this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code, tables or constants with the GPU path.

Everything is plain NumPy / SciPy in float64, written from the paper
(Kavouklis & Colella, "Computation of Volume Potentials on Structured Grids
via the Method of Local Corrections"), one function per step:

  stencils     Mehrstellen L19 / L27 Laplacians (sec. 2, appendix A.1)
  dgf          discrete Green's function by a Dirichlet solve (appendix A.1)
  geometry     index boxes, grow / coarsen operators, patches (sec. 2, sec. 4)
  convolution  local discrete convolution: literal sum, and Hockney's
               method (appendix A.2)
  legendre     Legendre moments by composite Boole quadrature (sec. 3, sec. 4.1)
  interp       coplanar tensor-product Lagrange interpolation (sec. 3.1, 4.1)
  mlc          the fully discrete two-level algorithm, steps 1-3 (sec. 4.1)

Parity status of each function is stated in its docstring; the pins are the
`-m "not gpu"` tests under tests/.  Functions without an independent pin say
"parity unpinned".
"""
