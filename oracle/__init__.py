"""CPU FP64 oracle for the parallel-in-time combination method.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, deliberately
unoptimised restatement of what the method computes, used to check the GPU
library. Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product path never does, and nothing here
shares code with the HIP kernels or the C library.

Modules and what they restate:

  index_set  the combination index set and coefficients (Section 2.1.1,
             combination formula; Section 2.2.2, layer of a subproblem)
  grids      component grids Omega_l and sampling of the initial value
  operators  the discrete spatial operators L_l for the four operator kinds
  propagate  the backward-Euler propagator Phi = (I + dt L)^-1 and
             time-sequential stepping (Section 2, time propagation equation;
             Algorithm 1)
  krylov     textbook CG and BiCGStab (Section 4.1 solver choice), used only
             to cross-check the direct solves
  mgrit      two-level and multilevel MGRIT in linear error-correction form
             (Section 2.3.1, Algorithm 2 and the remark after it)
  combine    the combination of component solutions at arbitrary points and
             the combine-then-project operator (Section 2.1.1; Section 2.2.2)
  solve      the whole method: Algorithm 3 with time-sequential propagation
             inside each recombination block (its converged MGRIT fixed point)

All arithmetic is IEEE float64. Every function says which passage of the
paper it follows and which test pins it.
"""
