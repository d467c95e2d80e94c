"""CPU FP64 oracle for the space-time Petrov-Galerkin heat solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
import, call or execute anything in this package; only the test-suite, the
``smoke()`` check and the benchmark's CPU-baseline leg use it.  It shares no
code with the HIP path: operators are assembled here by element loops, the
time matrices by quadrature of the trial/test functions, and the solvers are
plain sparse-direct / dense routines from SciPy and NumPy.

Contents (each function cites the passage it follows):

* ``fem``         time matrices (Sec. 3, eq. (par1)) and spatial P1/Q1
                  stiffness and mass matrices by element assembly.
* ``exact``       the exact discrete space-time solution: Kronecker system
                  (Sec. 3 and Sec. 4, eq. (Kroneckersum)), Crank-Nicolson
                  stepping (Sec. 3, equivalence remark), also in resumable
                  chunks, 1-D modal solves (mode loop; DST-based for large
                  grids), 3-D modal solve,
                  Sylvester residual (Sec. 4, eq. (Sylv_Heat)).
* ``projection``  the Galerkin projection method of Sec. 4 with an extended
                  Krylov space, exact inner solves and a dense reduced solve.
* ``closed_form`` special cases with closed-form solutions (1-D sine mode,
                  manufactured continuous solution).

Pins (tests marked ``not gpu``): hand-derived time matrices and textbook
element matrices (tests/golden), closed-form eigenvalues, Kronecker versus
Crank-Nicolson versus modal solves, the rank-one closed form, O(h^2 + dt^2)
convergence to a manufactured solution, and planted-mistake checks.
"""
