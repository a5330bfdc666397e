"""CPU FP64 oracle for the El-WaveHoltz filter-operator path (arXiv 2205.12344).

This package is TEST INFRASTRUCTURE. It is a plain, slow, obviously correct
NumPy/SciPy restatement of what the GPU library computes, written from the
paper and sharing no code, headers or tables with the HIP library.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does.

Modules
  problem   grid, boundary faces, unknown-node mask, trapezoid weights
  operator  the discrete stress divergence L_h, assembled from a discrete
            elastic energy (Sec. 4.1, eq. (symmetric FD); reading of Sec. 4.1
            for the Cartesian specialisation and the free-surface closure)
  stepping  time-step rule, corrected leapfrog, filter weights, the filter
            Pi_h, the affine split A_h = I - S_h, b = Pi_h 0 (Sec. 3, 4.3, 4.5);
            the modified trapezoid weights of the remark closing Sec. 4.4
  krylov    CG / conjugate residual / MINRES / GMRES in the M inner product
            (Sec. 4.5; MINRES: the remark in Sec. 4.4)
  direct    direct solve of the discrete Helmholtz system (Sec. 4.3)
  spectral  continuous and trapezoid filter transfer functions (Sec. 3, App. B)
  curvilinear  the stress divergence on a mapped 2-D grid (Sec. 4.1; the
            annular sectors of Sec. 5.5), same interface as operator
  curvilinear3d  the same on a mapped 3-D grid (Sec. 4.1; the partial
            toroidal shell of Sec. 5.11)
  twofield  the two-field (displacement, velocity) filter for impedance faces
            (the remark of Sec. 3), damped corrected leapfrog, GMRES

All arithmetic is IEEE float64.  Parity status of each function is stated in
its docstring; the free-surface closure is a reading of the paper (the paper
defers the exact boundary stencils to another publication) and its absolute
values are "parity unpinned" beyond the invariants listed there.
"""

from . import problem, operator, stepping, krylov, direct, spectral, curvilinear, curvilinear3d, twofield  # noqa: F401
