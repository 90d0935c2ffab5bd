"""FP64 CPU oracle for the k-space-preconditioned PDHG hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import or call anything in this
package; the product library never does, and this package imports nothing
from the product.  Every routine is a plain, slow, deliberately unfused
restatement of the paper (Ong, Uecker, Lustig, "Accelerating Non-Cartesian
MRI Reconstruction Convergence using k-space Preconditioning"), in float64 /
complex128, with numpy/scipy library primitives (FFT, sort, eigvalsh, CG) as
the only building blocks.

Modules
-------
ndft      exact multi-coil SENSE forward model and its adjoint (Problem Setup,
          Eq. model_i / model)
kb        Kaiser-Bessel kernel, its Fourier transform and grid sizes (the
          NUFFT of Beatty et al. with the oversampling and width of the
          Experiments section)
nufft     canonical float32 grid coordinates, bin keys, stable sort, tile
          touch lists, gridding NUFFT forward / adjoint
precond   l2-optimised diagonal k-space preconditioner: its definition,
          the single-channel closed form (Eq. sc_precond), the multi-channel
          form (Eq. mc_precond) and the efficient FFT/NUFFT build
wavelet   periodised Daubechies-4 (8-tap) multi-level transform and the
          complex soft threshold
pdhg      power method, step-size schedule, preconditioned PDHG, objective,
          dual objective, CG reference
unrolled  differentiable unrolled PDHG with a hand-derived reverse recursion

Pinning status of every function is listed in each module docstring.
"""
