"""CPU oracle for Magnetic-Gaussian evaluation on voxel grids (FP64).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import, call, link or execute anything in this package.
It shares no code with the HIP path and never imports it.

Contents
  recipe.py  the binding box recipe (which voxels a Gaussian touches), FP64, own exp
  gauss.py   the plain definitions: covariance, conic, amplitude, slice-profile convolution,
             rendering, analytic gradients, losses, Adam (FP64)
  brute.c    brute-force FP64 sums over every (voxel, Gaussian) pair, OpenMP
  nrf.py     the neural residual field in FP64
  warm.py    the warm-start network in FP64
  ssim.py    the SSIM term of the reconstruction loss on whole stack slices, FP64
  progressive.py  the lattice resolution transition of progressive training, FP64

Parity unpinned: nothing in this package is pinned against the paper's own outputs (the
paper prints no worked example, and its datasets are not available); every function is
pinned instead by closed forms, invariants, brute force on tiny inputs and finite /
complex-step differences, as the tests under tests/test_oracle_*.py show.
"""
