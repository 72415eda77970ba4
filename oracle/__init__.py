"""CPU FP64 oracle for the laminography operators (test infrastructure only).

This package is the checker, not the product.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP library and imports nothing from it.

Modules
-------
geometry  scan geometry, sample grids and sizes (eq:fwd, eq:uneqspace)
filters   ramp / Shepp-Logan / Parzen transfer functions (operator W)
phantom   analytic ellipsoids and Gaussian blobs: exact line integrals and
          exact 3D Fourier transforms (used for pins)
nudft     O2: the exact discrete Fourier pair L, L*, FBP written out as
          non-uniform DFT sums (eq:fftfwd, eq:fftadj, eq:fftfwdsplit)
usfft     O3: the same operators evaluated with a Gaussian USFFT in the
          paper's step order (divide by psi, FFT, convolution)
direct    O1: the direct line-integral discretisation with linear
          interpolation (a C/OpenMP library, `direct.c`)
cg        O4: conjugate gradients for the least-squares problem
          (Dai-Yuan direction + exact line search, and textbook CGLS)
prologue  O6: dark/flat field correction and negative logarithm of raw counts
search    O7: rotation-axis offset (phase ramp on the row spectra) and tilt sweeps
tv        O5: total-variation regularised reconstruction by ADMM
          (forward-difference gradient, divergence, isotropic soft
          threshold, dual update, CG on the tomography sub-problem)
"""
