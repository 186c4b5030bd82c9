"""FP64 CPU oracle for the truncated-Green's-function FFT convolution.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test-suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the GPU library (no kernels, no
tables, no twiddles, no constants generator): both sides receive the same seeded
densities from the separate `workloads` module and nothing else.

What it computes (Vico, Greengard, Ferrando, "Fast convolution with free-space
Green's functions"):

* greens.py      -- the truncated kernels' Fourier transforms G^L(s) of Tables 1
                    and 2 (3D/2D Laplace and Helmholtz), in algebraically equal
                    forms that avoid cancellation where the printed forms lose
                    digits.
* operator.py    -- the discrete operator of Section 4: the kernel spectrum on
                    the 4N-oversampled frequency lattice (Section 2), T as its
                    inverse DFT (the delta response), its spectrum on the 2N box,
                    the 2N aperiodic convolution, the direct 4N route, spectral
                    gradients, and a direct O(N^(2d)) summation.
* closed_form.py -- potentials and gradients of a normalised Gaussian source
                    (Section 5.1), written from their derivations, plus
                    independent radial quadratures used to pin them.
* fft.c, fft.py  -- the oracle's own DFTs: a recursive mixed-radix Cooley-Tukey
                    FFT in C (gcc, OpenMP over pencils) and the O(n^2)
                    definition that pins it.

Everything is float64 / complex128.  The FFT above and a matrix product serve
as steps; nothing is blocked, fused or reordered beyond the definitions written
in each function's docstring.
"""
