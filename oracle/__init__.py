"""FP64 CPU oracle for the line-of-sight-dependent power-spectrum multipoles of
Bianchi, Gil-Marin, Ruggeri & Percival (2015), "Measuring line-of-sight-dependent
Fourier-space clustering using FFTs".

TEST INFRASTRUCTURE. This package is the slow, plain reference against which the
HIP path is checked. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does, and it imports
nothing from the product package.

Modules
-------
estimator   the gridded Yamamoto estimator written out (Sec. 2-3, Eqs. 1-13):
            catalogue scalars, per-particle LOS weighting, CIC/TSC assignment,
            one 3D FFT per monomial grid, the k-hat contraction, the Legendre
            combination, shell averages, shot noise and normalisation.
direct      cross-paths that use neither grids-plus-FFTs nor the Cartesian
            decomposition: the interpolated-phase direct sum over particles,
            the sum over galaxies (Sec. 4, "sum-gal") and the sum over grid cells
            (Sec. 4, "sum-grid").
mlp         FP64 reference of the small correction network (forward, backward,
            Adam) used to check the GPU training kernels.
"""
