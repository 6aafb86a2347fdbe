"""Plain CPU reference ("oracle") for the axisymmetric MFS solver of
Liu & Barnett, "Efficient numerical solution of acoustic scattering from
doubly-periodic arrays of axisymmetric objects" (J. Comput. Phys., 2016).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may call it.  It shares no code with the GPU path: the only
common dependency is the seeded input description in ``workloads``.

Everything here is complex128 numpy/scipy, written for readability rather
than speed: each function follows one passage of the paper (cited in its
docstring) in the paper's order and notation.  Library primitives used as
single steps: numpy FFT, numpy/scipy SVD and least squares, scipy spherical
Bessel functions and spherical harmonics.

Modules
  geometry  generating curve, normals, collocation and complexified sources
  kernel    Helmholtz fundamental solution and its target-normal derivative
  onebody   ring-kernel modal fill, RHS Fourier data, per-mode truncated-SVD
            least squares, point-source form and field evaluation
  mie       Mie series for a sound-hard sphere (textbook special case)
  periodic  periodizing scheme: walls, spherical-harmonic and Rayleigh-Bloch
            bases, the A_else / B / C / Q blocks, Schur-complement GMRES,
            recovery of the Bragg amplitudes and the error metrics
  gmres     unrestarted GMRES (Arnoldi with modified Gram-Schmidt)

Parity status of each function is stated in its docstring; every function
used on the hot path is pinned by a ``-m "not gpu"`` test against a closed
form, an invariant or an independent route.
"""
