"""FP64 CPU oracle for plain multislice STEM and the Lattice Multislice Algorithm (LMA).

TEST INFRASTRUCTURE ONLY. This package is the slow, plain, obviously-correct reference
that the GPU path is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it. The product library never imports, links or
calls anything here, and this package imports nothing from the product.

Contents (paper: Doberstein & Binev, "Lattice Multislice Algorithm for Fast Simulation
of Scanning Transmission Electron Microscopy Images"):
  physics     electron constants, frequency grid, probe (eqs. probe_wave_function,
              aberration_function, aperture_function), transmission and Fresnel
              propagator (Sec. 3.2), 2-D, 3-D and 4-D STEM outputs (Sec. 3.1, step 3)
  multislice  the multislice loop (Fig. multislice_pseudocode) and the plain STEM image
  lma         lattices (Sec. 4.2.1), nearest-translate sets and least-squares
              coefficients (Sec. 4.2.2), the LMA image (Fig. lma_pseudocode), local
              recompute (Sec. 4.2.6)
  partition   the image partition and its multislice-call count (Sec. 4.2.4)
  dft         brute-force O(N^2) DFT used to pin the FFT step

Readings of the paper where it is silent or garbled are listed in each function.
The least-squares coefficients are pinned by the normal equations where the translate set
has full column rank (they are unique there); for a rank-deficient set only the approximant
they produce is unique, and only that is pinned.
"""
