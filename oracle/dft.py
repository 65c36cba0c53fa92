"""Brute-force O(N^2) discrete Fourier transform. TEST INFRASTRUCTURE ONLY.

F(psi)[ky, kx] = sum_{y, x} psi[y, x] exp(-2 pi i (kx x / X + ky y / Y)), written out as a
double sum so it can pin the FFT step of the oracle on tiny grids.
"""
from __future__ import annotations

import cmath


def dft2(a, inverse: bool = False):
    """Forward (or inverse, with 1/(XY)) 2-D DFT of a nested list / array, pure Python."""
    ny = len(a)
    nx = len(a[0])
    sgn = 1.0 if inverse else -1.0
    out = [[0j] * nx for _ in range(ny)]
    for ky in range(ny):
        for kx in range(nx):
            s = 0j
            for y in range(ny):
                for x in range(nx):
                    s += complex(a[y][x]) * cmath.exp(sgn * 2j * cmath.pi * (kx * x / nx + ky * y / ny))
            out[ky][kx] = s / (nx * ny) if inverse else s
    return out
