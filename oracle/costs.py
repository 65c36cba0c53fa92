"""Operation-count models of the paper (Sec. 3.2 complexity, Sec. 4.2.1). TEST INFRASTRUCTURE ONLY.

T_MS = N (2 XY + 2 XY log XY) per wave (FFT propagation), T~_MS = N (XY + XY K1 K2)
(real-space convolution), T_LMA = |I_f| T_MS + |P| L X'Y'. Reading: log is base 2 (the
paper's worked threshold, f >= 4 at 2048^2 with a 25 x 25 kernel, holds only then).
"""
from __future__ import annotations

import math


def t_multislice(n_slices: int, X: int, Y: int) -> float:
    return n_slices * (2 * X * Y + 2 * X * Y * math.log2(X * Y))


def t_multislice_realspace(n_slices: int, X: int, Y: int, K1: int, K2: int) -> float:
    return n_slices * (X * Y + X * Y * K1 * K2)


def t_lma(n_translates: int, n_probes: int, L: int, n_slices: int, X: int, Y: int, Xw: int, Yw: int) -> float:
    return n_translates * t_multislice(n_slices, X, Y) + n_probes * L * Xw * Yw


def realspace_breakeven_f(X: int, Y: int, K1: int, K2: int, log=math.log2) -> float:
    """Smallest real f with f^2 >= (1 + K1 K2) / (2 (1 + log XY)) (Sec. 4.2.1)."""
    return math.sqrt(0.5 * (1 + K1 * K2) / (1 + log(X * Y)))
