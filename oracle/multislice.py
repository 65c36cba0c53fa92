"""The multislice loop and the plain STEM image. TEST INFRASTRUCTURE ONLY.

Follows Fig. multislice_pseudocode: for j = 0..N-1, transmission psi <- t_j psi, then
propagation psi <- q * psi, the convolution done in Fourier space (Sec. 3.2, complexity
paragraph: q * psi = F^{-1}(F(q) F(psi))). The propagation step after the last slice is
applied, as the pseudocode states. Waves may be batched along a leading axis; each wave
is processed independently with exactly these steps.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph


def multislice(psi0: np.ndarray, potential: np.ndarray, sigma: float, prop: np.ndarray) -> np.ndarray:
    """Exit wave(s) psi_exit (real space) for initial wave(s) psi0 of shape (..., Y, X).

    potential: (N, Y, X) projected potential per slice in V*Angstrom.
    prop: Fourier-space propagator (Y, X), e.g. ``physics.propagator``."""
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    for j in range(potential.shape[0]):
        psi = ph.transmission(potential[j], sigma) * psi          # transmission step
        psi = np.fft.ifft2(prop * np.fft.fft2(psi))               # propagation step
    return psi


class Setup:
    """Microscope, grid and specimen-independent tables of one simulation.

    Arguments follow the paper's problem statement: grid X x Y over lx x ly, wavelength,
    interaction constant sigma, slice thickness dz, band limit (fraction of Nyquist),
    aperture alpha_max (rad), defocus Z and C_s (Angstrom), scan Px x Py, detectors as
    (inner_rad, outer_rad) pairs."""

    def __init__(self, nx, ny, lx, ly, wavelength, sigma, dz, bandlimit, alpha_max, defocus, cs,
                 scan, detectors):
        self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
        self.wavelength, self.sigma, self.dz = float(wavelength), float(sigma), float(dz)
        self.bandlimit, self.alpha_max = float(bandlimit), float(alpha_max)
        self.defocus, self.cs = float(defocus), float(cs)
        self.Px, self.Py = int(scan[0]), int(scan[1])
        self.detectors = [(float(a), float(b)) for a, b in detectors]
        self.spec0 = ph.probe_spectrum(nx, ny, lx, ly, wavelength, alpha_max, defocus, cs)
        self.prop = ph.propagator(nx, ny, lx, ly, wavelength, dz, bandlimit)
        self.masks = ph.ring_masks(nx, ny, lx, ly, wavelength, bandlimit, self.detectors)

    def probe_position(self, a: int, b: int):
        """Probe lattice point a p_x e1 + b p_y e2 with p_x = lx/Px (Sec. 4.2, set P)."""
        return (a * self.lx / self.Px, b * self.ly / self.Py)

    def probe(self, a: int, b: int) -> np.ndarray:
        return ph.probe_wave(self.spec0, self.lx, self.ly, self.probe_position(a, b))


def plain_exit_spectra(setup: Setup, potential: np.ndarray, probes, batch: int = 16) -> dict:
    """F(psi_p^exit) of every probe (a, b) in ``probes``, each propagated directly (Sec. 3.1
    steps 1-2)."""
    out = {}
    probes = list(probes)
    for s in range(0, len(probes), batch):
        chunk = probes[s:s + batch]
        psi0 = np.stack([setup.probe(a, b) for a, b in chunk])
        spec = np.fft.fft2(multislice(psi0, potential, setup.sigma, setup.prop))
        for p, sp in zip(chunk, spec):
            out[p] = sp
    return out


def plain_image(setup: Setup, potential: np.ndarray, probes=None, batch: int = 16) -> np.ndarray:
    """Plain multislice STEM image: every probe propagated directly (Sec. 3.1 steps 1-3).

    Returns float64 [n_det][Py][Px]; entries for probes not in ``probes`` (a list of (a, b)
    scan indices, default all) are NaN."""
    img = np.full((len(setup.detectors), setup.Py, setup.Px), np.nan)
    if probes is None:
        probes = [(a, b) for b in range(setup.Py) for a in range(setup.Px)]
    for (a, b), sp in plain_exit_spectra(setup, potential, probes, batch).items():
        img[:, b, a] = ph.detector_values(sp, setup.masks)
    return img


def exit_spectrum_at(setup: Setup, potential: np.ndarray, psi0: np.ndarray) -> np.ndarray:
    """DFT of the exit wave of initial wave psi0 (Y, X)."""
    return np.fft.fft2(multislice(psi0, potential, setup.sigma, setup.prop))
