"""Physics of the oracle: constants, grids, probe, transmission, propagator, detectors.

TEST INFRASTRUCTURE ONLY (see the package docstring). Everything is numpy float64 /
complex128.

DFT convention (the paper is silent): forward F(psi)[k] = sum_x psi[x] exp(-2 pi i k.x),
inverse with a 1/(XY) factor (numpy's convention). Frequencies are in FFT order:
k_m = m/l for m < X/2 and (m - X)/l otherwise, which is the paper's centred map g
(Sec. 4.1) up to an index shift.
"""
from __future__ import annotations

import numpy as np

HC_EV_A = 12398.4198      # h*c in eV*Angstrom
M0C2_EV = 510998.95       # electron rest energy in eV


def electron_wavelength(kv: float) -> float:
    """Relativistic electron wavelength in Angstrom, lambda = hc / sqrt(eV (2 m0 c^2 + eV)).

    Textbook formula; the paper prints lambda = 0.0250793 A for 200 kV (Fig. 6 caption)."""
    ev = kv * 1e3
    return HC_EV_A / np.sqrt(ev * (2.0 * M0C2_EV + ev))


def interaction_constant(kv: float) -> float:
    """Beam-sample interaction constant sigma in rad/(V*Angstrom) of eq. schroedinger_equation:
    sigma = 2 pi / (lambda V) * (m0 c^2 + eV) / (2 m0 c^2 + eV). The paper does not print it."""
    ev = kv * 1e3
    lam = electron_wavelength(kv)
    return 2.0 * np.pi / (lam * ev) * (M0C2_EV + ev) / (2.0 * M0C2_EV + ev)


def freqs(n: int, length: float) -> np.ndarray:
    """Spatial frequencies (1/Angstrom) of an n-point grid over ``length``, FFT order."""
    m = np.arange(n)
    m = np.where(m < (n + 1) // 2, m, m - n)
    return m.astype(np.float64) / length


def k_grid(nx: int, ny: int, lx: float, ly: float):
    """(kx, ky, k2) arrays of shape (ny, nx); k2 = kx*kx + ky*ky."""
    kx = freqs(nx, lx)[None, :] * np.ones((ny, 1))
    ky = freqs(ny, ly)[:, None] * np.ones((1, nx))
    return kx, ky, kx * kx + ky * ky


def aberration(k2: np.ndarray, wavelength: float, defocus: float, cs: float) -> np.ndarray:
    """chi(k) = 1/2 pi C_s lambda^3 |k|^4 - pi Z lambda |k|^2 (eq. aberration_function)."""
    return 0.5 * np.pi * cs * wavelength ** 3 * k2 * k2 - np.pi * defocus * wavelength * k2


def aperture(k2: np.ndarray, wavelength: float, alpha_max: float) -> np.ndarray:
    """A(k) = 1 iff lambda |k| < alpha_max, strict (eq. aperture_function).

    Tested as (lambda*lambda)*k2 < alpha_max*alpha_max in float64."""
    t2 = (wavelength * wavelength) * k2
    return (t2 < alpha_max * alpha_max).astype(np.float64)


def probe_spectrum(nx, ny, lx, ly, wavelength, alpha_max, defocus, cs) -> np.ndarray:
    """Fourier coefficients of the probe at the origin, exp(-i chi) A (eq. probe_wave_function),
    scaled so that the real-space probe has unit L2 norm: sum_x |psi|^2 = 1, i.e.
    sum_k |psi_hat|^2 = XY. (Reading: the paper does not normalise; unit norm makes detector
    values fractions of the incident intensity.)"""
    _, _, k2 = k_grid(nx, ny, lx, ly)
    a = aperture(k2, wavelength, alpha_max)
    spec = a * np.exp(-1j * aberration(k2, wavelength, defocus, cs))
    nk = a.sum()
    if nk == 0:
        raise ValueError("aperture contains no grid frequency")
    return spec * np.sqrt(nx * ny / nk)


def gaussian_spectrum(nx, ny, lx, ly, sigma: float) -> np.ndarray:
    """Input wave u = g_sigma(x) = exp(-|x|^2 / (2 sigma^2)) of Sec. 4.2.3 (Gaussians), centred
    at the origin of the periodic cell: sampled on the grid with minimum-image distances, then
    the DFT, scaled like the probe (sum_x |u|^2 = 1, so sum_k |u_hat|^2 = XY)."""
    x = np.arange(nx) * (lx / nx)
    y = np.arange(ny) * (ly / ny)
    x = x - lx * np.round(x / lx)
    y = y - ly * np.round(y / ly)
    g = np.exp(-(x[None, :] ** 2 + y[:, None] ** 2) / (2.0 * sigma * sigma))
    g = g / np.linalg.norm(g)
    return np.fft.fft2(g)


def trig_weights(n: int) -> np.ndarray:
    """cos(k pi / (2n + 2)) for k = -n..n: the weights of the localised trigonometric polynomial
    phi_n(t) = sum_k exp(i k t) cos(k pi / (2n + 2)) of eq. rauhut (index k + n)."""
    k = np.arange(-n, n + 1)
    return np.cos(k * np.pi / (2 * n + 2))


def trigpoly_spectrum(nx, ny, lx, ly, n_x: int, n_y: int) -> np.ndarray:
    """Input wave u(x, y) = phi_{n_x}(2 pi x / lx) phi_{n_y}(2 pi y / ly) of Sec. 2 / Sec. 4.2.3
    (the tensor product of localised trigonometric polynomials, eq. rauhut, with the cell as
    their period): phi_n evaluated at the grid points by its defining sum, the product taken,
    scaled to unit L2 norm like the probe, then the DFT (sum_k |u_hat|^2 = XY)."""
    def phi(n, npts, length):
        t = 2.0 * np.pi * np.arange(npts) * (length / npts) / length
        w = trig_weights(n)
        return np.array([np.sum(w * np.exp(1j * np.arange(-n, n + 1) * tt)) for tt in t])
    u = phi(n_y, ny, ly)[:, None] * phi(n_x, nx, lx)[None, :]
    u = u / np.linalg.norm(u)
    return np.fft.fft2(u)


def shift_spectrum(spec: np.ndarray, lx: float, ly: float, pos) -> np.ndarray:
    """Spectrum of f(. - pos): multiply by the modulation mu_{-pos}(k) = exp(-2 pi i k.pos)
    (Sec. 4.1, translations become modulations)."""
    ny, nx = spec.shape
    kx = freqs(nx, lx)[None, :]
    ky = freqs(ny, ly)[:, None]
    return spec * np.exp(-2j * np.pi * (kx * float(pos[0]) + ky * float(pos[1])))


def probe_wave(spec: np.ndarray, lx: float, ly: float, pos) -> np.ndarray:
    """Real-space probe psi_p^init = F^{-1}(exp(-i chi) A)(x - p) on the grid."""
    return np.fft.ifft2(shift_spectrum(spec, lx, ly, pos))


def band_radius(nx, ny, lx, ly, bandlimit: float) -> float:
    """k_bw = bandlimit * min(X/(2 lx), Y/(2 ly)) (reading of the 2/3-Nyquist band limit)."""
    return bandlimit * min(nx / (2.0 * lx), ny / (2.0 * ly))


def band_mask(nx, ny, lx, ly, bandlimit: float) -> np.ndarray:
    """1 where |k| < k_bw, strict; tested as k2 < kbw*kbw in float64."""
    _, _, k2 = k_grid(nx, ny, lx, ly)
    kbw = band_radius(nx, ny, lx, ly, bandlimit)
    return (k2 < kbw * kbw).astype(np.float64)


def propagator(nx, ny, lx, ly, wavelength, dz, bandlimit) -> np.ndarray:
    """Fourier-space Fresnel propagator exp(-i pi lambda eps |k|^2) times the band limit.

    The paper writes the real-space kernel q = (-i/(lambda eps)) exp(i pi (x^2+y^2)/(lambda eps))
    (Sec. 3.2); its Fourier transform, and equally the Laplacian term of eq.
    schroedinger_equation integrated over one slice (Delta -> -4 pi^2 |k|^2), is the factor
    used here. The band limit multiplies the propagator only (reading)."""
    _, _, k2 = k_grid(nx, ny, lx, ly)
    return np.exp(-1j * np.pi * wavelength * dz * k2) * band_mask(nx, ny, lx, ly, bandlimit)


def transmission(v_slice: np.ndarray, sigma: float) -> np.ndarray:
    """t = exp(i sigma v_eps) (Sec. 3.2), v in V*Angstrom (float32 input upcast to float64)."""
    return np.exp(1j * sigma * v_slice.astype(np.float64))


def ring_masks(nx, ny, lx, ly, wavelength, bandlimit, detectors) -> np.ndarray:
    """Boolean masks (n_det, ny, nx) of the 2-D STEM detectors (Sec. 3.1, step 3).

    Ring r is B_{outer} minus B_{inner} in scattering angle theta = lambda |k|: inner <= theta
    < outer, tested as inner^2 <= (lambda*lambda)*k2 < outer^2. Only frequencies inside the
    band limit can carry intensity; the mask is intersected with it.
    ``detectors`` is a sequence of (inner_rad, outer_rad)."""
    _, _, k2 = k_grid(nx, ny, lx, ly)
    t2 = (wavelength * wavelength) * k2
    band = band_mask(nx, ny, lx, ly, bandlimit) > 0
    out = np.zeros((len(detectors), ny, nx), dtype=bool)
    for r, (lo, hi) in enumerate(detectors):
        out[r] = (t2 >= lo * lo) & (t2 < hi * hi) & band
    return out


def detector_pattern(exit_spectrum: np.ndarray, pixels: np.ndarray) -> np.ndarray:
    """4-D STEM output of one exit wave (Sec. 3.1, step 3, pixelated detector): |F(psi_exit)|^2
    / (XY) at the pixels where the boolean (ny, nx) mask ``pixels`` holds, in row-major order."""
    ny, nx = exit_spectrum.shape
    return (np.abs(exit_spectrum) ** 2)[pixels] / (nx * ny)


def annulus_values(exit_spectrum: np.ndarray, lx: float, ly: float, wavelength: float, width: float,
                   nbins: int, pixels: np.ndarray) -> np.ndarray:
    """3-D STEM output of one exit wave (Sec. 3.1, step 3, many small annuli): for a = 0..nbins-1
    the sum of |F(psi_exit)|^2 / (XY) over the pixels of ``pixels`` whose scattering angle
    theta = lambda |k| satisfies a * width <= theta < (a + 1) * width (annulus index taken as
    floor(theta / width) in float64)."""
    ny, nx = exit_spectrum.shape
    kx, ky, _ = k_grid(nx, ny, lx, ly)
    a = np.floor(wavelength * np.sqrt(kx * kx + ky * ky) / width)
    inten = np.abs(exit_spectrum) ** 2 / (nx * ny)
    return np.array([inten[pixels & (a == b)].sum() for b in range(nbins)])


def detector_values(exit_spectrum: np.ndarray, masks: np.ndarray) -> np.ndarray:
    """I_r = sum over ring r of |F(psi_exit)|^2 / (XY) for one exit wave (its DFT given)."""
    ny, nx = exit_spectrum.shape
    inten = np.abs(exit_spectrum) ** 2
    return np.array([inten[m].sum() for m in masks]) / (nx * ny)
