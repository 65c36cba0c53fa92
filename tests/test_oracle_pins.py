"""Pins of the FP64 oracle against values the paper prints, closed forms, invariants and
brute force. None of these recompute the oracle's own formula as its expected value."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import physics as ph
from oracle import costs
from oracle.dft import dft2
from oracle.lma import LMA, Lattice, least_squares, recompute_sets, translate_wave
from oracle.multislice import Setup, multislice, plain_image
from oracle.partition import multislice_calls, union
from tests._cases import rel_l2


def _setup(nx=32, ny=32, lx=6.4, ly=6.4, kv=200.0, dz=2.0, bandlimit=2 / 3, alpha=0.02,
           defocus=0.0, cs=0.0, scan=(4, 4), detectors=((0.0, 0.015), (0.016, 0.04), (0.041, 0.2))):
    return Setup(nx, ny, lx, ly, ph.electron_wavelength(kv), ph.interaction_constant(kv), dz,
                 bandlimit, alpha, defocus, cs, scan, detectors)


# ---------------------------------------------------------------------------------------
# constants: values printed in the paper, and an independent SI route
# ---------------------------------------------------------------------------------------
def test_wavelength_matches_printed_value():
    # Fig. 6 / 7 / 8 captions: lambda = 0.0250793 A at 200 kV
    assert abs(ph.electron_wavelength(200.0) - 0.0250793) < 5e-8


def test_gaussian_width_matches_printed_value():
    # Sec. 4.2.3 Gaussians: sigma = lambda / (2 alpha_max) printed as 0.482 A for 26 mrad
    assert round(ph.electron_wavelength(200.0) / (2 * 0.026), 3) == 0.482


def test_gaussian_input_wave_spectrum_closed_form():
    # the Fourier transform of exp(-|x|^2 / (2 s^2)) is proportional to exp(-2 pi^2 s^2 |k|^2);
    # sampled on a grid much finer than s in a cell much larger than s, the DFT of the samples
    # agrees with it (aliasing and wrap-around far below 1e-12); non-square grid and cell
    nx, ny, lx, ly, s = 96, 64, 12.0, 9.6, 0.6
    got = ph.gaussian_spectrum(nx, ny, lx, ly, s)
    kx = np.fft.fftfreq(nx, d=lx / nx)[None, :]
    ky = np.fft.fftfreq(ny, d=ly / ny)[:, None]
    want = np.exp(-2 * np.pi ** 2 * s * s * (kx ** 2 + ky ** 2))
    want = want * np.sqrt(nx * ny / (np.abs(want) ** 2).sum())
    assert rel_l2(got, want) < 1e-12
    # centred at the origin: real spectrum; unit norm in real space
    assert np.abs(got.imag).max() < 1e-12 * np.abs(got).max()
    assert abs(np.linalg.norm(np.fft.ifft2(got)) - 1.0) < 1e-12


def test_interaction_constant_si_route():
    # sigma = 2 pi m e lambda / h^2 with the relativistic mass, in SI, then per V*Angstrom
    m0, e, h, c = 9.1093837015e-31, 1.602176634e-19, 6.62607015e-34, 299792458.0
    for kv in (100.0, 200.0, 300.0):
        V = kv * 1e3
        m = m0 * (1 + e * V / (m0 * c * c))
        lam = h / math.sqrt(2 * m0 * e * V * (1 + e * V / (2 * m0 * c * c)))
        sig_si = 2 * math.pi * m * e * lam / h ** 2          # rad / (V m)
        assert abs(lam * 1e10 - ph.electron_wavelength(kv)) / (lam * 1e10) < 1e-7
        assert abs(sig_si * 1e-10 - ph.interaction_constant(kv)) / (sig_si * 1e-10) < 1e-6


# ---------------------------------------------------------------------------------------
# FFT step against the DFT definition (brute force)
# ---------------------------------------------------------------------------------------
def test_slice_step_matches_bruteforce_dft():
    rng = np.random.default_rng(1)
    st = _setup(nx=6, ny=4, lx=1.3, ly=0.9, bandlimit=2.0)
    v = rng.uniform(0, 30, size=(1, 4, 6)).astype(np.float32)
    psi0 = rng.standard_normal((4, 6)) + 1j * rng.standard_normal((4, 6))
    got = multislice(psi0, v, st.sigma, st.prop)
    t = np.exp(1j * st.sigma * v[0].astype(np.float64))
    spec = np.array(dft2((t * psi0).tolist()))
    want = np.array(dft2((st.prop * spec).tolist(), inverse=True))
    assert rel_l2(got, want) < 1e-13


def test_fft_parseval_and_delta():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((5, 7)) + 1j * rng.standard_normal((5, 7))
    A = np.array(dft2(a.tolist()))
    assert abs((np.abs(A) ** 2).sum() - a.size * (np.abs(a) ** 2).sum()) < 1e-10
    d = np.zeros((4, 4))
    d[0, 0] = 1
    assert np.allclose(np.array(dft2(d.tolist())), 1.0)


# ---------------------------------------------------------------------------------------
# propagator: sign and scale by the Gaussian closed form; composition
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("nslices,dz", [(1, 50.0), (4, 25.0)])
def test_fresnel_gaussian_closed_form(nslices, dz):
    # exp(-x^2/(2 a^2) - y^2/(2 b^2)) propagated over z in free space becomes
    # prod over axes of (s0/s) exp(-r^2/(2 s^2)) with s^2 = s0^2 + i lambda z / (2 pi).
    # Non-square grid and cell so that a swapped kx/ky would fail.
    nx, ny, lx, ly = 96, 64, 19.2, 12.8
    st = _setup(nx=nx, ny=ny, lx=lx, ly=ly, bandlimit=1.0)
    lam = st.wavelength
    z = nslices * dz
    st = Setup(nx, ny, lx, ly, lam, st.sigma, dz, 1.0, 0.02, 0.0, 0.0, (1, 1), [(0, 1)])
    x = (np.arange(nx) - nx // 2) * (lx / nx)
    y = (np.arange(ny) - ny // 2) * (ly / ny)
    X, Y = np.meshgrid(x, y)
    a0, b0 = 1.1, 0.8
    psi0 = np.exp(-X ** 2 / (2 * a0 ** 2) - Y ** 2 / (2 * b0 ** 2))
    got = multislice(psi0, np.zeros((nslices, ny, nx), np.float32), st.sigma, st.prop)
    sa2 = a0 ** 2 + 1j * lam * z / (2 * np.pi)
    sb2 = b0 ** 2 + 1j * lam * z / (2 * np.pi)
    want = (a0 / np.sqrt(sa2)) * (b0 / np.sqrt(sb2)) * np.exp(-X ** 2 / (2 * sa2) - Y ** 2 / (2 * sb2))
    assert rel_l2(got, want) < 1e-10
    # the opposite sign convention is far off
    wrong = (a0 / np.sqrt(np.conj(sa2))) * (b0 / np.sqrt(np.conj(sb2))) * np.exp(
        -X ** 2 / (2 * np.conj(sa2)) - Y ** 2 / (2 * np.conj(sb2)))
    assert rel_l2(got, wrong) > 1e-2


def test_propagator_composition_two_dz_equals_2dz():
    rng = np.random.default_rng(3)
    st1 = _setup(nx=40, ny=48, lx=4.0, ly=5.6, dz=1.5)
    st2 = _setup(nx=40, ny=48, lx=4.0, ly=5.6, dz=3.0)
    psi0 = rng.standard_normal((48, 40)) + 1j * rng.standard_normal((48, 40))
    two = multislice(psi0, np.zeros((2, 48, 40), np.float32), st1.sigma, st1.prop)
    one = multislice(psi0, np.zeros((1, 48, 40), np.float32), st2.sigma, st2.prop)
    assert rel_l2(two, one) < 1e-13


def test_defocus_equals_free_propagation():
    # eq. aberration_function and the propagator agree: an in-focus probe propagated over z
    # in vacuum equals the probe with focus Z = -z (both band-limited identically).
    z = 40.0
    st0 = _setup(nx=64, ny=64, lx=12.8, ly=12.8, dz=z, defocus=0.0, bandlimit=1.0)
    stz = _setup(nx=64, ny=64, lx=12.8, ly=12.8, dz=z, defocus=-z, bandlimit=1.0)
    psi = multislice(st0.probe(0, 0), np.zeros((1, 64, 64), np.float32), st0.sigma, st0.prop)
    assert rel_l2(psi, stz.probe(0, 0)) < 1e-12


def test_aberration_stationary_phase_centroid():
    # eq. aberration_function through its physical effect: a wave packet A(k) exp(-i chi(k))
    # with a narrow real A around k0 is centred at <x> = <grad chi> / (2 pi) (the position
    # operator is i/(2 pi) d/dk in Fourier space; the A A' term integrates to zero). With
    # chi = 1/2 pi C_s lambda^3 |k|^4 - pi Z lambda |k|^2 the gradient over 2 pi is
    # C_s lambda^3 |k|^2 k - Z lambda k, averaged here with the weights |A|^2. A wrong
    # factor or power in the C_s term, or a wrong sign, moves the centroid by Angstroms.
    nx = ny = 512
    lx = ly = 160.0
    lam = 0.0250793
    k0, s = np.array([0.5, 0.2]), 0.04
    kx, ky, k2 = ph.k_grid(nx, ny, lx, ly)
    amp = np.exp(-((kx - k0[0]) ** 2 + (ky - k0[1]) ** 2) / (2 * s * s))
    w2 = amp ** 2 / (amp ** 2).sum()
    x = np.arange(nx) * (lx / nx)
    x = x - lx * np.round(x / lx)                  # minimum image about the origin
    y = np.arange(ny) * (ly / ny)
    y = y - ly * np.round(y / ly)
    for cs, z in ((1.0e7, 0.0), (1.0e7, 100.0), (-2.0e6, -50.0)):
        psi = np.fft.ifft2(amp * np.exp(-1j * ph.aberration(k2, lam, z, cs)))
        p = np.abs(psi) ** 2
        got = np.array([(p.sum(axis=0) * x).sum(), (p.sum(axis=1) * y).sum()]) / p.sum()
        want = np.array([(w2 * (cs * lam ** 3 * k2 * kg - z * lam * kg)).sum() for kg in (kx, ky)])
        assert np.abs(got - want).max() < 1e-6, (cs, z, got, want)
        assert np.abs(want).max() > 1.0              # the shift is many pixels (0.31 A)


# ---------------------------------------------------------------------------------------
# transmission, norm, linearity, equivariance
# ---------------------------------------------------------------------------------------
def test_transmission_zero_and_constant_potential():
    rng = np.random.default_rng(4)
    st = _setup()
    psi0 = st.probe(1, 2)
    free = multislice(psi0, np.zeros((3, 32, 32), np.float32), st.sigma, st.prop)
    v0 = 17.0
    const = multislice(psi0, np.full((3, 32, 32), v0, np.float32), st.sigma, st.prop)
    assert rel_l2(const, np.exp(1j * st.sigma * v0 * 3) * free) < 1e-13
    assert rel_l2(const, np.exp(-1j * st.sigma * v0 * 3) * free) > 1e-2
    t = ph.transmission(rng.uniform(0, 100, (32, 32)).astype(np.float32), st.sigma)
    assert np.allclose(np.abs(t), 1.0)


def test_norm_non_increasing_and_conserved_inside_band():
    rng = np.random.default_rng(5)
    st = _setup()
    v = rng.uniform(0, 60, (6, 32, 32)).astype(np.float32)
    psi = st.probe(0, 0)
    norms = [np.linalg.norm(psi)]
    for j in range(6):
        psi = multislice(psi, v[j:j + 1], st.sigma, st.prop)
        norms.append(np.linalg.norm(psi))
    assert abs(norms[0] - 1.0) < 1e-12
    assert all(b <= a + 1e-13 for a, b in zip(norms, norms[1:]))
    assert norms[-1] < norms[0] - 1e-6          # the band limit removed something
    free = multislice(st.probe(0, 0), np.zeros((6, 32, 32), np.float32), st.sigma, st.prop)
    assert abs(np.linalg.norm(free) - 1.0) < 1e-12


def test_linearity():
    rng = np.random.default_rng(6)
    st = _setup()
    v = rng.uniform(0, 60, (4, 32, 32)).astype(np.float32)
    u1, u2 = st.probe(0, 0), st.probe(1, 3)
    a, b = 0.3 - 1.2j, -0.7 + 0.4j
    lhs = multislice(a * u1 + b * u2, v, st.sigma, st.prop)
    rhs = a * multislice(u1, v, st.sigma, st.prop) + b * multislice(u2, v, st.sigma, st.prop)
    assert rel_l2(lhs, rhs) < 1e-13


def test_translation_equivariance_and_roll():
    rng = np.random.default_rng(7)
    st = _setup(nx=32, ny=32, lx=6.4, ly=6.4)
    patch = rng.uniform(0, 60, (3, 8, 8)).astype(np.float32)
    v = np.tile(patch, (1, 4, 4))                 # periodic with 8 px
    u = st.probe(0, 0)
    sx, sy = 8, 16
    shifted = translate_wave(st, st.spec0, (sx * st.lx / st.nx, sy * st.ly / st.ny))
    assert rel_l2(shifted, np.roll(u, (sy, sx), axis=(0, 1))) < 1e-12
    out = multislice(shifted, v, st.sigma, st.prop)
    ref = np.roll(multislice(u, v, st.sigma, st.prop), (sy, sx), axis=(0, 1))
    assert rel_l2(out, ref) < 1e-12


def test_probe_aperture_and_band_pixel_counts():
    # pixel counts of the aperture and band discs against their areas pi r^2 / dk^2
    st = _setup(nx=256, ny=256, lx=25.6, ly=25.6)
    dk = 1 / 25.6
    n_ap = (np.abs(st.spec0) > 0).sum()
    assert abs(n_ap - math.pi * (0.02 / st.wavelength / dk) ** 2) / n_ap < 0.03
    n_band = ph.band_mask(256, 256, 25.6, 25.6, 2 / 3).sum()
    assert abs(n_band - math.pi * ((2 / 3) * 5.0 / dk) ** 2) / n_band < 0.01
    assert abs(np.linalg.norm(st.probe(3, 1)) - 1.0) < 1e-12


# ---------------------------------------------------------------------------------------
# detector rings
# ---------------------------------------------------------------------------------------
def test_detector_rings_partition_the_band():
    rng = np.random.default_rng(8)
    st = _setup()
    spec = np.fft.fft2(rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32)))
    rings = [(0.0, 0.03), (0.03, 0.07), (0.07, 10.0)]
    masks = ph.ring_masks(32, 32, st.lx, st.ly, st.wavelength, st.bandlimit, rings)
    vals = ph.detector_values(spec, masks)
    band = ph.band_mask(32, 32, st.lx, st.ly, st.bandlimit) > 0
    assert abs(vals.sum() - (np.abs(spec[band]) ** 2).sum() / 1024) < 1e-9 * vals.sum()
    assert not np.any(masks[0] & masks[1]) and not np.any(masks[1] & masks[2])


def test_detector_ring_inner_edge_inclusive_outer_exclusive():
    lam = 0.5                                    # exactly representable
    masks = ph.ring_masks(8, 8, 1.0, 1.0, lam, 1.0, [(0.5, 1.0), (0.0, 0.5)])
    # frequency (kx, ky) = (1, 0) /A -> theta = 0.5 exactly: in [0.5, 1.0), not in [0, 0.5)
    assert masks[0][0, 1] and not masks[1][0, 1]


def test_4d_output_of_a_probe_in_vacuum_is_the_aperture():
    # no specimen: the exit spectrum is the probe's times unit-modulus propagators inside the
    # band, so the pattern is 1/|K| on the aperture pixels (unit incident intensity) and 0 off it
    from oracle.multislice import plain_exit_spectra
    st = _setup(nx=64, ny=64, lx=12.8, ly=12.8, defocus=40.0, cs=1e4, scan=(8, 8))
    spec = plain_exit_spectra(st, np.zeros((3, 64, 64), np.float32), [(3, 5)])[(3, 5)]
    pixels = st.masks.any(axis=0)
    pat = ph.detector_pattern(spec, pixels)
    ap = (np.abs(st.spec0) > 0)[pixels]
    n_ap = int((np.abs(st.spec0) > 0).sum())
    assert np.abs(pat[ap] - 1.0 / n_ap).max() < 1e-14
    assert np.abs(pat[~ap]).max() < 1e-28
    # pixel order: row-major over the frequency grid
    ky, kx = np.nonzero(pixels)
    assert np.array_equal(ky * 64 + kx, np.sort(ky * 64 + kx))


def test_3d_output_of_a_probe_in_vacuum_counts_aperture_pixels():
    # annulus a collects the aperture pixels with a w <= lambda |k| < (a + 1) w, each 1/|K|;
    # counted here pixel by pixel from the frequency definition k_m = m / l (m in FFT order)
    from oracle.multislice import plain_exit_spectra
    st = _setup(nx=64, ny=64, lx=12.8, ly=12.8, scan=(8, 8), detectors=((0.0, 0.2),))
    spec = plain_exit_spectra(st, np.zeros((2, 64, 64), np.float32), [(0, 0)])[(0, 0)]
    pixels = st.masks.any(axis=0)
    w, nb = 0.0025, 10
    got = ph.annulus_values(spec, st.lx, st.ly, st.wavelength, w, nb, pixels)
    counts = [0] * nb
    n_ap = 0
    for my in range(64):
        for mx in range(64):
            fx = (mx if mx < 32 else mx - 64) / 12.8
            fy = (my if my < 32 else my - 64) / 12.8
            if (st.wavelength ** 2) * (fx * fx + fy * fy) < 0.02 ** 2:
                n_ap += 1
                a = math.floor(st.wavelength * math.sqrt(fx * fx + fy * fy) / w)
                if a < nb:
                    counts[a] += 1
    assert np.abs(got - np.array(counts) / n_ap).max() < 1e-14
    assert abs(got.sum() - 1.0) < 1e-12          # 10 x 2.5 mrad cover the 20 mrad aperture


def test_3d_and_4d_outputs_agree_with_the_2d_rings():
    # a 2-D ring [w, 2w) equals annulus 1 of width w over the same pixels, and the sum of a
    # ring's 4-D pattern
    rng = np.random.default_rng(12)
    st = _setup(detectors=((0.01, 0.02),))
    spec = np.fft.fft2(rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32)))
    pixels = st.masks.any(axis=0)
    ring = ph.detector_values(spec, st.masks)[0]
    ann = ph.annulus_values(spec, st.lx, st.ly, st.wavelength, 0.01, 4, pixels)
    assert abs(ann[1] - ring) < 1e-12 * ring and ann[0] == 0 and ann[2] == 0 and ann[3] == 0
    assert abs(ph.detector_pattern(spec, pixels).sum() - ring) < 1e-12 * ring


# ---------------------------------------------------------------------------------------
# windowed translate propagation (option (ii) of Sec. 4.2.1)
# ---------------------------------------------------------------------------------------
def _windowed_case(window):
    st = _setup(scan=(8, 8))
    lat = Lattice(st, (8, 8), 1, (0, 0), 4)           # translates every 4 px, on pixels
    return st, lat, LMA(st, lat, window=window)


def test_window_of_the_whole_cell_is_plain_propagation():
    # a window as large as the cell is the cell itself, rolled: same exit spectra
    rng = np.random.default_rng(21)
    v = rng.uniform(0, 40, (3, 32, 32)).astype(np.float32)
    st, lat, lw = _windowed_case((32, 32))
    lf = LMA(st, lat)
    ts = [(0, 0), (3, 5), (7, 7)]
    bw, bf = lw.propagate(v, ts), lf.propagate(v, ts)
    for t in ts:
        assert rel_l2(bw[t], bf[t]) < 1e-12


def test_windowed_translate_sees_only_its_window():
    rng = np.random.default_rng(22)
    v = rng.uniform(0, 40, (3, 32, 32)).astype(np.float32)
    st, lat, lw = _windowed_case((16, 8))
    t = (2, 5)                                          # at pixel (8, 20): window x 0..15, y 16..23
    cx, cy = lw.window_origin(*t)
    assert (cx, cy) == (0, 16)
    base = lw.propagate(v, [t])[t]
    out = v.copy()
    out[:, 10, 20] += 30.0                              # outside the window
    out[:, 24, 3] += 30.0
    assert np.array_equal(lw.propagate(out, [t])[t], base)
    corner = v.copy()
    corner[1, 23, 15] += 30.0                           # last row and column of the window
    assert rel_l2(lw.propagate(corner, [t])[t], base) > 1e-6
    centre = v.copy()
    centre[1, 20, 8] += 30.0
    assert rel_l2(lw.propagate(centre, [t])[t], base) > 1e-3


def test_windowed_translation_covariance():
    # rolling the specimen by one translate spacing moves the window with the translate: the
    # exit spectrum of the next translate is the modulated spectrum of this one
    rng = np.random.default_rng(23)
    v = rng.uniform(0, 40, (3, 32, 32)).astype(np.float32)
    st, lat, lw = _windowed_case((16, 16))
    a = lw.propagate(v, [(3, 1)])[(3, 1)]
    b = lw.propagate(np.roll(v, 4, axis=2), [(4, 1)])[(4, 1)]
    kx = ph.freqs(32, st.lx)[None, :]
    assert rel_l2(b, a * np.exp(-2j * np.pi * kx * (4 * st.lx / 32))) < 1e-12


# ---------------------------------------------------------------------------------------
# LMA: special cases, error bound, staircase, coefficient reuse
# ---------------------------------------------------------------------------------------
def test_lma_reduces_to_plain_multislice():
    # u = psi_0, I = P, f = 1, L = 1 gives back the standard algorithm (Sec. 4.2.3)
    rng = np.random.default_rng(9)
    st = _setup(scan=(4, 4))
    lat = Lattice(st, (4, 4), 1, (0, 0), 1)
    lma = LMA(st, lat)
    assert abs(lma.alpha[(0, 0)][0] - 1.0) < 1e-12
    v = rng.uniform(0, 50, (3, 32, 32)).astype(np.float32)
    probes = [(0, 0), (1, 2), (3, 3)]
    assert rel_l2(lma.image(v, probes)[:, [0, 2, 3], [0, 1, 3]],
                  plain_image(st, v, probes)[:, [0, 2, 3], [0, 1, 3]]) < 1e-12


def test_pixel_input_waves_with_every_translate_are_exact():
    # Sec. 4.3: pixel input waves (u a delta, I the pixel lattice) with L = all translates
    # represent any probe exactly, so LMA reproduces plain multislice
    rng = np.random.default_rng(21)
    st = _setup(nx=8, ny=8, lx=1.6, ly=1.6, scan=(2, 2), alpha=0.03)
    lat = Lattice(st, (8, 8), 1, (0, 0), 64)
    delta = np.ones((8, 8), dtype=np.complex128)          # DFT of a delta at the origin
    lma = LMA(st, lat, spec_u=delta)
    assert max(lma.residual.values()) < 1e-12
    v = rng.uniform(0, 50, (3, 8, 8)).astype(np.float32)
    probes = [(0, 0), (1, 0), (1, 1)]
    got = lma.image(v, probes)[:, [0, 0, 1], [0, 1, 1]]
    want = plain_image(st, v, probes)[:, [0, 0, 1], [0, 1, 1]]
    assert rel_l2(got, want) < 1e-10


def test_lma_case1_without_offset_is_exact():
    # R_f = 2 P and zero offset: every probe sits on a translate, alpha is a delta
    st = _setup(scan=(4, 4))
    lat = Lattice(st, (8, 8), 1, (0, 0), 5)
    al, nbr, res = least_squares(st, lat, st.spec0, 0, 0)
    assert res < 1e-12
    assert abs(al[0] - 1) < 1e-10 and np.all(np.abs(al[1:]) < 1e-10)


def test_lma_exit_error_bounded_by_probe_residual():
    # propagation is linear and each slice a contraction, so the LMA exit-wave error is at
    # most the residual of the initial approximation
    rng = np.random.default_rng(10)
    st = _setup(scan=(4, 4))
    lat = Lattice(st, (8, 8), 1, (0.5, 0.5), 12)
    lma = LMA(st, lat)
    v = rng.uniform(0, 50, (4, 32, 32)).astype(np.float32)
    for a, b in [(0, 0), (2, 1)]:
        approx = lma.approximant(a, b)
        exact = st.probe(a, b)
        e_init = np.linalg.norm(approx - exact)
        e_exit = np.linalg.norm(multislice(approx, v, st.sigma, st.prop) - multislice(exact, v, st.sigma, st.prop))
        assert e_exit <= e_init * (1 + 1e-9)
        assert e_init > 1e-4                         # non-trivial case


@pytest.mark.parametrize("R,f,offset,L,probe,defocus", [((8, 8), 1, (0.5, 0.5), 12, (2, 1), 30.0),
                                                          ((16, 16), 2, (0.5, 0.5), 9, (1, 2), -40.0),
                                                          ((8, 8), 1, (0.25, 0.5), 16, (3, 0), 0.0)])
def test_least_squares_coefficients_solve_the_normal_equations(R, f, offset, L, probe, defocus):
    # Sec. 4.2.2: alpha minimises || psi_p - sum_j alpha_j u_{i_j} ||. The minimiser is the
    # alpha whose residual is orthogonal to every translate of the set (B^H r = 0), and it is
    # unique when B has full column rank, so these sets fix the coefficients themselves. A
    # defocused probe is complex, so a conjugation slip cannot pass
    st = _setup(scan=(8, 8), defocus=defocus)
    lat = Lattice(st, R, f, offset, L)
    al, nbr, res = least_squares(st, lat, st.spec0, *probe)
    B = np.stack([translate_wave(st, st.spec0, lat.translate_position(ta, tb)).ravel() for ta, tb in nbr], axis=1)
    psi = st.probe(*probe).ravel()
    r = psi - B @ al
    sv = np.linalg.svd(B, compute_uv=False)
    assert sv[-1] > 1e-3 * sv[0]                     # full column rank, well conditioned
    assert np.abs(B.conj().T @ r).max() < 1e-12 * sv[0] * np.linalg.norm(psi)
    assert res == pytest.approx(np.linalg.norm(r) / np.linalg.norm(psi), rel=1e-12)
    assert 1e-6 < res < 1                            # a true approximation, not an exact one


def test_residual_staircase_non_increasing_in_L():
    st = _setup(nx=64, ny=64, lx=12.8, ly=12.8, scan=(16, 16))
    res = []
    for L in (1, 4, 8, 12, 16, 24, 36):
        lat = Lattice(st, (32, 32), 1, (0.5, 0.5), L)
        res.append(least_squares(st, lat, st.spec0, 0, 0)[2])
    assert all(b <= a + 1e-12 for a, b in zip(res, res[1:]))
    assert res[-1] < 0.1 * res[0]


def test_coefficient_reuse_case2_same_error_for_shifted_probe():
    # Case 2 (P = c R_f): probes a and a + c share coefficients (eq. lma_approximation_exit2)
    st = _setup(nx=32, ny=32, lx=6.4, ly=6.4, scan=(8, 8))
    lat = Lattice(st, (4, 4), 1, (0.5, 0.5), 9)
    assert (lat.ncls_x, lat.ncls_y) == (2, 2)
    lma = LMA(st, lat)
    for a, b in [(2, 4), (3, 5), (5, 2)]:
        al_direct, nbr, res = least_squares(st, lat, st.spec0, a, b)
        approx = lma.approximant(a, b)
        assert rel_l2(approx, st.probe(a, b)) == pytest.approx(res, rel=1e-8)
        assert lma.residual[lat.coefficient_class(a, b)] == pytest.approx(res, rel=1e-8)


def test_nearest_translates_complete_first_shell():
    # offset (1/2, 1/2) of the spacing, Case 1 with c = 1: the 4 nearest are the four
    # translates at (+-1/2, +-1/2) spacing from the probe
    st = _setup(nx=32, ny=32, lx=6.4, ly=6.4, scan=(8, 8))
    lat = Lattice(st, (8, 8), 1, (0.5, 0.5), 4)
    got = set(lat.nearest(3, 5))
    assert got == {(3, 5), (2, 5), (3, 4), (2, 4)}


# ---------------------------------------------------------------------------------------
# lattice counts, partition counts and the cost model printed in the paper
# ---------------------------------------------------------------------------------------
def test_printed_translate_and_probe_counts():
    # Sec. 4.2.6: (Px, Py) = (424, 400), I = P + p/2, f = 2 -> |I_f| = 212 * 200 = 42400
    st = Setup(16, 16, 84.536, 79.941, 0.0250793, 7e-4, 2.0, 2 / 3, 0.026, 100.0, -2000.0,
               (424, 400), [(0.0, 0.015)])
    lat = Lattice(st, (424, 400), 2, (0.5, 0.5), 59)
    assert lat.n_translates == 42400 and st.Px * st.Py == 169600
    assert (lat.ncls_x, lat.ncls_y) == (2, 2)


def _partition_example_sets(L):
    # Fig. lmastrategy_examples: X = 512, P = 158, l = 31.208 A, I = P + p/2, f = 2, 48 x 48
    # sub-image. Neighbour lists of the four class representatives are computed by the
    # oracle and shifted to every probe (the shift rule is checked by the Case 2 test above).
    st = Setup(8, 8, 31.208, 31.208, 0.0250793, 7e-4, 2.0, 2 / 3, 0.026, 100.0, -2000.0,
               (158, 158), [(0.0, 0.015)])
    lat = Lattice(st, (158, 158), 2, (0.5, 0.5), L)
    reps = {(cx, cy): lat.nearest(cx, cy) for cx in (0, 1) for cy in (0, 1)}
    sets = {}
    for b in range(48):
        for a in range(48):
            A, B = a + 1, b + 1                  # the sub-image starts at an odd index
            sets[(a, b)] = [((ta + A // 2) % lat.Rfx, (tb + B // 2) % lat.Rfy)
                            for ta, tb in reps[(A % 2, B % 2)]]
    return sets


@pytest.mark.slow
def test_printed_minimum_multislice_calls_L75():
    sets = _partition_example_sets(75)
    assert len(union(sets, sets.keys())) == 1077
    # full-width strips reach the minimum (the paper's second example, row strategy)
    strips = [[(a, b) for a in range(48)] for b in range(48)]
    assert multislice_calls(sets, strips) == 1077
    assert multislice_calls(sets, [list(sets.keys())]) == 1077


def test_rectangle_partition_second_example():
    # Fig. lmastrategy_examples, bottom row (L = 51): the rectangle strategy keeps about a
    # quarter of the trivial strategy's multislice solutions (P_1 = P, T = |I_{f,P,L}|) in
    # memory, yet makes exactly as many multislice calls, with l = 48 rectangles
    from oracle.partition import rectangles, tiling
    sets = _partition_example_sets(51)
    region = (0, 0, 48, 48)
    U = len(union(sets, sets.keys()))               # the paper prints 953; our tie rule gives 955
    assert abs(U - 953) <= 2
    M = -(-U // 4)
    parts = rectangles(sets, region, M)
    assert len(parts) == 48
    assert multislice_calls(sets, parts) == U
    peak = max(len(union(sets, q)) for q in parts)
    assert peak <= M and peak > 0.2 * U
    # no partition beats the trivial strategy's count, which is reached with M = |I_{f,P,L}|;
    # every partition covers the sub-image once, its parts within M
    for m in (60, 100, 170, M, 300, 600, U):
        parts = rectangles(sets, region, m)
        cover = [p for q in parts for p in q]
        assert sorted(cover) == sorted(sets.keys())
        assert all(len(union(sets, q)) <= m for q in parts)
        assert multislice_calls(sets, parts) >= U
    assert len(rectangles(sets, region, U)) == 1
    # the widest rectangles first: at M no wider tiling fits, and the chosen height is the
    # tallest that fits at that width
    parts = rectangles(sets, region, M)
    h = max(b for _, b in parts[0]) + 1
    assert any(len(union(sets, q)) > M for q in tiling(region, 48, h + 1))


# ---------------------------------------------------------------------------------------
# trigonometric input waves (Sec. 2, Sec. 4.2.3)
# ---------------------------------------------------------------------------------------
def test_trig_transform_inverse_factor():
    # M M^-1 = I with the factor 1 / (2n + 1); the printed 1 / (2n + 1)^2 leaves I / (2n + 1)
    from oracle.lma import trig_transform
    for n in (1, 3, 7, 10):
        M, Minv = trig_transform(n)
        assert np.abs(M @ Minv - np.eye(2 * n + 1)).max() < 1e-13
        assert np.abs(Minv @ M - np.eye(2 * n + 1)).max() < 1e-13
        printed = Minv / (2 * n + 1)
        assert np.abs((2 * n + 1) * (M @ printed) - np.eye(2 * n + 1)).max() < 1e-13


def test_trigpoly_wave_is_the_shifted_dirichlet_sum():
    # cos(k theta) = (e^{ik theta} + e^{-ik theta}) / 2 with theta = pi / (2n + 2) turns eq. rauhut
    # into phi_n(t) = (D_n(t + theta) + D_n(t - theta)) / 2, D_n(x) = sin((n + 1/2) x) / sin(x / 2)
    # (the Dirichlet kernel); the oracle's u is the product of two such functions
    n_x, n_y, nx, ny = 6, 4, 48, 40
    u = np.fft.ifft2(ph.trigpoly_spectrum(nx, ny, 9.6, 8.0, n_x, n_y))

    def dirichlet_form(n, npts):
        th = np.pi / (2 * n + 2)
        t = 2 * np.pi * np.arange(npts) / npts
        def d(x):
            s2 = np.sin(x / 2)
            small = np.abs(s2) < 1e-12                 # x = 0 mod 2 pi: D_n = 2n + 1
            return np.where(small, 2 * n + 1, np.sin((n + 0.5) * x) / np.where(small, 1.0, s2))
        return 0.5 * (d(t + th) + d(t - th))
    want = dirichlet_form(n_y, ny)[:, None] * dirichlet_form(n_x, nx)[None, :]
    want = want / np.linalg.norm(want)
    assert rel_l2(u, want) < 1e-12
    assert np.abs(u.imag).max() < 1e-14               # real and even, peaked at the origin
    assert np.argmax(np.abs(u)) == 0


def test_trigpoly_basis_represents_every_probe_exactly():
    # the tensor phi_n over the full (2n + 1)^2 lattice spans K_+, which holds the aperture:
    # every probe, wherever it sits, is an exact combination of the translates, with the closed
    # form M^-1 coefficients; the least-squares solver finds the same coefficients
    from oracle.lma import trig_coefficients
    st = _setup(nx=64, ny=64, lx=12.8, ly=12.8, scan=(42, 42))
    n = 10                                            # lambda |k| < 20 mrad needs |m| <= 10 at 12.8 A
    assert int(np.floor(st.alpha_max / st.wavelength * st.lx)) == n
    su = ph.trigpoly_spectrum(64, 64, 12.8, 12.8, n, n)
    for offset in ((0, 0), (0.5, 0.5)):
        lat = Lattice(st, (21, 21), 1, offset, 441)
        for a, b in ((0, 0), (1, 0), (5, 7), (13, 30)):
            al = trig_coefficients(st, lat, su, a, b)
            approx = sum(al[tb, ta] * translate_wave(st, su, lat.translate_position(ta, tb))
                         for tb in range(21) for ta in range(21))
            assert rel_l2(approx, st.probe(a, b)) < 1e-12
        al_ls, nbr, res = least_squares(st, lat, su, 1, 0)
        full = trig_coefficients(st, lat, su, 1, 0)
        al_cf = np.array([full[tb, ta] for ta, tb in nbr])
        assert res < 1e-12 and np.abs(al_cf - al_ls).max() < 1e-9 * np.abs(al_ls).max()
    # too low a degree: the coefficients project the probe onto K_+ (its error is the energy
    # outside K_+)
    st15 = _setup(nx=64, ny=64, lx=12.8, ly=12.8, scan=(15, 15))
    lat = Lattice(st15, (15, 15), 1, (0, 0), 225)
    su7 = ph.trigpoly_spectrum(64, 64, 12.8, 12.8, 7, 7)
    om = LMA(st15, lat, spec_u=su7, coefficients="trigpoly")
    spec = st.spec0
    k = np.fft.fftfreq(64, 1 / 64)
    outside = (np.abs(k)[None, :] > 7) | (np.abs(k)[:, None] > 7)
    want = np.sqrt((np.abs(spec[outside]) ** 2).sum() / (np.abs(spec) ** 2).sum())
    assert abs(om.residual[(0, 0)] - want) < 1e-12


def test_cost_model_log_base_two():
    # Sec. 4.2.1: at 2048^2 with a 25 x 25 kernel, real-space propagation wins iff f >= 4
    assert math.ceil(costs.realspace_breakeven_f(2048, 2048, 25, 25)) == 4
    assert math.ceil(costs.realspace_breakeven_f(2048, 2048, 25, 25, log=math.log)) != 4
    assert costs.t_multislice(1, 4, 4) == 2 * 16 + 2 * 16 * 4


def test_recompute_sets_distance_rule():
    # Sec. 4.2.6 selection (reading: Euclidean distance from a translate's centre to the span of
    # edited pixel positions, periodic, inclusive): checked on a single edited pixel whose
    # distances to the translates are known exactly
    st = _setup(scan=(8, 8))                             # 32 px over 6.4 A: 0.2 A per pixel
    lat = Lattice(st, (8, 8), 1, (0, 0), 4)              # translates every 4 px = 0.8 A, at (0, 0) + k
    box = (8, 8, 9, 9)                                   # pixel (8, 8) = (1.6, 1.6) A = translate (2, 2)
    R0, _ = recompute_sets(lat, box, 1e-9)
    assert R0 == {(2, 2)}
    # the four neighbours at 0.8 A (the cell length 6.4 is a binary double, so the distances
    # are 0.8 to within 1e-15, and rho is read to 1/2^24, hence the tolerance), the diagonals at 1.13 A
    R1, _ = recompute_sets(lat, box, 0.8 + 1e-6)
    assert R1 == {(2, 2), (1, 2), (3, 2), (2, 1), (2, 3)}
    R2, _ = recompute_sets(lat, box, 0.8 * math.sqrt(2) - 1e-6)
    assert R2 == R1
    R2b, _ = recompute_sets(lat, box, 0.8 * math.sqrt(2) + 1e-6)
    assert R2b == R1 | {(1, 1), (3, 1), (1, 3), (3, 3)}
    # periodic: a box at the cell's last pixel reaches translate (0, 0) across the edge
    R3, _ = recompute_sets(lat, (31, 31, 32, 32), 0.2 * math.sqrt(2) + 1e-6)
    assert (0, 0) in R3
    # every translate for rho <= 0; the probes are those whose neighbour sets meet R
    Rall, Pall = recompute_sets(lat, box, 0.0)
    assert len(Rall) == 64 and len(Pall) == 64
    _, P1 = recompute_sets(lat, box, 0.8 + 1e-6)
    assert P1 == {(a, b) for b in range(8) for a in range(8) if set(lat.nearest(a, b)) & R1}
    assert (2, 2) in P1 and (6, 6) not in P1


def test_phonon_average_linear():
    rng = np.random.default_rng(11)
    st = _setup(scan=(2, 2))
    vs = [rng.uniform(0, 50, (2, 32, 32)).astype(np.float32) for _ in range(3)]
    imgs = [plain_image(st, v) for v in vs]
    from oracle.lma import phonon_average
    avg = phonon_average(imgs)
    assert np.allclose(avg, (imgs[0] + imgs[1] + imgs[2]) / 3, rtol=1e-14)
    assert np.array_equal(phonon_average(imgs[:1]), imgs[0])
