"""Builders shared by the tests: oracle set-ups from the named workloads, and small cases."""
from __future__ import annotations

import numpy as np

from oracle import physics as ph
from oracle.multislice import Setup
from oracle.lma import Lattice
from synth import WORKLOADS


def det_rad(w):
    return [(lo * 1e-3, hi * 1e-3) for _, lo, hi in w.detectors]


def oracle_setup(w, scan=None, detectors=None, **over):
    lam = ph.electron_wavelength(w.kv)
    sig = ph.interaction_constant(w.kv)
    kw = dict(nx=w.nx, ny=w.ny, lx=w.lx, ly=w.ly, wavelength=lam, sigma=sig, dz=w.dz,
              bandlimit=w.bandlimit, alpha_max=w.alpha_mrad * 1e-3, defocus=w.defocus, cs=w.cs,
              scan=scan or w.scan, detectors=detectors or det_rad(w))
    kw.update(over)
    return Setup(**kw)


def oracle_lattice(w, setup, L=None, f=1, R=None, offset=None):
    if R is None:
        R = (w.nx // w.basis_px * f, w.ny // w.basis_px * f)
    return Lattice(setup, R, f, offset if offset is not None else w.offset_frac, L or w.L)


def small_workload(name="tiny"):
    return WORKLOADS[name]


def random_wave(rng, ny, nx):
    return rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))


def rel_l2(a, b):
    """||a - b|| / ||b||; for an all-zero b, 0 if a is zero too, else inf."""
    a = np.asarray(a)
    b = np.asarray(b)
    d, n = np.linalg.norm((a - b).ravel()), np.linalg.norm(b.ravel())
    if n == 0.0:
        return 0.0 if d == 0.0 else float("inf")
    return float(d / n)


def longest_zero_run(zero):
    """(start, end) of the longest run of True in a 1-D boolean sequence ((0, 0) if none)."""
    best, x, n = (0, 0), 0, len(zero)
    while x < n:
        if not zero[x]:
            x += 1
            continue
        e = x
        while e < n and zero[e]:
            e += 1
        if e - x > best[1] - best[0]:
            best = (x, e)
        x = e
    return best


# ------------------------------------------------------------------------------------------
# The FP32 floor of an image: the same multislice and combination steps carried out in
# complex64 with numpy (single-precision FFTs; phases formed in FP64 and rounded, as on the
# GPU). Its error against the FP64 oracle is what FP32 arithmetic itself leaves on a ring;
# a ring carrying ~1e-12 of the incident intensity cannot be resolved to 1e-4 by it.
# ------------------------------------------------------------------------------------------
def _c64(a):
    return np.asarray(a).astype(np.complex64)


def c64_exit_spectra(st, v, init_spectra):
    """F(psi_exit) in complex64 for initial waves given by their FP64 spectra [n][Y][X]."""
    prop = _c64(st.prop)
    psi = np.fft.ifft2(_c64(init_spectra))
    for j in range(v.shape[0]):
        t = _c64(np.exp(1j * st.sigma * v[j].astype(np.float64)))
        psi = t * psi
        psi = np.fft.ifft2(prop * np.fft.fft2(psi))
    out = np.fft.fft2(psi)
    assert out.dtype == np.complex64
    return out


def _shifted(st, spec, pos):
    return ph.shift_spectrum(spec, st.lx, st.ly, (float(pos[0]), float(pos[1])))


def c64_plain_image(st, v, probes, batch=32):
    """Plain multislice image in complex64 (NaN where not computed), [n_det][Py][Px]."""
    img = np.full((len(st.detectors), st.Py, st.Px), np.nan)
    probes = list(probes)
    for s in range(0, len(probes), batch):
        chunk = probes[s:s + batch]
        init = np.stack([_shifted(st, st.spec0, st.probe_position(a, b)) for a, b in chunk])
        for (a, b), sp in zip(chunk, c64_exit_spectra(st, v, init)):
            img[:, b, a] = ph.detector_values(sp.astype(np.complex128), st.masks)
    return img


def c64_basis(om, v, translates, batch=32):
    """Propagated translates in complex64, {(ta, tb): F(U_i)}, for an oracle LMA object ``om``."""
    out = {}
    translates = list(translates)
    for s in range(0, len(translates), batch):
        chunk = translates[s:s + batch]
        init = np.stack([_shifted(om.setup, om.spec_u, om.lat.translate_position(*t)) for t in chunk])
        for t, sp in zip(chunk, c64_exit_spectra(om.setup, v, init)):
            out[t] = sp
    return out


def c64_exit_spectrum(om, a, b, basis):
    """Probe (a, b)'s exit spectrum combined in complex64 from a complex64 basis."""
    al = om.alpha[om.lat.coefficient_class(a, b)].astype(np.complex64)
    spec = np.zeros((om.setup.ny, om.setup.nx), dtype=np.complex64)
    for c, t in zip(al, om.lat.nearest(a, b)):
        spec += c * basis[t]
    return spec


def c64_lma_image(om, basis, probes):
    st = om.setup
    img = np.full((len(st.detectors), st.Py, st.Px), np.nan)
    for a, b in probes:
        img[:, b, a] = ph.detector_values(c64_exit_spectrum(om, a, b, basis).astype(np.complex128), st.masks)
    return img


def ring_floor(c64_img, ref, probes):
    """Relative L2 per ring of a complex64 image against the oracle's, over ``probes``."""
    idx = (slice(None), [b for _, b in probes], [a for a, _ in probes])
    return [rel_l2(c64_img[idx][r], ref[idx][r]) for r in range(ref.shape[0])]
