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
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


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
