"""The Lattice Multislice Algorithm, written from Sec. 4.2 of the paper. TEST INFRASTRUCTURE ONLY.

Steps in the paper's order (Fig. lma_pseudocode):
  initialisation  input wave u (here the probe, Sec. 4.2.3: u = psi_0^init), input-wave
                  lattice I and its every-f-th sublattice I_f (Sec. 4.2.1, option (i)),
                  L nearest translates per probe (option (iii)), least-squares
                  coefficients (Sec. 4.2.2) reused across probes (eqs.
                  lma_approximation_exit1 / lma_approximation_exit2)
  step 1          U_i = multislice(u_i) for i in I_f
  step 2          psi_p^exit ~ sum_j alpha_{p,j} U_{i_j}, then the detector (Sec. 3.1)

Readings (the paper is silent or garbled):
  * translate u_i(x) = u(x - i) (Sec. 2 definition; the later u o t_i with t_i(x) = x + i
    has the opposite sign and is not used);
  * lattice cover: R_x r_x = l_x, the offset free (the printed cover equation subtracts
    the offset, which cannot hold for the paper's own I = P + p/2);
  * the offset of I is given as a fraction of the spacing r of I and is kept exact;
  * the coefficient-reuse structure is taken between P and I_f: along each axis one of
    P and R/f must divide the other (Case 1 / Case 2), and the number of coefficient sets
    along that axis is P / gcd(P, R/f);
  * "the L closest input waves": rank by squared periodic distance, minimum-image offset
    taken in [-l/2, l/2); exact ties broken by the offset (probe minus translate) in y,
    then in x, smaller first. Distances are exact rationals;
  * coefficients are the minimum-norm least-squares solution over the whole grid
    (numpy.linalg.lstsq, rcond=None).
"""
from __future__ import annotations

from fractions import Fraction
from math import gcd

import numpy as np

from . import physics as ph
from .multislice import Setup, multislice


def _frac(x) -> Fraction:
    return x if isinstance(x, Fraction) else Fraction(x).limit_denominator(1 << 24)


def _min_image(d: Fraction, length: Fraction) -> Fraction:
    """Periodic offset in [-l/2, l/2)."""
    half = length / 2
    return (d + half) % length - half


class Lattice:
    """Probe lattice P and input-wave lattice I_f with the nearest-translate rule."""

    def __init__(self, setup: Setup, R, f: int, offset_frac, L: int):
        self.setup = setup
        self.Rx, self.Ry = int(R[0]), int(R[1])
        self.f = int(f)
        if self.Rx % self.f or self.Ry % self.f:
            raise ValueError("R must be a multiple of f (Sec. 4.2.1, option (i))")
        self.Rfx, self.Rfy = self.Rx // self.f, self.Ry // self.f
        self.L = int(L)
        if not 1 <= self.L <= self.Rfx * self.Rfy:
            raise ValueError("L out of range")
        self.lx, self.ly = Fraction(setup.lx), Fraction(setup.ly)
        self.rx, self.ry = self.lx / self.Rx, self.ly / self.Ry
        self.ox, self.oy = _frac(offset_frac[0]) * self.rx, _frac(offset_frac[1]) * self.ry
        Px, Py = setup.Px, setup.Py
        for P, Rf in ((Px, self.Rfx), (Py, self.Rfy)):
            if P % Rf and Rf % P:
                raise ValueError("probe and input-wave lattices incompatible (Case 1 / Case 2)")
        self.ncls_x = Px // gcd(Px, self.Rfx)
        self.ncls_y = Py // gcd(Py, self.Rfy)
        self._nearest = {}

    # --- positions -----------------------------------------------------------------
    def translate_position(self, a: int, b: int):
        """Exact position of I_f point (a, b): a f r_x e1 + b f r_y e2 + I_offset."""
        return (a * self.f * self.rx + self.ox, b * self.f * self.ry + self.oy)

    def probe_position_exact(self, a: int, b: int):
        return (a * self.lx / self.setup.Px, b * self.ly / self.setup.Py)

    @property
    def n_translates(self) -> int:
        return self.Rfx * self.Rfy

    def translate_index(self, a: int, b: int) -> int:
        return b * self.Rfx + a

    # --- option (iii): the L closest input waves -----------------------------------
    def nearest(self, a: int, b: int):
        """I_{f,p,L} for probe (a, b) as a list of (ta, tb) translate indices, nearest first."""
        key = (a, b)
        if key not in self._nearest:
            self._nearest[key] = self._nearest_uncached(a, b)
        return self._nearest[key]

    def _nearest_uncached(self, a: int, b: int):
        px, py = self.probe_position_exact(a, b)
        keys = []
        for tb in range(self.Rfy):
            for ta in range(self.Rfx):
                tx, ty = self.translate_position(ta, tb)
                dx = _min_image(px - tx, self.lx)
                dy = _min_image(py - ty, self.ly)
                keys.append((dx * dx + dy * dy, dy, dx, ta, tb))
        keys.sort()
        return [(k[3], k[4]) for k in keys[:self.L]]

    def coefficient_class(self, a: int, b: int):
        """Index of the coefficient set used by probe (a, b) (Case 1: one set; Case 2: c*d)."""
        return (a % self.ncls_x, b % self.ncls_y)


def translate_wave(setup: Setup, spec_u: np.ndarray, pos) -> np.ndarray:
    """u_i = u(. - i) on the grid, by Fourier modulation (exact roll for whole-pixel shifts)."""
    return np.fft.ifft2(ph.shift_spectrum(spec_u, setup.lx, setup.ly, (float(pos[0]), float(pos[1]))))


def least_squares(setup: Setup, lat: Lattice, spec_u: np.ndarray, a: int, b: int):
    """alpha = argmin || psi_p^init - sum_j alpha_j u_{i_j} ||_2 over the grid (Sec. 4.2.2),
    minimum-norm solution; returns (alpha, neighbours, relative residual)."""
    nbr = lat.nearest(a, b)
    B = np.stack([translate_wave(setup, spec_u, lat.translate_position(ta, tb)).ravel()
                  for ta, tb in nbr], axis=1)
    target = setup.probe(a, b).ravel()
    alpha, *_ = np.linalg.lstsq(B, target, rcond=None)
    res = np.linalg.norm(target - B @ alpha) / np.linalg.norm(target)
    return alpha, nbr, res


def trig_transform(n: int):
    """(M, M^-1) of Sec. 2 for degree n: with W[k, j] = exp(-2 pi i j k / (2n + 1)) (the
    modulation matrix; the printed entry lacks the i) and c_k = cos(k pi / (2n + 2)),
    M = W diag(c) holds in row j the coefficients of the translate phi_n(t - 2 pi j / (2n + 1))
    over the elementary waves exp(i k t) (W is symmetric), so a function with coefficient row
    vector f has translate coefficients f M^-1. M^-1 = (1 / (2n + 1)) diag(1 / c) W*: the
    paper prints the factor 1 / (2n + 1)^2, but W W* = (2n + 1) I (W / sqrt(2n + 1) is unitary),
    so that factor gives M M^-1 = I / (2n + 1). Indices k, j run over -n..n."""
    k = np.arange(-n, n + 1)
    W = np.exp(-2j * np.pi * np.outer(k, k) / (2 * n + 1))
    c = np.cos(k * np.pi / (2 * n + 2))
    M = W @ np.diag(c)
    Minv = np.diag(1.0 / c) @ W.conj().T / (2 * n + 1)
    return M, Minv


def trig_coefficients(setup: Setup, lat: "Lattice", spec_u: np.ndarray, a: int, b: int) -> np.ndarray:
    """Closed-form coefficients of probe (a, b) over every translate of I_f for the tensor
    trigonometric input wave (Sec. 2, Sec. 4.2.3): the cell is the period and I_f has
    2n + 1 points per axis (R_f = 2n + 1). The probe's spectrum on K_+ (|k_x| <= n_x,
    |k_y| <= n_y, grid frequency indices), divided by u's scale s (u_hat = s c_kx c_ky), times
    M^-1 along each axis; the translate lattice's offset o enters as the probe shifted by -o.
    Returns alpha[tb][ta] (translate (ta, tb) at (ta r_x f + o_x, tb r_y f + o_y)); frequencies
    outside K_+ are dropped (projection of the probe onto span(u_i))."""
    if lat.Rfx % 2 == 0 or lat.Rfy % 2 == 0:
        raise ValueError("the trigonometric input wave needs an odd number of translates per axis")
    nx_, ny_ = (lat.Rfx - 1) // 2, (lat.Rfy - 1) // 2
    st = setup
    px, py = setup.probe_position(a, b)
    spec_p = ph.shift_spectrum(st.spec0, st.lx, st.ly, (px - float(lat.ox), py - float(lat.oy)))
    kxs, kys = np.arange(-nx_, nx_ + 1), np.arange(-ny_, ny_ + 1)
    f = spec_p[np.ix_(kys % st.ny, kxs % st.nx)] / spec_u[0, 0]      # [ky][kx], u_hat[0, 0] = s
    _, Mx = trig_transform(nx_)
    _, My = trig_transform(ny_)
    # row-vector convention per axis: alpha[jy][jx] = sum_ky sum_kx f[ky][kx] My[ky, jy] Mx[kx, jx]
    al = My.T @ f @ Mx                                                # [jy][jx], j = -n..n
    # translate index ta = j mod (2n + 1)
    return np.roll(np.roll(al, -ny_, axis=0), -nx_, axis=1)


class LMA:
    """LMA with u = psi_0^init (Sec. 4.2.3). Coefficients are computed once per class
    (the Case 1 / Case 2 reuse of Sec. 4.2.2).

    window = (X', Y') selects option (ii) of Sec. 4.2.1: every translate is propagated on an
    X' x Y' pixel window centred on it (origin c = i - (X'/2, Y'/2) in pixels; translates must
    lie on pixels) with the potential cropped to that window, per the DFT's periodicity on the
    window. Readings: the initial wave is u_i cropped to the window; the window propagator has
    the same physical band limit (same pixel size); after the last transmission the window is
    embedded (zero outside) in the cell and the last propagation step is taken there, so the
    exit spectrum is P F(embedded wave) on the cell's frequency grid, as without a window."""

    def __init__(self, setup: Setup, lat: Lattice, spec_u: np.ndarray | None = None, window=None,
                 coefficients: str = "least_squares"):
        self.setup, self.lat = setup, lat
        self.window = None if window is None else (int(window[0]), int(window[1]))
        self.spec_u = setup.spec0 if spec_u is None else spec_u
        self.alpha = {}
        self.residual = {}
        for sy in range(lat.ncls_y):
            for sx in range(lat.ncls_x):
                if coefficients == "trigpoly":
                    # the closed form over all of I_f, kept at the L nearest translates
                    full = trig_coefficients(setup, lat, self.spec_u, sx, sy)
                    self.alpha[(sx, sy)] = np.array([full[tb, ta] for ta, tb in lat.nearest(sx, sy)])
                    target = setup.probe(sx, sy)
                    self.residual[(sx, sy)] = (np.linalg.norm(target - self.approximant(sx, sy)) /
                                               np.linalg.norm(target))
                else:
                    al, _, res = least_squares(setup, lat, self.spec_u, sx, sy)
                    self.alpha[(sx, sy)] = al
                    self.residual[(sx, sy)] = res

    def approximant(self, a: int, b: int) -> np.ndarray:
        """sum_j alpha_j u_{i_j} for probe (a, b) in real space."""
        al = self.alpha[self.lat.coefficient_class(a, b)]
        nbr = self.lat.nearest(a, b)
        out = np.zeros((self.setup.ny, self.setup.nx), dtype=np.complex128)
        for c, (ta, tb) in zip(al, nbr):
            out += c * translate_wave(self.setup, self.spec_u, self.lat.translate_position(ta, tb))
        return out

    def window_origin(self, ta: int, tb: int):
        """Pixel origin of the window of translate (ta, tb): i - (X'/2, Y'/2)."""
        st = self.setup
        tx, ty = self.lat.translate_position(ta, tb)
        ix, iy = tx * st.nx / self.lat.lx, ty * st.ny / self.lat.ly
        if ix.denominator != 1 or iy.denominator != 1:
            raise ValueError("windowed propagation needs translates on pixels")
        return int(ix) - self.window[0] // 2, int(iy) - self.window[1] // 2

    def _propagate_windowed(self, potential: np.ndarray, t) -> np.ndarray:
        st = self.setup
        wx, wy = self.window
        cx, cy = self.window_origin(*t)
        rows = (cy + np.arange(wy)) % st.ny
        cols = (cx + np.arange(wx)) % st.nx
        psi = translate_wave(st, self.spec_u, self.lat.translate_position(*t))[np.ix_(rows, cols)]
        prop_w = ph.propagator(wx, wy, st.lx * wx / st.nx, st.ly * wy / st.ny, st.wavelength, st.dz, st.bandlimit)
        n = potential.shape[0]
        for j in range(n):
            psi = ph.transmission(potential[j][np.ix_(rows, cols)], st.sigma) * psi
            if j + 1 < n:
                psi = np.fft.ifft2(prop_w * np.fft.fft2(psi))
        full = np.zeros((st.ny, st.nx), dtype=np.complex128)
        full[np.ix_(rows, cols)] = psi
        return st.prop * np.fft.fft2(full)

    def propagate(self, potential: np.ndarray, translates, batch: int = 16) -> dict:
        """Step 1: U_i for the given (ta, tb) translates; returns {(ta, tb): DFT(U_i)}."""
        out = {}
        translates = list(translates)
        if self.window is not None:
            for t in translates:
                out[t] = self._propagate_windowed(potential, t)
            return out
        for s in range(0, len(translates), batch):
            chunk = translates[s:s + batch]
            u0 = np.stack([translate_wave(self.setup, self.spec_u, self.lat.translate_position(ta, tb))
                           for ta, tb in chunk])
            ex = np.fft.fft2(multislice(u0, potential, self.setup.sigma, self.setup.prop))
            for t, e in zip(chunk, ex):
                out[t] = e
        return out

    def needed_translates(self, probes):
        need = []
        seen = set()
        for a, b in probes:
            for t in self.lat.nearest(a, b):
                if t not in seen:
                    seen.add(t)
                    need.append(t)
        return need

    def image(self, potential: np.ndarray, probes=None, basis: dict | None = None) -> np.ndarray:
        """Step 2 plus the detector: float64 [n_det][Py][Px], NaN where not computed."""
        st = self.setup
        if probes is None:
            probes = [(a, b) for b in range(st.Py) for a in range(st.Px)]
        probes = list(probes)
        if basis is None:
            basis = self.propagate(potential, self.needed_translates(probes))
        img = np.full((len(st.detectors), st.Py, st.Px), np.nan)
        for a, b in probes:
            img[:, b, a] = ph.detector_values(self.exit_spectrum(a, b, basis), st.masks)
        return img

    def exit_spectrum(self, a: int, b: int, basis: dict) -> np.ndarray:
        """Step 2 in Fourier space: sum_j alpha_j F(U_{i_j}) for probe (a, b), from the
        propagated translates ``basis`` ({(ta, tb): F(U_i)}, as returned by propagate)."""
        st = self.setup
        al = self.alpha[self.lat.coefficient_class(a, b)]
        spec = np.zeros((st.ny, st.nx), dtype=np.complex128)
        for c, t in zip(al, self.lat.nearest(a, b)):
            spec += c * basis[t]
        return spec


def phonon_average(images) -> np.ndarray:
    """Frozen-phonon image: the mean of the per-configuration images (Sec. 3.1)."""
    return np.mean(np.stack(list(images)), axis=0)


def recompute_sets(lat: Lattice, bbox_px, rho: float):
    """Local recompute after a specimen edit (Sec. 4.2.6).

    Reading of "close enough to the changes": a translate is re-propagated when its centre
    lies within ``rho`` (Angstrom) of the edited pixels, the box x0..x1-1, y0..y1-1 (pixel
    indices, periodic; distance along each axis to the box's span of pixel positions,
    combined as a Euclidean distance). rho <= 0 selects every translate. The probes to
    re-form are those whose L-nearest set contains a re-propagated translate.
    Returns (translates R as a set of (ta, tb), probes P' as a set of (a, b))."""
    st = lat.setup
    x0, y0, x1, y1 = bbox_px
    dx, dy = lat.lx / st.nx, lat.ly / st.ny
    lo_x, hi_x = x0 * dx, (x1 - 1) * dx
    lo_y, hi_y = y0 * dy, (y1 - 1) * dy

    def axis(c, lo, hi, length):
        if hi - lo >= length:
            return Fraction(0)
        t = (c - lo) % length
        if t <= hi - lo:
            return Fraction(0)
        return min(t - (hi - lo), length - t)

    R = set()
    r2 = _frac(rho) ** 2 if rho > 0 else None
    for tb in range(lat.Rfy):
        for ta in range(lat.Rfx):
            tx, ty = lat.translate_position(ta, tb)
            d2 = axis(tx, lo_x, hi_x, lat.lx) ** 2 + axis(ty, lo_y, hi_y, lat.ly) ** 2
            if r2 is None or d2 <= r2:
                R.add((ta, tb))
    Pp = set()
    for b in range(st.Py):
        for a in range(st.Px):
            if any(t in R for t in lat.nearest(a, b)):
                Pp.add((a, b))
    return R, Pp
