"""Seeded synthetic crystal specimens and the named workloads.

A specimen is a set of atom sites on a simple-cubic or FCC lattice inside a periodic
lx x ly cell of thickness nslices*dz. Each site carries a projected-potential amplitude
(V*Angstrom, read as the peak value of its Gaussian). A frozen-phonon configuration
displaces every site by independent N(0, sigma_d^2) offsets per coordinate. The
potential of slice j is the sum, over the atoms whose displaced z falls in slice j, of
isotropic Gaussians of standard deviation 0.3 Angstrom evaluated on the pixel grid
with periodic minimum-image distances and truncated at 2.4 Angstrom per axis.

Seeds: ``numpy.random.default_rng([workload_id, stream, index])``; species draws use
stream 0 (fixed across phonon configurations), displacements of configuration c use
stream 1, index c.

The result is float32 [nslices][ny][nx]; every consumer (GPU path and oracle) reads
the same float32 array.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

ATOM_SIGMA = 0.3     # Angstrom, Gaussian width of one projected atom
ATOM_CUTOFF = 2.4    # Angstrom, per-axis truncation of the Gaussian


@dataclass(frozen=True)
class Workload:
    name: str
    wid: int                      # seed component
    nx: int
    ny: int
    lx: float                     # Angstrom
    ly: float
    nslices: int
    dz: float                     # Angstrom
    lattice: str                  # "sc" | "fcc"
    a: float                      # lattice constant, Angstrom
    amplitudes: tuple             # V*Angstrom per species
    probs: tuple                  # species probabilities
    sigma_d: float                # displacement std, Angstrom
    kv: float                     # accelerating voltage, kV
    alpha_mrad: float             # probe aperture semi-angle
    defocus: float                # Z, Angstrom
    cs: float                     # C_s, Angstrom
    bandlimit: float              # fraction of Nyquist
    scan: tuple                   # (Px, Py)
    basis_px: int                 # spacing of the propagated translate lattice, pixels
    offset_frac: tuple            # translate-lattice offset as a fraction of its spacing
    L: int                        # nearest translates per probe
    n_phonons: int
    detectors: tuple = field(default_factory=tuple)   # ((name, inner_mrad, outer_mrad), ...)
    R: tuple = ()                 # input-wave lattice size (Rx, Ry) when not nx / basis_px
    f: int = 1                    # every f-th input wave is propagated

    def lattice_size(self):
        """(Rx, Ry) of the input-wave lattice I and f, so that I_f has (Rx / f, Ry / f) points."""
        if self.R:
            return tuple(self.R), self.f
        return (self.nx // self.basis_px, self.ny // self.basis_px), self.f

    @property
    def thickness(self) -> float:
        return self.nslices * self.dz


_STD_DET = (("BF", 0.0, 15.0), ("ADF", 16.0, 40.0), ("HAADF", 41.0, 200.0))

WORKLOADS = {
    # 128^2 over 12.8 A, 10 x 2 A slices, simple cubic a=4 A, one species of 20 V*A.
    "tiny": Workload("tiny", 1, 128, 128, 12.8, 12.8, 10, 2.0, "sc", 4.0, (20.0,), (1.0,),
                     0.05, 200.0, 20.0, 0.0, 0.0, 2.0 / 3.0, (16, 16), 4, (0.5, 0.5), 64, 1,
                     (("HAADF70", 70.0, 200.0),) + _STD_DET),
    # 512^2 over 51.2 A, 100 x 2 A slices, FCC a=4.05 A, species {14,29,79} V*A.
    "medium": Workload("medium", 2, 512, 512, 51.2, 51.2, 100, 2.0, "fcc", 4.05, (14.0, 29.0, 79.0),
                       (1 / 3, 1 / 3, 1 / 3), 0.08, 200.0, 20.0, 0.0, 0.0, 2.0 / 3.0, (128, 128), 4,
                       (0.5, 0.5), 144, 8, _STD_DET),
    # 2048^2 over 204.8 A, 250 x 2 A slices, FCC random alloy {29,79} V*A, 300 kV.
    "large": Workload("large", 3, 2048, 2048, 204.8, 204.8, 250, 2.0, "fcc", 4.05, (29.0, 79.0),
                      (0.5, 0.5), 0.1, 300.0, 25.0, -50.0, 0.0, 2.0 / 3.0, (256, 256), 4, (0.5, 0.5),
                      144, 16, _STD_DET),
    # The paper's local-edit experiment in shape only (Sec. 4.2.6): 1024^2 px over
    # 84.536 x 79.941 A, scan 424 x 400, I = P + p/2 with f = 2 (|I_f| = 42400), L = 59,
    # 200 kV, 26 mrad, Z = 100 A, C_s = -2000 A; the specimen is this module's synthetic FCC
    # crystal, 50 x 2 A slices (the paper's M1 specimen and thickness are not available).
    "paper": Workload("paper", 4, 1024, 1024, 84.536, 79.941, 50, 2.0, "fcc", 4.05, (14.0, 29.0, 79.0),
                      (1 / 3, 1 / 3, 1 / 3), 0.08, 200.0, 26.0, 100.0, -2000.0, 2.0 / 3.0, (424, 400), 0,
                      (0.5, 0.5), 59, 1, _STD_DET, R=(424, 400), f=2),
}


# Uneven batch: independent specimens of mixed grid sizes (0.1 A/px), slice counts and scans.
UNEVEN_SIDES = (96, 128, 192, 256, 384, 512, 640)


def uneven_batch(n: int = 64, seed: int = 0):
    """n specimens with square grids whose sides are drawn uniformly from UNEVEN_SIDES at
    0.1 A/px, slice counts uniform in 20..200 (2 A each), the medium workload's FCC
    specimen and optics, translates every 4 px, L = 144, and a scan of 32..128 positions
    per side drawn from those for which the coefficient sets per axis number 1 or 2
    (P divides R, or P = 2R, with R = side / 4). Seeds: default_rng([5, 3, seed])."""
    rng = np.random.default_rng([5, 3, seed])
    out = []
    for i in range(n):
        side = int(rng.choice(UNEVEN_SIDES))
        nsl = int(rng.integers(20, 201))
        R = side // 4
        scans = [P for P in range(32, 129) if R % P == 0 or P == 2 * R]
        P = int(rng.choice(scans))
        out.append(Workload(f"uneven{i}", 1000 + i, side, side, side * 0.1, side * 0.1, nsl, 2.0, "fcc", 4.05,
                            (14.0, 29.0, 79.0), (1 / 3, 1 / 3, 1 / 3), 0.08, 200.0, 20.0, 0.0, 0.0, 2.0 / 3.0,
                            (P, P), 4, (0.5, 0.5), 144, 1, _STD_DET))
    return out


def _basis(lattice: str) -> np.ndarray:
    if lattice == "sc":
        return np.zeros((1, 3))
    if lattice == "fcc":
        return np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    raise ValueError(f"unknown lattice {lattice!r}")


def atom_sites(w: Workload):
    """Undisplaced sites (n,3) in Angstrom and per-site amplitude (n,), species fixed by seed."""
    b = _basis(w.lattice)
    nxc = int(math.ceil(w.lx / w.a)) + 1
    nyc = int(math.ceil(w.ly / w.a)) + 1
    nzc = int(math.ceil(w.thickness / w.a)) + 1
    i, j, k = np.meshgrid(np.arange(nxc), np.arange(nyc), np.arange(nzc), indexing="ij")
    cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + b[None, :, :]).reshape(-1, 3) * w.a
    keep = (sites[:, 0] < w.lx) & (sites[:, 1] < w.ly) & (sites[:, 2] < w.thickness)
    sites = sites[keep]
    # deterministic order: by z, then y, then x
    order = np.lexsort((sites[:, 0], sites[:, 1], sites[:, 2]))
    sites = sites[order]
    rng = np.random.default_rng([w.wid, 0, 0])
    species = rng.choice(len(w.amplitudes), size=len(sites), p=np.asarray(w.probs))
    amps = np.asarray(w.amplitudes, dtype=np.float64)[species]
    return sites, amps


def phonon_positions(w: Workload, config: int, sites: np.ndarray | None = None) -> np.ndarray:
    """Sites displaced for frozen-phonon configuration ``config`` (x, y wrapped into the cell)."""
    if sites is None:
        sites, _ = atom_sites(w)
    rng = np.random.default_rng([w.wid, 1, config])
    pos = sites + rng.normal(0.0, w.sigma_d, size=sites.shape)
    pos[:, 0] = np.mod(pos[:, 0], w.lx)
    pos[:, 1] = np.mod(pos[:, 1], w.ly)
    return pos


def _axis_factors(coord: np.ndarray, n: int, length: float) -> np.ndarray:
    """Truncated 1-D Gaussian factors [n_atoms, n] with periodic minimum-image distance."""
    grid = np.arange(n, dtype=np.float64) * (length / n)
    d = grid[None, :] - coord[:, None]
    d = d - length * np.round(d / length)
    g = np.exp(-(d * d) / (2.0 * ATOM_SIGMA * ATOM_SIGMA))
    g[np.abs(d) > ATOM_CUTOFF] = 0.0
    return g


def potential_from_atoms(w: Workload, pos: np.ndarray, amps: np.ndarray,
                         slices: range | None = None) -> np.ndarray:
    """Projected potential float32 [len(slices)][ny][nx] from atom positions and amplitudes."""
    if slices is None:
        slices = range(w.nslices)
    sl = np.clip(np.floor(pos[:, 2] / w.dz).astype(np.int64), 0, w.nslices - 1)
    out = np.zeros((len(slices), w.ny, w.nx), dtype=np.float32)
    for o, j in enumerate(slices):
        sel = np.nonzero(sl == j)[0]
        if sel.size == 0:
            continue
        gx = _axis_factors(pos[sel, 0], w.nx, w.lx)
        gy = _axis_factors(pos[sel, 1], w.ny, w.ly)
        out[o] = ((gy * amps[sel, None]).T @ gx).astype(np.float32)
    return out


def potential_slices(w: Workload, config: int = 0) -> np.ndarray:
    """float32 [nslices][ny][nx] potential (V*Angstrom) of phonon configuration ``config``."""
    sites, amps = atom_sites(w)
    pos = phonon_positions(w, config, sites)
    return potential_from_atoms(w, pos, amps)


def edit_column(w: Workload, config: int, col_xy: tuple, seed: int = 0):
    """A local edit: the atoms of the undisplaced site column nearest ``col_xy`` (Angstrom)
    get a new amplitude drawn from the species set and each keeps its site with
    probability 1/2. Returns (pos, amps) of the edited specimen for configuration ``config``
    and the (x0, y0, x1, y1) pixel box, half-open, that bounds the edited Gaussians."""
    sites, amps = atom_sites(w)
    pos = phonon_positions(w, config, sites)
    dx = sites[:, 0] - col_xy[0]
    dy = sites[:, 1] - col_xy[1]
    d2 = dx * dx + dy * dy
    col = np.nonzero(d2 <= d2.min() + 1e-9)[0]
    rng = np.random.default_rng([w.wid, 2, seed])
    new_amp = float(np.asarray(w.amplitudes)[rng.integers(len(w.amplitudes))])
    keep = rng.random(col.size) < 0.5
    amps = amps.copy()
    amps[col] = new_amp
    drop = col[~keep]
    mask = np.ones(len(amps), dtype=bool)
    mask[drop] = False
    cx, cy = sites[col[0], 0], sites[col[0], 1]
    rx = pos[col, 0] - cx
    rx -= w.lx * np.round(rx / w.lx)
    ry = pos[col, 1] - cy
    ry -= w.ly * np.round(ry / w.ly)
    px = w.lx / w.nx
    py = w.ly / w.ny
    x0 = int(math.floor((cx + rx.min() - ATOM_CUTOFF) / px))
    x1 = int(math.ceil((cx + rx.max() + ATOM_CUTOFF) / px)) + 1
    y0 = int(math.floor((cy + ry.min() - ATOM_CUTOFF) / py))
    y1 = int(math.ceil((cy + ry.max() + ATOM_CUTOFF) / py)) + 1
    return pos[mask], amps[mask], (x0, y0, x1, y1)
