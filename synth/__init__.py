"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This package generates specimen potentials (the input of the multislice method) and
names the workloads. It holds none of the method's arithmetic: no wavelength, no
probe, no FFT, no propagation, no lattice or coefficient logic.
"""
from .specimen import WORKLOADS, Workload, potential_slices, atom_sites, phonon_positions

__all__ = ["WORKLOADS", "Workload", "potential_slices", "atom_sites", "phonon_positions"]
