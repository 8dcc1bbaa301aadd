"""Seeded synthetic initial conditions shared by the oracle and the HIP path.

This module draws particle sets only: masses, positions and velocities. It
holds none of the integrator's arithmetic (no forces, no energies, no time
steps), so that the oracle and the device path share nothing but their inputs.
"""
from .plummer import plummer, plummer_imf, plummer_with_bh, kepler_pair, WORKLOADS

__all__ = ["plummer", "plummer_imf", "plummer_with_bh", "kepler_pair", "WORKLOADS"]
