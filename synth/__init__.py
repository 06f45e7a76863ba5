"""Seeded synthetic Wannier-basis inputs shared by the oracle and the HIP path.

This package only draws random model parameters (lattice, H(R), force
constants, g(Re,Rp)) and names the workloads. It contains none of the
electron-phonon method's arithmetic: no Bloch sums, no eigensolves, no
scattering rates.
"""
from .systems import (  # noqa: F401
    System, Workload, make_system, workload, WORKLOADS, lattice_block,
    ws_block,
)
