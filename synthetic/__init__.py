"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package only *builds inputs*: gridded steady fields (B, E, grad|B|, b.grad b
in the local spherical basis) and injection recipes.  It contains none of the
particle method's arithmetic (no interpolation, no guiding-centre right-hand
side, no time stepping, no scattering).
"""
from .constants import AU, C_LIGHT, E_CHARGE, M_ELECTRON, OMEGA_SUN, V_WIND, B0_1AU
from .grid import SphericalGrid
from . import fields, workloads

__all__ = [
    "AU", "C_LIGHT", "E_CHARGE", "M_ELECTRON", "OMEGA_SUN", "V_WIND", "B0_1AU",
    "SphericalGrid", "fields", "workloads",
]
