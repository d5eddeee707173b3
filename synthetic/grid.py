"""Spherical node grid of the gridded field.

Node placement (the paper's MHD grid is stretched in r; this uniform grid
stands in for it):
  r_i  = r_min + i * (r_max - r_min) / (nr - 1),   i = 0 .. nr-1
  th_j = (j + 1/2) * pi / nth,                     j = 0 .. nth-1   (cell-centred, avoids the poles)
  ph_k = 2 pi k / nph,                             k = 0 .. nph-1   (periodic)
Node data are stored [nr][nth][nph][12], components in the local orthonormal
basis (r^, th^, ph^):
  0..2  B          (T)
  3..5  E          (V/m)
  6..8  grad |B|   (T/m)
  9..11 (b.grad) b (1/m)
"""
from dataclasses import dataclass
import math

import numpy as np

N_COMP = 12
COMP_NAMES = ("Br", "Bth", "Bph", "Er", "Eth", "Eph",
              "Gr", "Gth", "Gph", "Kr", "Kth", "Kph")
# optional second node array for the full guiding-centre equations, [nr][nth][nph][9]:
# A = (v_E.grad) b, C = (b.grad) v_E, D = (v_E.grad) v_E (v_E = E x B / B^2), local basis
N_EXTRA = 9
EXTRA_NAMES = ("Ar", "Ath", "Aph", "Cr", "Cth", "Cph", "Dr", "Dth", "Dph")


@dataclass(frozen=True)
class SphericalGrid:
    nr: int
    nth: int
    nph: int
    r_min: float   # m
    r_max: float   # m

    @property
    def dr(self) -> float:
        return (self.r_max - self.r_min) / (self.nr - 1)

    @property
    def dth(self) -> float:
        return math.pi / self.nth

    @property
    def dph(self) -> float:
        return 2.0 * math.pi / self.nph

    def r_nodes(self) -> np.ndarray:
        return self.r_min + np.arange(self.nr, dtype=np.float64) * self.dr

    def th_nodes(self) -> np.ndarray:
        return (np.arange(self.nth, dtype=np.float64) + 0.5) * self.dth

    def ph_nodes(self) -> np.ndarray:
        return np.arange(self.nph, dtype=np.float64) * self.dph

    @property
    def n_nodes(self) -> int:
        return self.nr * self.nth * self.nph

    def shape(self):
        return (self.nr, self.nth, self.nph, N_COMP)
