"""Closed forms that pin the oracles (and, through them, the input generator).

Clean ribbon: V = 0, 5-point stencil with hop -t, and leads of the same width
attached at both ends.  The device plus its two semi-infinite leads is then an
infinite ribbon, whose transverse modes u_j(x) = sqrt(2/(Nx+1)) sin(j x pi/(Nx+1))
decouple into 1D chains at energy z_j = E + 2t cos(j pi/(Nx+1)).  The local
Green's function of an infinite chain is 1/(sqrt(z-2t) sqrt(z+2t)), so
  G_(x,y),(x,y) = sum_j u_j(x)^2 / (sqrt(z_j-2t) sqrt(z_j+2t))  for every y.
Its transmission tends to the number of open modes #{j : |Re z_j| < 2t} as
eta -> 0.  Nx = 1 is the plain 1D chain.
"""
from __future__ import annotations

import numpy as np


def ribbon_local_G(Nx: int, E: complex, t: float = 1.0) -> np.ndarray:
    x = np.arange(1, Nx + 1)
    j = np.arange(1, Nx + 1)
    u = np.sqrt(2.0 / (Nx + 1)) * np.sin(np.outer(x, j) * np.pi / (Nx + 1))
    z = E + 2.0 * t * np.cos(j * np.pi / (Nx + 1))
    g = 1.0 / (np.sqrt(z - 2.0 * t) * np.sqrt(z + 2.0 * t))
    return (u ** 2) @ g


def ribbon_open_modes(Nx: int, E: float, t: float = 1.0) -> int:
    j = np.arange(1, Nx + 1)
    z = E + 2.0 * t * np.cos(j * np.pi / (Nx + 1))
    return int(np.sum(np.abs(z) < 2.0 * t))
