"""Recursive Green's function (RGF) sweep: an oracle independent of ``dense``.

The mesh ordered column by column (fixed y, Nx nodes each) makes A block
tridiagonal for both the 5- and the 9-point stencil (the diagonal hops only
couple adjacent columns).  The paper names RGF as the O(Nx^3 Ny) method FIND
is measured against (Sec. 1); it is used here only as a second, independent
way to get the same selected entries on meshes too large for a dense inverse.

Derivation (block LDU with left-connected Green's functions g_y):
  g_0 = A_00^{-1},  g_y = (A_yy - A_{y,y-1} g_{y-1} A_{y-1,y})^{-1}
  G_{N-1,N-1} = g_{N-1}
  G_yy = g_y + g_y A_{y,y+1} G_{y+1,y+1} A_{y+1,y} g_y
  G_{y,y+1} = -g_y A_{y,y+1} G_{y+1,y+1},  G_{y+1,y} = -G_{y+1,y+1} A_{y+1,y} g_y
  first block column:  G_{y,0} = G_yy Q_y,  Q_0 = I,  Q_y = -A_{y,y-1} g_{y-1} Q_{y-1}
  last block column:   G_{y,N-1} = P_y G_{N-1,N-1},  P_{N-1} = I,  P_y = -g_y A_{y,y+1} P_{y+1}
Sigma< lives on the two contact columns only, so
  G<_{a,b} = G_{a,0} Sigma<_L G_{b,0}^dagger + G_{a,N-1} Sigma<_R G_{b,N-1}^dagger.

With diagonal scattering self-energies (Sec. 1 takes the scattering
self-energy as typically diagonal) A_yy also loses diag(Sigma_d(y)) and every
column carries Sigma<_y = diag(Sigma<_d(y)) (+ the contact's on the first and
last).  G< = sum_j G_{:,j} Sigma<_j G_{:,j}^dagger then follows from the
left-connected lesser function g<_y = sum_{j<=y} gL_{y,j} Sigma<_j gL_{y,j}^dagger
(gL the inverse of the leading y+1 block rows and columns):
  g<_0 = g_0 Sigma<_0 g_0^dagger,
  g<_y = g_y (Sigma<_y + A_{y,y-1} g<_{y-1} A_{y,y-1}^dagger) g_y^dagger
(gL_{y,j} = -g_y A_{y,y-1} gL_{y-1,j} for j < y).  With G_{y,j} =
-g_y A_{y,y+1} G_{y+1,j} for j > y, G_{y+1,j} = -G_{y+1,y+1} A_{y+1,y} gL_{y,j}
and G_{y,j} = K_y gL_{y,j} for j <= y, K_y = I + g_y A_{y,y+1} G_{y+1,y+1} A_{y+1,y}:
  P_y = G<_{y+1,y+1} - G_{y+1,y+1} A_{y+1,y} g<_y A_{y+1,y}^dagger G_{y+1,y+1}^dagger
        (the part of G<_{y+1,y+1} from columns j > y),
  G<_yy = g_y A_{y,y+1} P_y A_{y,y+1}^dagger g_y^dagger + K_y g<_y K_y^dagger,
  G<_{y,y+1} = -g_y A_{y,y+1} G<_{y+1,y+1} - g<_y A_{y+1,y}^dagger G_{y+1,y+1}^dagger,
  G<_{y+1,y} = -(G<_{y,y+1})^dagger.
"""
from __future__ import annotations

import numpy as np

from paper_1104_0623_amd.inputs import bond_counts


def _blocks(Nx: int, Ny: int, H: np.ndarray, E: complex, sigma_e: np.ndarray, sd_e=None):
    nst = H.shape[0]
    D, Up = [], []  # diagonal blocks A_yy, super-diagonal blocks A_{y,y+1}
    for y in range(Ny):
        Hyy = np.diag(H[0, y]).astype(np.complex128)
        off = H[1, y, : Nx - 1]
        Hyy += np.diag(off, 1) + np.diag(off, -1)
        Ayy = E * np.eye(Nx) - Hyy
        if sd_e is not None:
            Ayy = Ayy - np.diag(sd_e[y])
        if y == 0:
            Ayy = Ayy - sigma_e[0]
        if y == Ny - 1:
            Ayy = Ayy - sigma_e[1]
        D.append(Ayy)
        if y + 1 < Ny:
            # H between column y (rows) and column y+1 (cols)
            Hc = np.diag(H[2, y]).astype(np.complex128)
            if nst == 5:
                # (x, y) -- (x+1, y+1): row x, col x+1
                Hc += np.diag(H[3, y, : Nx - 1], 1)
                # (x+1, y) -- (x, y+1): row x+1, col x
                Hc += np.diag(H[4, y, : Nx - 1], -1)
            Up.append(-Hc)
    return D, Up


def rgf_energy(Nx: int, Ny: int, H: np.ndarray, E: complex, sigma_e: np.ndarray,
               sless_e: np.ndarray, sd_e=None, sld_e=None):
    """Returns (Gd, Gup, Gdn, Glessd, Glessup, Glessdn) block lists:
    G_yy, G_{y,y+1}, G_{y+1,y} and the same for G<.  sd_e, sld_e: optional
    diagonal scattering Sigma and Sigma< ([Ny][Nx]) of this energy."""
    D, Up = _blocks(Nx, Ny, H, E, sigma_e, sd_e)
    Dn = [U.T.copy() for U in Up]  # A_{y+1,y} = A_{y,y+1}^T (H real symmetric)
    g = [None] * Ny
    Q = [None] * Ny
    g[0] = np.linalg.inv(D[0])
    Q[0] = np.eye(Nx, dtype=np.complex128)
    for y in range(1, Ny):
        g[y] = np.linalg.inv(D[y] - Dn[y - 1] @ g[y - 1] @ Up[y - 1])
        Q[y] = -Dn[y - 1] @ g[y - 1] @ Q[y - 1]
    Gd = [None] * Ny
    Gd[Ny - 1] = g[Ny - 1]
    P = [None] * Ny
    P[Ny - 1] = np.eye(Nx, dtype=np.complex128)
    Gup, Gdn = [None] * (Ny - 1), [None] * (Ny - 1)
    for y in range(Ny - 2, -1, -1):
        Gd[y] = g[y] + g[y] @ Up[y] @ Gd[y + 1] @ Dn[y] @ g[y]
        Gup[y] = -g[y] @ Up[y] @ Gd[y + 1]
        Gdn[y] = -Gd[y + 1] @ Dn[y] @ g[y]
        P[y] = -g[y] @ Up[y] @ P[y + 1]
    if sld_e is not None:
        return (Gd, Gup, Gdn) + _lesser_distributed(Nx, Ny, D, Up, Dn, g, Gd, sless_e, sld_e)
    C0 = [Gd[y] @ Q[y] for y in range(Ny)]          # G_{y,0}
    CN = [P[y] @ Gd[Ny - 1] for y in range(Ny)]     # G_{y,N-1}
    SL, SR = sless_e[0], sless_e[1]

    def gless(a, b):
        return C0[a] @ SL @ C0[b].conj().T + CN[a] @ SR @ CN[b].conj().T

    Gld = [gless(y, y) for y in range(Ny)]
    Glup = [gless(y, y + 1) for y in range(Ny - 1)]
    Gldn = [gless(y + 1, y) for y in range(Ny - 1)]
    return Gd, Gup, Gdn, Gld, Glup, Gldn


def _lesser_distributed(Nx, Ny, D, Up, Dn, g, Gd, sless_e, sld_e):
    """G< blocks with Sigma< on every column (module docstring)."""
    def sig(y):
        s = np.diag(sld_e[y]).astype(np.complex128)
        if y == 0:
            s = s + sless_e[0]
        if y == Ny - 1:
            s = s + sless_e[1]
        return s
    gl = [None] * Ny
    gl[0] = g[0] @ sig(0) @ g[0].conj().T
    for y in range(1, Ny):
        gl[y] = g[y] @ (sig(y) + Dn[y - 1] @ gl[y - 1] @ Dn[y - 1].conj().T) @ g[y].conj().T
    Gld = [None] * Ny
    Glup, Gldn = [None] * (Ny - 1), [None] * (Ny - 1)
    Gld[Ny - 1] = gl[Ny - 1]
    for y in range(Ny - 2, -1, -1):
        a_up, a_dn, G1 = Up[y], Dn[y], Gd[y + 1]           # A_{y,y+1}, A_{y+1,y}, G_{y+1,y+1}
        P = Gld[y + 1] - G1 @ a_dn @ gl[y] @ a_dn.conj().T @ G1.conj().T
        K = np.eye(Nx) + g[y] @ a_up @ G1 @ a_dn
        Gld[y] = g[y] @ a_up @ P @ a_up.conj().T @ g[y].conj().T + K @ gl[y] @ K.conj().T
        Glup[y] = -g[y] @ a_up @ Gld[y + 1] - gl[y] @ a_dn.conj().T @ G1.conj().T
        Gldn[y] = -Glup[y].conj().T
    return Gld, Glup, Gldn


def rgf_solve(Nx: int, Ny: int, stencil: int, H: np.ndarray, energies, sigma: np.ndarray,
              sigma_less: np.ndarray, bonds: bool = True, sigma_d=None, sigma_less_d=None) -> dict:
    """Same outputs as ``dense.dense_solve`` via the RGF sweep (optionally with
    diagonal scattering self-energies sigma_d, sigma_less_d [nE][Ny][Nx],
    both or neither)."""
    if (sigma_d is None) != (sigma_less_d is None):
        raise ValueError("sigma_d and sigma_less_d go together")
    energies = np.atleast_1d(np.asarray(energies, dtype=np.complex128))
    nE = energies.size
    out = dict(diag_G=np.empty((nE, Ny, Nx), np.complex128),
               diag_Gless=np.empty((nE, Ny, Nx), np.complex128))
    counts = bond_counts(Nx, Ny, stencil)
    nb = int(sum(counts))
    if bonds:
        out.update(bond_G=np.empty((nE, nb), np.complex128),
                   bond_Gless=np.empty((nE, nb), np.complex128),
                   bond_J=np.empty((nE, nb), np.float64))
    for e in range(nE):
        Gd, Gup, Gdn, Gld, Glup, Gldn = rgf_energy(
            Nx, Ny, H, energies[e], sigma[e], sigma_less[e],
            None if sigma_d is None else sigma_d[e], None if sigma_less_d is None else sigma_less_d[e])
        for y in range(Ny):
            out["diag_G"][e, y] = np.diag(Gd[y])
            out["diag_Gless"][e, y] = np.diag(Gld[y])
        if not bonds:
            continue
        bG, bL, bJ = out["bond_G"][e], out["bond_Gless"][e], out["bond_J"][e]
        k = 0
        # x-bonds: i=(x,y), j=(x+1,y)
        for y in range(Ny):
            for x in range(Nx - 1):
                h = H[1, y, x]
                bG[k] = Gd[y][x, x + 1]
                bL[k] = Gld[y][x, x + 1]
                bJ[k] = 2.0 * np.real(h * Gld[y][x + 1, x])
                k += 1
        # y-bonds: i=(x,y), j=(x,y+1)
        for y in range(Ny - 1):
            for x in range(Nx):
                h = H[2, y, x]
                bG[k] = Gup[y][x, x]
                bL[k] = Glup[y][x, x]
                bJ[k] = 2.0 * np.real(h * Gldn[y][x, x])
                k += 1
        if stencil == 9:
            # d+: i=(x,y), j=(x+1,y+1)
            for y in range(Ny - 1):
                for x in range(Nx - 1):
                    h = H[3, y, x]
                    bG[k] = Gup[y][x, x + 1]
                    bL[k] = Glup[y][x, x + 1]
                    bJ[k] = 2.0 * np.real(h * Gldn[y][x + 1, x])
                    k += 1
            # d-: i=(x+1,y), j=(x,y+1)
            for y in range(Ny - 1):
                for x in range(Nx - 1):
                    h = H[4, y, x]
                    bG[k] = Gup[y][x + 1, x]
                    bL[k] = Glup[y][x + 1, x]
                    bJ[k] = 2.0 * np.real(h * Gldn[y][x, x + 1])
                    k += 1
        assert k == nb
    return out
