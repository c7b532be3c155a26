"""Seeded synthetic inputs for FIND solves on an Nx x Ny tight-binding mesh.

This module only *generates inputs*; it holds none of the selected-inversion
arithmetic.  Both the GPU path (through the C-ABI) and the CPU oracle under
``oracle/`` consume what it returns.

Conventions (shared by every consumer):

* Mesh node (x, y), x in [0, Nx) transverse, y in [0, Ny) along transport.
  Linear index i = y * Nx + x.  The two contacts attach to the columns
  y = 0 (left, contact 0) and y = Ny - 1 (right, contact 1).
* ``H`` is real float64 of shape [nst][Ny][Nx], nst = 3 (5-point) or 5
  (9-point).  Entries are matrix *values* H_ij (hopping -t is stored as -t):

  - H[0][y][x]  on-site H_ii for node (x, y)
  - H[1][y][x]  H between (x, y) and (x+1, y)      (x < Nx-1, else 0)
  - H[2][y][x]  H between (x, y) and (x, y+1)      (y < Ny-1, else 0)
  - H[3][y][x]  H between (x, y) and (x+1, y+1)    (9-point only)
  - H[4][y][x]  H between (x+1, y) and (x, y+1)    (9-point only)

* Contact self-energies ``sigma`` are complex128 [nE][2][Nx][Nx] with
  sigma[e][c][a][b] = entry (row a, column b) of Sigma_c, indexed by the
  transverse coordinate x of the contact column.  ``sigma_less`` has the
  same layout.
* A(E) = E*I - H - Sigma_L - Sigma_R (Sigma_c placed on its contact column);
  G = A^{-1}, G< = G Sigma< G^dagger (paper, Sec. 1, the NEGF definitions).
* Energies are complex (E + i*eta).
* Bonds (pairs with H_ij != 0, i != j) are numbered family by family:
  x-bonds [Ny][Nx-1], y-bonds [Ny-1][Nx], then for 9-point meshes d+ bonds
  [Ny-1][Nx-1] and d- bonds [Ny-1][Nx-1].  Each bond has a first node i and a
  second node j (see :func:`bond_endpoints`); the bond current is
  J_{i->j} = 2 Re(H_ij G<_ji).

The lead self-energy is the textbook retarded surface term of a semi-infinite
ribbon of the same width with hopping -t, written in the transverse sine
basis: Sigma = U diag(sigma_j) U^T with U_xj = sqrt(2/(Nx+1)) sin(j x pi/(Nx+1))
(x, j counted from 1) and sigma_j = (z_j - sqrt(z_j-2t) sqrt(z_j+2t)) / 2,
z_j = E + 2t cos(j pi/(Nx+1)) (principal square roots; Im sigma_j <= 0 for
Im E >= 0).
"""
from __future__ import annotations

import numpy as np

STENCIL_NST = {5: 3, 9: 5}


def n_stencil_arrays(stencil: int) -> int:
    if stencil not in STENCIL_NST:
        raise ValueError(f"stencil must be 5 or 9, got {stencil}")
    return STENCIL_NST[stencil]


def make_hamiltonian(Nx: int, Ny: int, stencil: int = 5, t: float = 1.0,
                     tp: float = 0.1, vmax: float = 0.5, seed: int = 0,
                     onsite: np.ndarray | None = None) -> np.ndarray:
    """Tight-binding H: on-site V ~ U[-vmax, vmax] drawn with PCG64(seed) in
    linear-index order, nearest-neighbour hop value -t, diagonal hop value -tp
    (9-point only)."""
    nst = n_stencil_arrays(stencil)
    H = np.zeros((nst, Ny, Nx), dtype=np.float64)
    if onsite is not None:
        H[0] = np.asarray(onsite, dtype=np.float64).reshape(Ny, Nx)
    elif vmax != 0.0:
        rng = np.random.default_rng(seed)
        H[0] = rng.uniform(-vmax, vmax, size=(Ny, Nx))
    H[1, :, : Nx - 1] = -t
    H[2, : Ny - 1, :] = -t
    if stencil == 9:
        H[3, : Ny - 1, : Nx - 1] = -tp
        H[4, : Ny - 1, : Nx - 1] = -tp
    return H


def energies_linspace(a: float, b: float, n: int, eta: float = 1e-6) -> np.ndarray:
    """Inclusive equispaced real grid plus i*eta."""
    return np.linspace(a, b, n) + 1j * eta


def lead_mode_sigma(z: np.ndarray, t: float = 1.0) -> np.ndarray:
    """Retarded surface self-energy of a semi-infinite 1D chain (hop -t) at
    complex energy z: (z - sqrt(z-2t) sqrt(z+2t)) / 2, principal roots."""
    z = np.asarray(z, dtype=np.complex128)
    return 0.5 * (z - np.sqrt(z - 2.0 * t) * np.sqrt(z + 2.0 * t))


def transverse_modes(Nx: int) -> tuple[np.ndarray, np.ndarray]:
    """Orthonormal sine basis U (U[x, j]) and cos(j pi/(Nx+1)), j = 1..Nx."""
    x = np.arange(1, Nx + 1)
    j = np.arange(1, Nx + 1)
    U = np.sqrt(2.0 / (Nx + 1)) * np.sin(np.outer(x, j) * np.pi / (Nx + 1))
    return U, np.cos(j * np.pi / (Nx + 1))


def lead_self_energy(Nx: int, E: complex, t: float = 1.0) -> np.ndarray:
    U, c = transverse_modes(Nx)
    sig = lead_mode_sigma(E + 2.0 * t * c, t)
    return (U * sig[None, :]) @ U.T


def contact_self_energies(Nx: int, energies: np.ndarray, t: float = 1.0) -> np.ndarray:
    """[nE][2][Nx][Nx] complex: identical left and right leads."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.complex128))
    out = np.empty((energies.size, 2, Nx, Nx), dtype=np.complex128)
    for e, E in enumerate(energies):
        S = lead_self_energy(Nx, E, t)
        out[e, 0] = S
        out[e, 1] = S
    return out


def lesser_self_energies(sigma: np.ndarray, fL: float, fR: float) -> np.ndarray:
    """Sigma<_c = -f_c (Sigma_c - Sigma_c^dagger) per contact."""
    out = np.empty_like(sigma)
    f = (fL, fR)
    for c in range(2):
        S = sigma[:, c]
        out[:, c] = -f[c] * (S - np.conj(np.swapaxes(S, -1, -2)))
    return out


def scattering_self_energies(Nx: int, Ny: int, nE: int, gamma: float = 0.05, f: float = 0.5,
                             seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Diagonal scattering self-energies on every node (Buttiker-probe-like
    dephasing): Sigma_d = -i gamma_i / 2 with gamma_i ~ U[gamma/2, 3 gamma/2]
    (seeded, linear-index order, the same for every energy) and
    Sigma<_d = -f (Sigma_d - Sigma_d^*) = i f gamma_i.  Arrays [nE][Ny][Nx]."""
    rng = np.random.default_rng(seed)
    g = rng.uniform(0.5 * gamma, 1.5 * gamma, size=Nx * Ny).reshape(Ny, Nx)
    sd = np.ascontiguousarray(np.broadcast_to(-0.5j * g, (nE, Ny, Nx)), dtype=np.complex128)
    sl = -f * (sd - sd.conj())
    return sd, np.ascontiguousarray(sl)


def scattering_self_energies_varied(Nx: int, Ny: int, nE: int, gamma: float = 0.05, shift: float = 0.05,
                                    seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Diagonal scattering self-energies that differ per energy and per node
    (an energy-dependent local self-energy with a level shift):
    Sigma_d[e][y][x] = s - i g / 2 with s ~ U[-shift, shift] and
    g ~ U[gamma/2, 3 gamma/2], and Sigma<_d = i f_e g with an occupation
    f_e ~ U[0, 1] per energy (seeded).  Arrays [nE][Ny][Nx]."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(-shift, shift, size=(nE, Ny, Nx))
    g = rng.uniform(0.5 * gamma, 1.5 * gamma, size=(nE, Ny, Nx))
    f = rng.uniform(0.0, 1.0, size=(nE, 1, 1))
    return (s - 0.5j * g).astype(np.complex128), (1j * f * g).astype(np.complex128)


def bond_scattering_self_energies(Nx: int, Ny: int, stencil: int, nE: int, scale: float = 0.02,
                                  f: float = 0.5, symmetric: bool = False,
                                  seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Stencil-pattern (nearest-neighbour) scattering self-energies, laid out
    like H's bond planes with two values per bond: [nE][nst-1][Ny][Nx][2],
    index 0 the entry from the bond's first node to its second, index 1 the
    entry back (nst = 3 for the 5-point, 5 for the 9-point stencil; entries
    of bonds that leave the mesh are ignored).  Sigma_b = (a - i b) scale with
    a ~ U[-1, 1], b ~ U[0, 1] per entry and energy (seeded; the two directions
    equal with ``symmetric``, so that A stays complex symmetric), and
    Sigma<_b = -f (Sigma_b - Sigma_b^dagger), i.e. entry (i, j) is
    -f (Sigma_ij - conj(Sigma_ji))."""
    rng = np.random.default_rng(seed)
    nb = 2 if stencil == 5 else 4
    shape = (nE, nb, Ny, Nx, 2)
    sb = scale * (rng.uniform(-1.0, 1.0, size=shape) - 1j * rng.uniform(0.0, 1.0, size=shape))
    if symmetric:
        sb[..., 1] = sb[..., 0]
    sl = np.empty_like(sb)
    sl[..., 0] = -f * (sb[..., 0] - np.conj(sb[..., 1]))
    sl[..., 1] = -f * (sb[..., 1] - np.conj(sb[..., 0]))
    return sb.astype(np.complex128), sl.astype(np.complex128)


def general_contact_perturbation(nE: int, Nx: int, scale: float, seed: int = 0) -> np.ndarray:
    """A seeded complex perturbation [nE][2][Nx][Nx] with no symmetry
    (entries (a + i b) * scale, a, b ~ U[-1, 1]); added to the lead
    self-energies it gives contact blocks that are neither complex symmetric
    nor Hermitian, and as Sigma< one that is not anti-Hermitian."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=(nE, 2, Nx, Nx))
    im = rng.uniform(-1.0, 1.0, size=(nE, 2, Nx, Nx))
    return (scale * (re + 1j * im)).astype(np.complex128)


def bond_counts(Nx: int, Ny: int, stencil: int) -> list[int]:
    n = [max(Nx - 1, 0) * Ny, Nx * max(Ny - 1, 0)]
    if stencil == 9:
        d = max(Nx - 1, 0) * max(Ny - 1, 0)
        n += [d, d]
    return n


def n_bonds(Nx: int, Ny: int, stencil: int) -> int:
    return int(sum(bond_counts(Nx, Ny, stencil)))


def bond_endpoints(Nx: int, Ny: int, stencil: int) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """(first node i, second node j, stencil array index, flat index into
    H[k] of the bond value) for every bond in output order."""
    I, J, K, F = [], [], [], []
    ys, xs = np.meshgrid(np.arange(Ny), np.arange(Nx - 1), indexing="ij")
    I.append(ys * Nx + xs); J.append(ys * Nx + xs + 1); K.append(np.full(xs.shape, 1)); F.append(ys * Nx + xs)
    ys, xs = np.meshgrid(np.arange(Ny - 1), np.arange(Nx), indexing="ij")
    I.append(ys * Nx + xs); J.append((ys + 1) * Nx + xs); K.append(np.full(xs.shape, 2)); F.append(ys * Nx + xs)
    if stencil == 9:
        ys, xs = np.meshgrid(np.arange(Ny - 1), np.arange(Nx - 1), indexing="ij")
        I.append(ys * Nx + xs); J.append((ys + 1) * Nx + xs + 1); K.append(np.full(xs.shape, 3)); F.append(ys * Nx + xs)
        I.append(ys * Nx + xs + 1); J.append((ys + 1) * Nx + xs); K.append(np.full(xs.shape, 4)); F.append(ys * Nx + xs)
    cat = lambda L: np.concatenate([a.ravel() for a in L]).astype(np.int64)
    return cat(I), cat(J), cat(K), cat(F)


# Workload presets (mesh sizes, distributions and energy grids of the
# configurations the library is measured on).
PRESETS = {
    "c1_16x16": dict(Nx=16, Ny=16, stencil=5, vmax=0.5, seed=0,
                     energies=("list", [0.3]), fL=1.0, fR=0.0),
    "c2_64x64": dict(Nx=64, Ny=64, stencil=5, vmax=0.5, seed=0,
                     energies=("linspace", -3.5, 3.5, 16), fL=0.5, fR=0.5),
    "c3_128x128": dict(Nx=128, Ny=128, stencil=5, vmax=1.0, seed=0,
                       energies=("linspace", -3.5, 3.5, 256), fL=1.0, fR=0.0),
    "c5_512x512": dict(Nx=512, Ny=512, stencil=9, vmax=1.0, seed=0,
                       energies=("linspace", -3.0, 3.0, 32), fL=1.0, fR=0.0),
}


def preset_energies(spec, eta: float = 1e-6) -> np.ndarray:
    if spec[0] == "list":
        return np.asarray(spec[1], dtype=np.float64) + 1j * eta
    _, a, b, n = spec
    return energies_linspace(a, b, n, eta)


def make_problem(Nx: int, Ny: int, stencil: int = 5, vmax: float = 0.5, seed: int = 0,
                 energies=None, fL: float = 1.0, fR: float = 0.0, t: float = 1.0,
                 tp: float = 0.1, eta: float = 1e-6) -> dict:
    """All inputs of one solve as numpy arrays."""
    if energies is None:
        energies = np.array([0.3 + 1j * eta])
    energies = np.atleast_1d(np.asarray(energies, dtype=np.complex128))
    H = make_hamiltonian(Nx, Ny, stencil, t=t, tp=tp, vmax=vmax, seed=seed)
    sigma = contact_self_energies(Nx, energies, t)
    sless = lesser_self_energies(sigma, fL, fR)
    return dict(Nx=Nx, Ny=Ny, stencil=stencil, H=H, energies=energies,
                sigma=sigma, sigma_less=sless, fL=fL, fR=fR, t=t)


def make_preset(name: str, n_energies: int | None = None) -> dict:
    p = dict(PRESETS[name])
    E = preset_energies(p.pop("energies"))
    if n_energies is not None:
        E = E[:n_energies]
    return make_problem(energies=E, **p)


def random_problem(Nx: int, Ny: int, stencil: int, nE: int, seed: int,
                   vmax: float = 1.0, fL: float = 1.0, fR: float = 0.0,
                   emin: float = -3.5, emax: float = 3.5, eta: float = 1e-6) -> dict:
    """Energies i.i.d. uniform in [emin, emax] + i*eta (serving requests)."""
    rng = np.random.default_rng(seed)
    E = rng.uniform(emin, emax, size=nE) + 1j * eta
    return make_problem(Nx, Ny, stencil, vmax=vmax, seed=seed + 7919, energies=E, fL=fL, fR=fR)
