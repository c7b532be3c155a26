"""Numpy executor of an exported FIND plan (test helper, CPU only).

It walks the plan's stages exactly as the GPU does (same gather maps, same
pool slots) but performs each elimination with textbook dense algebra:
  U = A(B,B) - A(B,S) A(S,S)^{-1} A(S,B)                      (eq. major-update)
  L = A(B,S) A(S,S)^{-1}                                        (eq. express-L)
  R = S(B,B) - L S(S,B) - S(B,S) L^H + L S(S,S) L^H             (eq. gless-update-rule)
and for a final leaf block G = U^{-1}, G< = G R G^H (eq. gless-nn).
It checks the plan (sets, maps, schedule, output records) independently of
the HIP kernels; it is compared with the oracle, never used as one.
"""
from __future__ import annotations

import numpy as np

K_FINAL = 1


def orig_entries(nodes_r, nodes_c, Nx, Ny, Hm, E, sig, sless, sd=None, sld=None):
    """Original A and Sigma< entries between two node lists (dense lookup);
    sd, sld: diagonal scattering self-energies per node (flat), or None."""
    A = -Hm[np.ix_(nodes_r, nodes_c)].astype(np.complex128)
    same = nodes_r[:, None] == nodes_c[None, :]
    A += E * same
    S = np.zeros_like(A)
    if sd is not None:
        A -= np.where(same, sd[nodes_r][:, None], 0)
    if sld is not None:
        S += np.where(same, sld[nodes_r][:, None], 0)
    xr, yr = nodes_r % Nx, nodes_r // Nx
    xc, yc = nodes_c % Nx, nodes_c // Nx
    for c, ycol in ((0, 0), (1, Ny - 1)):
        mask = (yr[:, None] == ycol) & (yc[None, :] == ycol)
        vals = sig[c][xr[:, None], xc[None, :]]
        A -= np.where(mask, vals, 0)
        S += np.where(mask, sless[c][xr[:, None], xc[None, :]], 0)
    return A, S


def execute(plan_export: dict, Nx, Ny, stencil, Hm, E, sig, sless, want_bonds=True, record=None, fronts=None,
            sd=None, sld=None):
    ex = plan_export
    elims, maps, stages = ex["elims"], ex["maps"], ex["stages"]
    variant = 1 if want_bonds else 0
    pool = {}
    for first, count, phase, var in stages:
        if var >= 0 and var != variant:
            continue
        for k in range(first, first + count):
            kind, s, b, n, src0, ld0, src1, ld1, dst, mp = elims[k][:10]
            m = maps[mp: mp + n]
            node, src, pos = m[:, 0], m[:, 1], m[:, 2]
            if kind == K_FINAL:
                U0, R0 = pool[src0]
                G = np.linalg.inv(U0)
                pool[dst] = (-G, G @ R0 @ G.conj().T)
                continue
            A, S = orig_entries(node, node, Nx, Ny, Hm, E, sig, sless, sd, sld)
            for sid, off in ((0, src0), (1, src1)):
                sel = np.where(src == sid)[0]
                if sel.size:
                    U, R = pool[off]
                    A[np.ix_(sel, sel)] = U[np.ix_(pos[sel], pos[sel])]
                    S[np.ix_(sel, sel)] = R[np.ix_(pos[sel], pos[sel])]
            if fronts is not None:
                fronts[k] = (A.copy(), S.copy())
            Sx, Bx = slice(0, s), slice(s, n)
            if s:
                L = np.linalg.solve(A[Sx, Sx].T, A[Bx, Sx].T).T
                U = A[Bx, Bx] - L @ A[Sx, Bx]
                R = S[Bx, Bx] - L @ S[Sx, Bx] - S[Bx, Sx] @ L.conj().T + L @ S[Sx, Sx] @ L.conj().T
            else:
                U, R = A[Bx, Bx].copy(), S[Bx, Bx].copy()
            pool[dst] = (U, R)
            if record is not None:
                record[k] = (U, R)
    nn = Nx * Ny
    dG = np.zeros(nn, np.complex128); dL = np.zeros(nn, np.complex128)
    nb = int(ex["outbonds"][:, 0].max()) + 1 if ex["outbonds"].size else 0
    bG = {}; bL = {}; bJ = {}
    for (fe, n_nodes, nf, bf, nbond, var) in ex["leafout"]:
        if var != variant:
            continue
        Um, Rm = pool[elims[fe][8]]
        for node, l in ex["outnodes"][nf: nf + n_nodes]:
            dG[node] = -Um[l, l]; dL[node] = Rm[l, l]
        for bond, li, lj, kk, hf in ex["outbonds"][bf: bf + nbond]:
            bG[bond] = -Um[li, lj]; bL[bond] = Rm[li, lj]
            y, x = divmod(int(hf), Nx)
            bJ[bond] = (li, lj, kk, hf, Rm[lj, li])
    return dG.reshape(Ny, Nx), dL.reshape(Ny, Nx), bG, bL, bJ
