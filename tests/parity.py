"""Comparison helpers for the GPU parity tests (no GPU needed to import).

Errors per output vector and energy:
  normwise   ||x - x_ref||_inf / ||x_ref||_inf
  entrywise  max |x_i - x_ref,i| / |x_ref,i| over the entries with
             |x_ref,i| >= 1e-3 ||x_ref||_inf
Bond currents are compared normwise against max|J| + max|H| max|G<| (J can
be ~0 on degenerate meshes, where the G< entries it is formed from are not)."""
import numpy as np

TOL = 1e-10
ENTRY_FLOOR = 1e-3
# G< of the symmetric form that also halves R (symmetric = 2): R's lower
# triangle mirrored to an exactly anti-Hermitian R changes the rounding that
# G R G^dagger amplifies near resonances; a numpy execution of the same plan
# with LAPACK solves gave 1.8e-8 on a 64 x 128 9-point mesh, the GPU path
# 1.6e-8 there, 3e-8 at 128 x 128 (energy 128) and 7.9e-8 at 512 x 512.
PACKED_R_TOL = 2e-7


def nrel(x, ref):
    x, ref = np.asarray(x), np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def erel(x, ref, floor=ENTRY_FLOOR, norm=None):
    """Entrywise relative error over the entries at least `floor` times the
    vector's max-abs (`norm`, if the vector is a sample of a longer one)."""
    x, ref = np.asarray(x).ravel(), np.asarray(ref).ravel()
    if norm is None:
        norm = np.max(np.abs(ref))
    sel = np.abs(ref) >= floor * norm
    if not np.any(sel):
        return 0.0
    return float(np.max(np.abs(x[sel] - ref[sel]) / np.abs(ref[sel])))


def compare(out, ref, prob, bonds=True, tol=TOL, etol=None, label="", energies=None, ref_index=None,
            gless_tol=None):
    """Every energy e of `energies` (default all) of `out` against entry
    ref_index[e] (default e) of `ref`: normwise <= tol and entrywise <= etol
    (default 100 tol) for diag G, diag G<, bond G and bond G<; bond J
    normwise.  With gless_tol, the G< outputs (diag G<, bond G<, bond J)
    are held to gless_tol (entrywise 100 gless_tol) instead.  Returns the
    largest errors seen."""
    etol = 100 * tol if etol is None else etol
    nE = out["diag_G"].shape[0]
    energies = range(nE) if energies is None else energies
    worst = dict(norm=0.0, entry=0.0)
    keys = ["diag_G", "diag_Gless"] + (["bond_G", "bond_Gless"] if bonds and ref["bond_G"].shape[1] else [])
    for q, e in enumerate(energies):
        r = q if ref_index is None else ref_index[q]
        for k in keys:
            n_err, e_err = nrel(out[k][e], ref[k][r]), erel(out[k][e], ref[k][r])
            worst["norm"] = max(worst["norm"], n_err)
            worst["entry"] = max(worst["entry"], e_err)
            t, et = (gless_tol, 100 * gless_tol) if gless_tol is not None and "Gless" in k else (tol, etol)
            assert n_err <= t, (label, e, k, "normwise", n_err)
            assert e_err <= et, (label, e, k, "entrywise", e_err)
        if bonds and ref["bond_G"].shape[1]:
            hmax = np.max(np.abs(prob["H"][1:]))
            scale = np.max(np.abs(ref["bond_J"][r])) + hmax * np.max(np.abs(ref["bond_Gless"][r]))
            tj = tol if gless_tol is None else gless_tol
            assert np.max(np.abs(out["bond_J"][e] - ref["bond_J"][r])) <= tj * scale, (label, e, "bond_J")
    return worst
