"""Writes tests/golden/exact_*.json: exact brute-force outputs (oracle.exact)
for two tiny meshes.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402
from paper_1104_0623_amd import inputs  # noqa: E402

CASES = [
    dict(name="exact_3x3_5pt", Nx=3, Ny=3, stencil=5, seed=21, E=0.3 + 1e-3j, fL=1.0, fR=0.0),
    dict(name="exact_3x2_9pt", Nx=3, Ny=2, stencil=9, seed=22, E=-1.3 + 1e-2j, fL=1.0, fR=0.5),
]


def main():
    for c in CASES:
        p = inputs.make_problem(c["Nx"], c["Ny"], c["stencil"], vmax=0.5, seed=c["seed"],
                                energies=[c["E"]], fL=c["fL"], fR=c["fR"])
        bi, bj, _, _ = inputs.bond_endpoints(c["Nx"], c["Ny"], c["stencil"])
        dG, dGl, bonds = exact.exact_solve(c["Nx"], c["Ny"], p["H"], c["E"], p["sigma"][0],
                                           p["sigma_less"][0], list(zip(bi.tolist(), bj.tolist())))
        rec = dict(case=c | dict(E=[c["E"].real, c["E"].imag]),
                   source="oracle.exact (exact Gaussian-rational inverse of the float inputs)",
                   diag_G=[[z.real, z.imag] for z in dG],
                   diag_Gless=[[z.real, z.imag] for z in dGl],
                   bond_G=[[b[0].real, b[0].imag] for b in bonds],
                   bond_Gless=[[b[1].real, b[1].imag] for b in bonds],
                   bond_J=[b[2] for b in bonds])
        with open(os.path.join(HERE, c["name"] + ".json"), "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
