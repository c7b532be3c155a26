"""find_solve_noalloc, the entry point for callers that cannot allocate
device memory, through the C-ABI: two calls in a row on one plan, the second
with fewer energies, each equal to find_solve's outputs on the same inputs;
the second call leaves the device's free memory unchanged; a plan whose one
energy does not fit the fixed scratch is refused with FIND_E_NOMEM."""
import numpy as np
import pytest

from paper_1104_0623_amd import inputs
from tests.parity import TOL, nrel

pytestmark = pytest.mark.gpu


def find():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1104_0623_amd import find as f
    return f


def test_noalloc_equals_find_solve_on_two_calls():
    import torch
    f = find()
    dev = torch.device("cuda")
    E = inputs.energies_linspace(-3.2, 3.1, 9)
    prob = inputs.make_problem(40, 52, 9, vmax=1.0, seed=7, energies=E, fL=1.0, fR=0.2)
    plan = f.Plan(40, 52, 9)
    ref = f.run_problem(plan, prob, want_bonds=True)       # find_solve (allocating path)
    nb = f.n_bonds(40, 52, 9)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)
    for n in (9, 4):
        ins = [t(prob["energies"][:n]), t(prob["H"]), t(prob["sigma"][:n]), t(prob["sigma_less"][:n])]
        nan = complex(np.nan, np.nan)
        outs = dict(diag_G=torch.full((n, 52, 40), nan, dtype=torch.complex128, device=dev),
                    diag_Gless=torch.full((n, 52, 40), nan, dtype=torch.complex128, device=dev),
                    bond_G=torch.full((n, nb), nan, dtype=torch.complex128, device=dev),
                    bond_Gless=torch.full((n, nb), nan, dtype=torch.complex128, device=dev),
                    bond_J=torch.full((n, nb), np.nan, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        f.solve_noalloc(plan, *ins, outs["diag_G"], outs["diag_Gless"], outs["bond_G"], outs["bond_Gless"],
                        outs["bond_J"])
        f.sync_status(plan)
        free1 = torch.cuda.mem_get_info()[0]
        if n == 4:
            assert free1 == free0, (free0, free1)
        for k, v in outs.items():
            x = v.cpu().numpy()
            for e in range(n):
                assert nrel(x[e], ref[k][e]) <= TOL, (n, k, e)
            assert np.array_equal(x, ref[k][:n]), (n, k)     # the same kernels in the same order


def test_noalloc_refuses_a_plan_larger_than_the_scratch():
    f = find()
    plan = f.Plan(256, 512, 9)          # about 4 GiB per energy
    L = f.lib()
    import ctypes
    p = [ctypes.c_void_p(256)] * 6 + [None] * 3
    assert L.find_solve_noalloc(plan.handle, 1, *p, None) == f.FIND_E_NOMEM
    assert b"scratch" in L.find_last_error()
    small = f.Plan(16, 16, 5)           # fits, but has no tables on the device yet
    assert L.find_solve_noalloc(small.handle, 1, *p, None) == f.FIND_E_ARG
    assert b"find_solve" in L.find_last_error()
