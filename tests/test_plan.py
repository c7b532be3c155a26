"""Plan tests (CPU only): the C-ABI library loads and exports every symbol of
include/find.h; plans have the tree and set structure the paper describes; and
a numpy executor that follows the plan's gather maps reproduces the dense
oracle (so the plan is right before any kernel runs)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import dense
from paper_1104_0623_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def findlib():
    from paper_1104_0623_amd import find
    return find


def test_library_exports_every_declared_symbol():
    find = findlib()
    L = find.lib()
    hdr = open(os.path.join(ROOT, "include", "find.h")).read()
    declared = set(re.findall(r"^\s*(?:find_status|const char\*|int)\s+(find_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(find.EXPORTED), declared ^ set(find.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name


def test_argument_errors():
    find = findlib()
    with pytest.raises(find.FindError) as ei:
        find.Plan(0, 4, 5)
    assert ei.value.status == find.FIND_E_ARG
    with pytest.raises(find.FindError):
        find.Plan(4, 4, 7)
    with pytest.raises(find.FindError):
        find.Plan(4, 4, 5, leaf=-1)
    with pytest.raises(find.FindError):
        find.Plan(4, 4, 5, symmetric=3)
    # fronts beyond the kernels' 4096 nodes are refused at plan creation; those
    # beyond 2048 take the eight-wave form (configuration 7) only
    with pytest.raises(find.FindError) as ei:
        find.Plan(2100, 2, 5)
    assert ei.value.status == find.FIND_E_UNSUPPORTED
    p = find.Plan(1030, 2, 5)
    assert p.summary()["max_n"] > 2048
    ex = p.export()
    tiles, options = p.tiles(), p.tile_options()
    big = 0
    for k, (first, count, phase, variant) in enumerate(ex["stages"]):
        n = max(int(e[3]) for e in ex["elims"][first:first + count])
        if n > 2048:
            assert options[k] == [7] and tiles[k] == 7, (k, n, options[k], tiles[k])
            big += 1
    assert big > 0
    with pytest.raises(find.FindError) as ei:
        find.Plan(4097, 4097, 5)
    assert ei.value.status == find.FIND_E_UNSUPPORTED
    assert find.n_bonds(4, 3, 5) == 3 * 3 + 4 * 2
    assert find.n_bonds(4, 3, 9) == 3 * 3 + 4 * 2 + 2 * 3 * 2
    assert find.n_bonds(0, 3, 9) == -1
    L = find.lib()
    assert L.find_plan_destroy(None) == 0
    assert L.find_solve(None, 1, *([None] * 10)) == find.FIND_E_ARG
    assert b"NULL plan" in L.find_last_error()


def pool_slots(plan, pack):
    """Slots of the energy pool from a plan's export, one per (phase kind,
    cluster): the upward and downward U/R of each cluster, the leaf block
    (both output variants write it) and the final block G.  Returns
    {slot: [start, elements, first stage writing it, last stage reading it]};
    a read of a start belongs to the slot last written there."""
    ex = plan.export()
    el, st = ex["elims"].astype(np.int64), ex["stages"]
    KIND, B, SRC0, SRC1, DST, CLUSTER, PHASE = 0, 2, 4, 6, 8, 10, 11   # exported record fields (find.h)
    blk = lambda b, packed: b * (b + 1) // 2 if packed else b * b
    slots, owner = {}, {}
    for t, (first, count, _, _) in enumerate(st):
        for e in el[first:first + count]:
            for k in (SRC0, SRC1):
                if e[k] >= 0:
                    sid = owner[int(e[k])]          # a read needs an earlier write there
                    slots[sid][3] = max(slots[sid][3], t)
        for e in el[first:first + count]:
            b = int(e[B])
            size = b * b if e[KIND] == 1 else blk(b, pack & 1) + blk(b, pack & 2)
            sid = (int(e[PHASE]), int(e[CLUSTER]))
            rec = slots.setdefault(sid, [int(e[DST]), 0, t, t])
            assert rec[0] == int(e[DST])
            rec[1] = max(rec[1], size)
            owner[int(e[DST])] = sid
    return slots


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", [(64, 64, 5, 8), (33, 20, 9, 4), (16, 16, 5, 2), (24, 40, 5, 4)])
@pytest.mark.parametrize("half_leaves", [False, True])
def test_pool_slots_disjoint_while_live(Nx, Ny, stencil, leaf, half_leaves):
    """The energy pool holds each cluster's U and R from the stage that forms
    them to the last stage that reads them, and slots whose lifetimes overlap
    never share memory; the node diagonal (read by every stage) overlaps no
    slot.  In the symmetric forms U (symmetric = 1), or U and R
    (symmetric = 2), take b (b + 1) / 2 elements (Prop. 1 storage
    reduction), so the pool shrinks form by form."""
    find = findlib()
    sizes = []
    for sym, pack in ((0, 0), (1, 1), (2, 3)):
        plan = find.Plan(Nx, Ny, stencil, leaf=leaf, symmetric=sym, half_leaves=half_leaves)
        pool = plan.summary()["pool_per_energy"]
        sizes.append(pool)
        slots = sorted(tuple(v) for v in pool_slots(plan, pack).values())
        for k, (o, n, b0, d0) in enumerate(slots):
            assert 2 * Nx * Ny <= o and o + n <= pool, (sym, o, n)
            assert b0 <= d0
            for o2, n2, b2, d2 in slots[k + 1:]:
                if o2 >= o + n:
                    break   # sorted by start: no later slot overlaps this one in memory
                assert d0 < b2 or d2 < b0, ("live slots overlap", sym, (o, n, b0, d0), (o2, n2, b2, d2))
    assert sizes[0] > sizes[1] > sizes[2]


def test_pool_lifetimes_halve_the_128_pool():
    """At 128 x 128 (5-point, 8 x 8 leaves) the lifetime placement keeps the
    pool near the upward results plus two downward levels: less than half
    the sum of all slots."""
    find = findlib()
    plan = find.Plan(128, 128, 5)
    total = sum(v[1] for v in pool_slots(plan, 0).values())
    assert plan.summary()["pool_per_energy"] < 0.55 * total


def test_scattering_entry_points_reject_the_other_kind_of_plan():
    """find_solve refuses a scattering plan and find_solve_scattering a plain
    one (argument checks only: no device work, dummy pointers never read)."""
    find = findlib()
    L = find.lib()
    dummy = [ctypes.c_void_p(16)] * 11
    sp = find.Plan(6, 6, 5, scattering=True)
    pp = find.Plan(6, 6, 5)
    assert L.find_solve(sp.handle, 1, *dummy[:9], None) == find.FIND_E_ARG
    assert L.find_solve_scattering(pp.handle, 1, *dummy, None) == find.FIND_E_ARG
    assert L.find_solve_scattering(sp.handle, 1, *dummy[:4], None, *dummy[5:], None) == find.FIND_E_ARG
    assert L.find_solve_scattering(sp.handle, 1, *dummy[:5], None, *dummy[6:], None) == find.FIND_E_ARG
    o = find.PlanOpts(leaf=8, scattering=2)
    h = ctypes.c_void_p()
    assert L.find_plan_create(6, 6, 5, ctypes.byref(o), ctypes.byref(h)) == find.FIND_E_ARG
    # find_solve_scattering_bonds: a plain plan, a missing bond array, 3M
    # complex products (the bond reads are compiled for 4M only)
    d13 = [ctypes.c_void_p(16)] * 13
    assert L.find_solve_scattering_bonds(pp.handle, 1, *d13, None) == find.FIND_E_ARG
    assert L.find_solve_scattering_bonds(sp.handle, 1, *d13[:6], None, *d13[7:], None) == find.FIND_E_ARG
    assert L.find_solve_scattering_bonds(sp.handle, 1, *d13[:7], None, *d13[8:], None) == find.FIND_E_ARG
    p3 = find.Plan(6, 6, 5, scattering=True, complex_mode=find.CPLX_3M)
    assert L.find_solve_scattering_bonds(p3.handle, 1, *d13, None) == find.FIND_E_UNSUPPORTED


def test_tile_and_complex_mode_options():
    find = findlib()
    with pytest.raises(find.FindError) as ei:
        find.Plan(8, 8, 5, complex_mode=2)
    assert ei.value.status == find.FIND_E_ARG
    plan = find.Plan(64, 64, 5, complex_mode=find.CPLX_3M)
    n = plan.summary()["n_stages"]
    assert plan.tiles() == [0] * n
    ex = plan.export()
    stages, elims = ex["stages"], ex["elims"]
    opts = plan.tile_options()
    assert len(opts) == n
    for st, o in zip(stages, opts):
        maxn = int(elims[st[0]:st[0] + st[1], 3].max())
        maxb = int(elims[st[0]:st[0] + st[1], 2].max())
        maxrs = int(elims[st[0]:st[0] + st[1], 14].max())
        final = st[2] == 3
        # Schur stages whose fronts stay <= 512 have the four wave tiles and the
        # workgroup tile; the final leaf blocks only the default; fronts <= 128
        # also the one-wave form, fronts <= 256 the two-wave form; final stages
        # of the diagonal outputs with blocks <= 64 and R_K on <= 28 nodes the
        # Gauss-Jordan form
        gj = final and st[3] == 0 and maxb <= 64 and maxrs <= 28
        want = (([0] if final else [0, 1, 2, 3]) + ([4] if maxn <= 128 else []) + ([5] if maxn <= 256 else [])
                + ([6] if not final and maxn <= 512 else []) + ([] if final else [7]) + ([8] if gj else []))
        assert o == want, (st, maxn, o)
    pick = [o[-1] for o in opts]
    plan.set_tiles(pick)
    assert plan.tiles() == pick
    bad = list(pick)
    k = [i for i, o in enumerate(opts) if 1 not in o][0]
    bad[k] = 1
    with pytest.raises(find.FindError):
        plan.set_tiles(bad)
    with pytest.raises(find.FindError):
        plan.set_tiles(pick[:-1])
    with pytest.raises(find.FindError):
        plan.set_tiles([6] * n)
    assert plan.tiles() == pick          # a rejected call changes nothing
    L = find.lib()
    assert L.find_plan_autotune(None, 1, *([None] * 6), 2, None) == find.FIND_E_ARG
    assert L.find_plan_autotune(plan.handle, 0, *([None] * 6), 2, None) == find.FIND_E_ARG
    assert L.find_plan_set_tiles(plan.handle, None, n) == find.FIND_E_ARG


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", [(12, 20, 5, 3), (9, 16, 9, 4)])
def test_zero_sigma_fronts_are_flagged_exactly(Nx, Ny, stencil, leaf):
    """Upward eliminations flagged R = 0 (the cluster touches neither contact
    column) have an exactly zero R in the definition-level executor, and the
    flop model drops their W and R products."""
    from tests.plan_exec import execute
    find = findlib()
    E = np.array([0.37 + 1e-3j])
    prob = inputs.make_problem(Nx, Ny, stencil, vmax=1.0, seed=4, energies=E, fL=1.0, fR=0.5)
    p = find.Plan(Nx, Ny, stencil, leaf=leaf)
    ex = p.export()
    rec = {}
    Hm = dense.hamiltonian_matrix(Nx, Ny, prob["H"])
    execute(ex, Nx, Ny, stencil, Hm, E[0], prob["sigma"][0], prob["sigma_less"][0], want_bonds=False,
            record=rec)
    el = ex["elims"]
    flagged = [k for k in range(len(el)) if el[k][13] == 1]
    assert flagged, "no front away from the contacts"
    for k in range(len(el)):
        if k not in rec:
            continue
        U, R = rec[k]
        if el[k][13] == 1:
            assert el[k][11] == 0                     # upward pass only
            assert np.all(R == 0), k
        elif el[k][11] == 0 and el[k][0] == 0 and R.size:
            assert np.any(R != 0), k                  # flag is as tight as the structure allows
    # flop model: a flagged elimination counts s^3/3 + s^2 b + s b^2 multiply-adds;
    # the others add b q^2 for W_q and (q + q0) b^2 for R (q0 = q when a kept
    # node carries Sigma<, else 0)
    ok = 0.0
    for first, count, phase, var in ex["stages"]:
        if var == 1:
            continue
        for k in range(first, first + count):
            kind, s_, q_, q0 = el[k][0], float(el[k][1]), float(el[k][14]), float(el[k][15])
            b_ = float(el[k][16]) if kind == 0 else float(el[k][2])
            if kind == 1:
                ok += 8 * (s_ ** 3 + q_ ** 2 * s_)
            elif el[k][13]:
                ok += 8 * (s_ ** 3 / 3 + s_ ** 2 * b_ + s_ * b_ ** 2)
            else:
                ok += 8 * (s_ ** 3 / 3 + s_ ** 2 * b_ + s_ * b_ ** 2 + b_ * q_ ** 2 + (q_ + q0 * q_) * b_ ** 2)
    assert abs(p.flops_per_energy(False) - ok) <= 1e-9 * ok


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", [(12, 20, 5, 3), (9, 16, 9, 4), (16, 16, 5, 8), (5, 7, 5, 2)])
def test_sigma_support_prefix_is_exact(Nx, Ny, stencil, leaf):
    """The plan puts the eliminated nodes that carry Sigma< first in S (ssig of
    them) and flags whether a kept node carries it: in the definition-level
    executor the assembled Sigma_g has exactly zero rows and columns for the
    other eliminated nodes, and for the kept nodes when the flag is 0.  These
    are the zeros the kernels skip."""
    from tests.plan_exec import execute
    find = findlib()
    E = np.array([-0.83 + 1e-3j])
    prob = inputs.make_problem(Nx, Ny, stencil, vmax=1.0, seed=11, energies=E, fL=0.7, fR=0.4)
    p = find.Plan(Nx, Ny, stencil, leaf=leaf)
    ex = p.export()
    fronts, rec = {}, {}
    Hm = dense.hamiltonian_matrix(Nx, Ny, prob["H"])
    for bonds in (False, True):
        execute(ex, Nx, Ny, stencil, Hm, E[0], prob["sigma"][0], prob["sigma_less"][0], want_bonds=bonds,
                fronts=fronts, record=rec)
    el = ex["elims"]
    # final leaf blocks: R_K vanishes outside its first ssig rows and columns
    # (the final stage follows its leaf-extraction stage, leaf by leaf)
    st = [tuple(x) for x in ex["stages"]]
    for i, (first, count, phase, var) in enumerate(st):
        if phase != 3:
            continue
        lfirst = st[i - 1][0]
        assert st[i - 1][2] == 2 and st[i - 1][1] == count
        for q in range(count):
            k, j = first + q, lfirst + q
            R = rec[j][1]
            rs = el[k][14]
            assert el[k][2] == R.shape[0] and 0 <= rs <= R.shape[0]
            assert np.all(R[rs:, :] == 0) and np.all(R[:, rs:] == 0), (k, rs)
    partial = inert = 0
    for k, (Ag, Sg) in fronts.items():
        kind, s_, b_, rz, q, bs, ba = (el[k][0], el[k][1], el[k][2], el[k][13], el[k][14], el[k][15],
                                       el[k][16])
        assert kind == 0
        # kept nodes past the first ba are not coupled to S in A_g or Sigma_g
        assert 0 <= ba <= b_ and (ba == b_ or el[k][11] == 2), k     # (reordered in leaf extraction only)
        na = s_ + ba
        for M in (Ag, Sg):
            assert np.all(M[na:, :s_] == 0) and np.all(M[:s_, na:] == 0), k
        inert += b_ - ba
        if rz:
            assert np.all(Sg == 0), k
            continue
        assert 0 <= q <= s_
        assert np.all(Sg[q:s_, :] == 0) and np.all(Sg[:, q:s_] == 0), k
        if not bs:
            assert np.all(Sg[s_:na, :s_] == 0) and np.all(Sg[:s_, s_:na] == 0), k
        # the support is tracked per node through the stored R blocks, so it is
        # tight: every eliminated node counted in q has a non-zero row
        assert np.all(np.any(Sg[:q, :] != 0, axis=1)), k
        partial += q < s_
    assert partial > 0, "no front with a partial Sigma support"
    assert inert > 0, "no kept node uncoupled from S"



def test_tree_shape_128():
    find = findlib()
    p = find.Plan(128, 128, 5)
    s = p.summary()
    assert (s["n_clusters"], s["depth"], s["n_leaves"]) == (511, 8, 256)
    ex = p.export()
    el = ex["elims"]
    up = el[el[:, 11] == 0]; dn = el[el[:, 11] == 1]
    # upward level 1 merges two 128 x 64 halves: S = the two middle columns, B = both contact columns
    l1 = up[up[:, 12] == 1]
    assert set(l1[:, 1]) == {252} and set(l1[:, 2]) == {128}
    leaves = up[up[:, 12] == 8]
    assert leaves[:, 1].min() == 36 and leaves[:, 1].max() == 42
    assert leaves[:, 2].min() == 22 and leaves[:, 2].max() == 28
    d1 = dn[dn[:, 12] == 1]
    assert set(d1[:, 1]) == {0} and set(d1[:, 2]) == {128}
    d3 = dn[dn[:, 12] == 3]
    assert d3[:, 1].max() == 190 and d3[:, 2].max() == 160
    # dense-per-front count with the Sigma< support skipped (about 15.3 GFLOP
    # per energy if every front carried Sigma< on all its nodes)
    assert 10e9 < p.flops_per_energy() < 14e9


def test_tree_shape_small_and_degenerate():
    find = findlib()
    s = find.Plan(16, 16, 5).summary()
    assert (s["n_clusters"], s["depth"], s["n_leaves"]) == (7, 2, 4)
    s = find.Plan(5, 3, 5).summary()     # whole mesh is one leaf
    assert (s["n_clusters"], s["depth"], s["n_leaves"]) == (1, 0, 1)
    s = find.Plan(1, 40, 5).summary()    # 1D chain
    assert s["n_leaves"] == 8


CASES = [(16, 16, 5, 8), (12, 9, 9, 4), (7, 13, 5, 3), (1, 11, 5, 2), (4, 3, 9, 8), (9, 1, 5, 2),
         (10, 10, 9, 2), (6, 17, 5, 4)]


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", CASES)
@pytest.mark.parametrize("want_bonds", [False, True])
def test_plan_executor_matches_oracle(Nx, Ny, stencil, leaf, want_bonds):
    from tests.plan_exec import execute
    find = findlib()
    E = 0.41 + 1e-3j
    prob = inputs.make_problem(Nx, Ny, stencil, vmax=0.8, seed=Nx * 31 + Ny, energies=[E], fL=1.0, fR=0.2)
    p = find.Plan(Nx, Ny, stencil, leaf=leaf)
    Hm = dense.hamiltonian_matrix(Nx, Ny, prob["H"])
    dG, dL, bG, bL, bJ = execute(p.export(), Nx, Ny, stencil, Hm, E, prob["sigma"][0], prob["sigma_less"][0],
                                 want_bonds)
    ref = dense.dense_solve(Nx, Ny, stencil, prob["H"], prob["energies"], prob["sigma"], prob["sigma_less"])
    sc = np.max(np.abs(ref["diag_G"][0]))
    assert np.max(np.abs(dG - ref["diag_G"][0])) < 1e-11 * sc
    assert np.max(np.abs(dL - ref["diag_Gless"][0])) < 1e-11 * np.max(np.abs(ref["diag_Gless"][0]))
    if want_bonds:
        nb = inputs.n_bonds(Nx, Ny, stencil)
        assert sorted(bG) == list(range(nb))
        g = np.array([bG[k] for k in range(nb)]); l = np.array([bL[k] for k in range(nb)])
        assert np.max(np.abs(g - ref["bond_G"][0])) < 1e-11 * sc
        assert np.max(np.abs(l - ref["bond_Gless"][0])) < 1e-11 * np.max(np.abs(ref["bond_Gless"][0]))
        # J from the G<_ji entry the output record points at
        H = prob["H"]
        J = np.array([2 * np.real(H[bJ[k][2]].ravel()[bJ[k][3]] * bJ[k][4]) for k in range(nb)])
        assert np.max(np.abs(J - ref["bond_J"][0])) < 1e-10 * (np.max(np.abs(ref["bond_J"][0])) + 1e-3)


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", [(12, 9, 9, 4), (16, 16, 5, 8), (7, 13, 5, 3)])
def test_scattering_plan_executor_matches_oracle(Nx, Ny, stencil, leaf):
    """A plan for diagonal scattering self-energies (every node carries Sigma<:
    no front flagged R = 0, every eliminated node in the Sigma prefix) gives
    the oracle's outputs through the definition-level executor, and its
    assembled fronts keep the zeros the flags promise."""
    from tests.plan_exec import execute
    find = findlib()
    E = 0.41 + 1e-3j
    prob = inputs.make_problem(Nx, Ny, stencil, vmax=0.8, seed=Nx * 7 + Ny, energies=[E], fL=1.0, fR=0.2)
    sd, sl = inputs.scattering_self_energies(Nx, Ny, 1, gamma=0.06, f=0.3, seed=5)
    p = find.Plan(Nx, Ny, stencil, leaf=leaf, scattering=True)
    ex = p.export()
    el = ex["elims"]
    schur = el[el[:, 0] == 0]
    assert not np.any(schur[:, 13]) and np.all(schur[:, 14] == schur[:, 1])
    Hm = dense.hamiltonian_matrix(Nx, Ny, prob["H"])
    fronts = {}
    dG, dL, bG, bL, bJ = execute(ex, Nx, Ny, stencil, Hm, E, prob["sigma"][0], prob["sigma_less"][0], True,
                                 fronts=fronts, sd=sd[0].reshape(-1), sld=sl[0].reshape(-1))
    ref = dense.dense_solve(Nx, Ny, stencil, prob["H"], prob["energies"], prob["sigma"], prob["sigma_less"],
                            sigma_d=sd, sigma_less_d=sl)
    assert np.max(np.abs(dG - ref["diag_G"][0])) < 1e-11 * np.max(np.abs(ref["diag_G"][0]))
    assert np.max(np.abs(dL - ref["diag_Gless"][0])) < 1e-11 * np.max(np.abs(ref["diag_Gless"][0]))
    nb = inputs.n_bonds(Nx, Ny, stencil)
    l = np.array([bL[k] for k in range(nb)])
    assert np.max(np.abs(l - ref["bond_Gless"][0])) < 1e-11 * np.max(np.abs(ref["bond_Gless"][0]))
    for k, (Ag, Sg) in fronts.items():
        s_, b_, ba = el[k][1], el[k][2], el[k][16]
        na = s_ + ba
        for M in (Ag, Sg):
            assert np.all(M[na:, :s_] == 0) and np.all(M[:s_, na:] == 0), k


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", [(12, 20, 5, 3), (9, 16, 9, 4), (16, 16, 5, 8), (7, 13, 5, 3)])
def test_schur_blocks_independent_of_elimination_order(Nx, Ny, stencil, leaf):
    """Theorem 1 and its corollaries (Sec. 2.2 and the appendix's final
    conclusion): the U and R each elimination of the plan produces depend
    only on which nodes have been eliminated, not on the order.  Every U_g
    (and R_g) of the tree-ordered, level-by-level executor equals the Schur
    complement onto B_g taken in one step from the original A (and Sigma<)
    over all nodes eliminated below it, for the upward clusters, the
    complement clusters and the leaf extraction fronts alike."""
    from tests.plan_exec import execute
    find = findlib()
    E = 0.29 + 1e-3j
    prob = inputs.make_problem(Nx, Ny, stencil, vmax=0.8, seed=Nx * 3 + Ny, energies=[E], fL=1.0, fR=0.4)
    p = find.Plan(Nx, Ny, stencil, leaf=leaf)
    ex = p.export()
    el, maps = ex["elims"], ex["maps"]
    Hm = dense.hamiltonian_matrix(Nx, Ny, prob["H"])
    rec = {}
    for bonds in (False, True):
        execute(ex, Nx, Ny, stencil, Hm, E, prob["sigma"][0], prob["sigma_less"][0], want_bonds=bonds, record=rec)
    A = dense.dense_A(Nx, Ny, prob["H"], E, prob["sigma"][0])
    Sl = dense.embed_contacts(Nx, Ny, prob["sigma_less"][0])
    # pool slots are reused once dead: a source is the last elimination
    # before the reader (in stage order) that wrote its offset
    by_dst = {}
    for k in range(len(el)):
        if el[k][0] == 0:
            by_dst.setdefault(int(el[k][8]), []).append(k)
    elim_set = {}

    def source(k, off):
        return max(j for j in by_dst[off] if j < k)

    def eliminated(k):
        if k not in elim_set:
            s_, n_, mp = el[k][1], el[k][3], el[k][9]
            out = set(maps[mp: mp + s_, 0].tolist())
            for f_ in (4, 6):
                if el[k][f_] >= 0:
                    out |= eliminated(source(k, int(el[k][f_])))
            elim_set[k] = out
        return elim_set[k]

    checked = {0: 0, 1: 0, 2: 0}
    for k in range(len(el)):
        if el[k][0] != 0 or k not in rec:
            continue
        s_, n_, mp = el[k][1], el[k][3], el[k][9]
        B = maps[mp + s_: mp + n_, 0]
        I = np.array(sorted(eliminated(k)), dtype=int)
        assert not set(I.tolist()) & set(B.tolist())
        Lm = np.linalg.solve(A[np.ix_(I, I)].T, A[np.ix_(B, I)].T).T if I.size else np.zeros((B.size, 0))
        U = A[np.ix_(B, B)] - Lm @ A[np.ix_(I, B)]
        R = (Sl[np.ix_(B, B)] - Lm @ Sl[np.ix_(I, B)] - Sl[np.ix_(B, I)] @ Lm.conj().T
             + Lm @ Sl[np.ix_(I, I)] @ Lm.conj().T)
        Uk, Rk = rec[k]
        assert np.max(np.abs(Uk - U)) <= 1e-10 * max(1.0, np.max(np.abs(U))), k
        assert np.max(np.abs(Rk - R)) <= 1e-10 * max(1.0, np.max(np.abs(R))), k
        checked[int(el[k][11])] += 1
    assert all(v > 0 for v in checked.values()), checked
    # the leaf-extraction fronts eliminate every node outside their kept set
    for k in range(len(el)):
        if el[k][0] == 0 and el[k][11] == 2 and k in rec:
            assert len(eliminated(k)) + el[k][2] == Nx * Ny, k


def test_solve_rejects_scattering_inputs_for_a_plain_plan():
    """A contacts-only plan refuses Sigma_d / Sigma<_d instead of ignoring them
    (checked before any device work)."""
    find = findlib()
    plan = find.Plan(6, 6, 5)
    with pytest.raises(ValueError):
        find.solve(plan, None, None, None, None, None, None, sigma_d=object(), sigma_less_d=object())
    with pytest.raises(ValueError):
        find.solve(plan, None, None, None, None, None, None, sigma_b=object(), sigma_less_b=object())
    with pytest.raises(ValueError):   # the two bond arrays go together
        find.solve(find.Plan(6, 6, 5, scattering=True), None, None, None, None, None, None,
                   sigma_d=object(), sigma_less_d=object(), sigma_b=object())


@pytest.mark.parametrize("Nx,Ny,stencil,leaf", [(16, 16, 5, 2), (12, 10, 5, 2), (9, 14, 5, 2), (8, 8, 5, 1),
                                                (10, 12, 9, 2), (12, 16, 5, 4), (1, 11, 5, 2), (7, 6, 5, 2)])
@pytest.mark.parametrize("want_bonds", [False, True])
def test_half_leaf_extraction_matches_oracle(Nx, Ny, stencil, leaf, want_bonds):
    """Current density from half of the leaves (Sec. 4.3, Fig. cd-opt): the
    chosen leaves keep the ring around them and output its diagonal and bond
    entries; every node and bond is output exactly once; the definition-level
    executor of the plan gives the dense oracle's values.  With 2 x 2 leaves
    and the 5-point stencil about half of the leaves run the extraction."""
    from tests.plan_exec import execute
    find = findlib()
    E = 0.37 + 1e-3j
    prob = inputs.make_problem(Nx, Ny, stencil, vmax=0.8, seed=Nx * 11 + Ny, energies=[E], fL=1.0, fR=0.3)
    p = find.Plan(Nx, Ny, stencil, leaf=leaf, half_leaves=True)
    full = find.Plan(Nx, Ny, stencil, leaf=leaf)
    ex = p.export()
    var = 1 if want_bonds else 0
    lo = ex["leafout"][ex["leafout"][:, 5] == var]
    nodes = np.concatenate([ex["outnodes"][r[2]: r[2] + r[1], 0] for r in lo])
    assert sorted(nodes.tolist()) == list(range(Nx * Ny))           # every node exactly once
    if want_bonds:
        bonds = np.concatenate([ex["outbonds"][r[3]: r[3] + r[4], 0] for r in lo])
        assert sorted(bonds.tolist()) == list(range(inputs.n_bonds(Nx, Ny, stencil)))
    n_leaves = p.summary()["n_leaves"]
    if stencil == 5 and leaf == 2 and Nx % 4 == 0 and Ny % 4 == 0:
        # the checkerboard, plus the skipped leaves on the mesh edge (their
        # edge-side bond has no chosen neighbour beyond the edge)
        assert len(lo) <= n_leaves // 2 + Nx // 2 + Ny // 2, (len(lo), n_leaves)
    Hm = dense.hamiltonian_matrix(Nx, Ny, prob["H"])
    dG, dL, bG, bL, bJ = execute(ex, Nx, Ny, stencil, Hm, E, prob["sigma"][0], prob["sigma_less"][0], want_bonds)
    ref = dense.dense_solve(Nx, Ny, stencil, prob["H"], prob["energies"], prob["sigma"], prob["sigma_less"])
    sc = np.max(np.abs(ref["diag_G"][0]))
    assert np.max(np.abs(dG - ref["diag_G"][0])) < 1e-11 * sc
    assert np.max(np.abs(dL - ref["diag_Gless"][0])) < 1e-11 * np.max(np.abs(ref["diag_Gless"][0]))
    if want_bonds:
        nb = inputs.n_bonds(Nx, Ny, stencil)
        g = np.array([bG[k] for k in range(nb)]); l_ = np.array([bL[k] for k in range(nb)])
        assert np.max(np.abs(g - ref["bond_G"][0])) < 1e-11 * sc
        assert np.max(np.abs(l_ - ref["bond_Gless"][0])) < 1e-11 * np.max(np.abs(ref["bond_Gless"][0]))
    # the flop model counts fewer final-stage flops than extracting every leaf
    if stencil == 5 and leaf <= 2 and Nx * Ny >= 64:
        assert p.flops_per_energy(want_bonds) < full.flops_per_energy(want_bonds)


def test_closed_device_plan_matches_table_null_boundary_cost():
    """Table NullBoundaryCost (appendix; Sec. 4.4 for the physical boundary):
    for an N x N 5-point mesh with no contacts, per tree level (root = level
    0), the summed cost s^3/3 + s^2 b + s b^2 of the upward and downward
    eliminations in units of N^3.  The table is exact for the large clusters
    near the root (levels 1-4) and an estimate that ignores the physical
    boundary for the smaller ones, so the plan's levels 1-4 must match within
    15% and its levels 5 and 6 may not exceed the table's."""
    find = findlib()
    N = 256
    up_tab = {1: 4.666, 2: 9.332, 3: 2.040 + 4.540, 4: 3.168 + 4.080 + 1.168,
              5: 0.2552 + 0.3958 + 1.703 + 2.312, 6: 6.336}
    dn_tab = {2: 9.332, 3: 14.624 + 4.540, 4: 4.332 + 2.040 + 14.624 + 9.332, 5: 52.672, 6: 38.976}
    el = find.Plan(N, N, 5, no_contacts=True).export()["elims"]
    up, dn = {}, {}
    for r in el:
        if r[0] != 0 or r[11] not in (0, 1):
            continue
        s, b = r[1] / N, r[2] / N
        d = up if r[11] == 0 else dn
        d[int(r[12])] = d.get(int(r[12]), 0.0) + s ** 3 / 3 + s * s * b + s * b * b
    assert dn.get(1, 0.0) == 0.0                       # level 1: the root's halves eliminate nothing
    for tab, got in ((up_tab, up), (dn_tab, dn)):
        for lev, c in tab.items():
            if lev <= 4:
                assert abs(got[lev] - c) <= 0.15 * c, (lev, got[lev], c)
            else:
                assert got[lev] <= c, (lev, got[lev], c)
    # with contacts the contact columns join the boundary sets: more work
    with_contacts = find.Plan(N, N, 5).export()["elims"]
    cost = lambda E: sum(float(r[1]) ** 3 / 3 + float(r[1]) ** 2 * r[2] + float(r[1]) * float(r[2]) ** 2
                         for r in E if r[0] == 0)
    assert cost(with_contacts) > cost(el)
