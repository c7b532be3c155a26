"""Benchmark: energy-point solves/s of the FIND hot path on one MI355X.

Workload (default): 128 x 128 mesh, 5-point stencil, on-site V ~ U[-1, 1]
(seed 0), 256 energies linspace(-3.5, 3.5) + 1e-6 i, f_L = 1, f_R = 0; one
step = one solve of the whole 256-energy batch (diag G + diag G<), inputs
resident in HBM.  Prints one JSON line (see the repository's DESIGN notes for
the roofline and CPU-baseline definitions).

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--precision fp64|mixed|mixed-gless]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X dense MFMA TFLOP/s: FP64, FP32 for the form whose Schur products are all
# FP32, FP64 for the one that keeps U in FP64 (most of its flops)
PEAK = {"fp64": 78.6, "mixed": 157.3, "mixed-gless": 78.6}
PRECISION = {"fp64": 0, "mixed": 1, "mixed-gless": 2}   # find_precision values

# HBM bytes per elimination-kernel launch of the 128x128 x 256-energy FP64
# solve, from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs (calibrated on a
# plain copy; profiles/elim_kernels_c3_128x128_fp64.md).  Valid only for the
# native sources (kernels, plan, C-ABI) they were measured on.
TRAFFIC_BYTES_PER_LAUNCH = 31470178020.38
TRAFFIC_KERNEL_SHA = "d7bcad8cff15fdad"
TRAFFIC_TILES = "445510763600105141418000"
TRAFFIC_FORM = (0, 1)   # (symmetric form, energy groups) of the counter runs


def native_source_sha() -> str:
    """sha256 prefix over the native sources (csrc/*, sorted by name)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1104_0623_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        h.update(name.encode())
        h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(preset: str, precision: str, tiles: str, cmode: str, form: tuple):
    sha = native_source_sha()
    if (sha != TRAFFIC_KERNEL_SHA or tiles != TRAFFIC_TILES or preset != "c3_128x128" or precision != "fp64"
            or cmode != "4m" or form != TRAFFIC_FORM):
        return None
    return TRAFFIC_BYTES_PER_LAUNCH


def plain_find_flops(plan) -> float:
    """Flops per energy of the plain dense-per-front FIND on the same tree
    (diagonal outputs): 8 (s^3/3 + 2 s^2 b + 3 s b^2) per elimination and 16 b^3
    per final leaf block, with no structural zero left out and nothing halved."""
    ex = plan.export()
    el = ex["elims"].astype(float)
    total = 0.0
    for first, count, phase, var in ex["stages"]:
        if var not in (-1, 0):
            continue
        for k in range(first, first + count):
            s_, b_ = el[k][1], el[k][2]
            total += 16 * b_ ** 3 if el[k][0] == 1 else 8 * (s_ ** 3 / 3 + 2 * s_ * s_ * b_ + 3 * s_ * b_ * b_)
    return total


def cpu_baseline(prob: dict, budget_s: float = 12.0, scat: dict | None = None) -> dict:
    """The RGF oracle, timed on this host over a bounded sample of the same
    workload's energies (one energy at a time until ~budget_s of work)."""
    import numpy as np
    from oracle import rgf
    try:
        import threadpoolctl
        threads = max(int(i.get("num_threads", 1)) for i in threadpoolctl.threadpool_info())
    except Exception:
        threads = os.cpu_count() or 1
    Nx, Ny, st = prob["Nx"], prob["Ny"], prob["stencil"]
    E = prob["energies"]
    order = np.random.default_rng(1).permutation(E.size)
    t0 = time.perf_counter()
    done = 0
    for e in order:
        sc = {k: v[e:e + 1] for k, v in scat.items()} if scat else {}
        rgf.rgf_solve(Nx, Ny, st, prob["H"], E[e:e + 1], prob["sigma"][e:e + 1], prob["sigma_less"][e:e + 1],
                      bonds=False, **sc)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"RGF oracle (numpy/OpenBLAS, complex128) on {done} of the {E.size} energies of the "
                      f"same {Nx}x{Ny} workload{', with the scattering self-energies' if scat else ''}, {dt:.1f} s"}


def serve_bench(args) -> dict:
    """Serving: a bounded Poisson trace of uneven (mesh, energies) requests,
    served with continuous batching, in the plain FP64 and the mixed form."""
    import torch
    from paper_1104_0623_amd import find
    from paper_1104_0623_amd.serve import GpuExecutor, Server, poisson_trace
    res = {}
    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    for prec_name in args.serve_precisions.split(","):
        prec = PRECISION[prec_name]
        for rate in rates:
            trace = poisson_trace(args.serve_requests, rate=rate, seed=0)
            ex = GpuExecutor(n_slots=args.slots, precision=prec, plan_budget=16 << 30, cache_limit=96 << 30,
                             keep_outputs=False, symmetric=args.symmetric)
            # warm the plan cache (host trees, device maps) outside the timed trace
            for key in sorted({r.key for r in trace}):
                plan = ex.cache.take(key)
                ex.cache.give(key, plan, plan.footprint(64), 0)
            srv = Server(ex, n_slots=args.slots, hbm_budget=160 << 30)
            srv.run(trace)
            torch.cuda.synchronize()
            st = srv.stats()
            st["rate_req_per_s"] = rate
            res.setdefault(prec_name, []).append(st)
            print(json.dumps({"serving": prec_name, **st}), file=sys.stderr, flush=True)
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed-gless"], default="fp64")
    ap.add_argument("--preset", default="c3_128x128")
    ap.add_argument("--leaf", type=int, default=8, help="largest leaf-cluster side of the tree")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark (Poisson trace of mixed meshes) instead of the batched solve")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--rates", default="", help="comma-separated arrival rates for a sweep")
    ap.add_argument("--serve-requests", type=int, default=40)
    ap.add_argument("--serve-precisions", default="fp64,mixed-gless",
                    help="comma-separated forms served in turn (fp64, mixed, mixed-gless)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--no-serve-summary", action="store_true",
                    help="skip the short serving traces (Poisson arrivals at 200 and 4 requests/s, FP64 and the "
                         "G<-only mixed form) whose p50/p99 latency the benchmark line carries")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch each step eagerly instead of replaying one captured hipGraph")
    ap.add_argument("--complex-mode", choices=["4m", "3m"], default="4m",
                    help="real split of the complex Schur products")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default wave tile (32x32) for every stage instead of tuning it")
    ap.add_argument("--symmetric", type=int, nargs="?", const=1, default=0, choices=[0, 1, 2],
                    help="assert that A is complex symmetric (true for these inputs): 1 forms and stores only "
                         "the lower half of each U, 2 also of each R (about half the energy pool; G< loses "
                         "accuracy near resonances).  By default the general form runs (it keeps the 1e-10 "
                         "accuracy at the ill-conditioned energies where the mirrored U loses a factor of a few)")
    ap.add_argument("--streams", type=int, default=1,
                    help="energy groups solved concurrently (0/1 = one; with the stages split by front size, "
                         "one group measured about 1%% faster than two)")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="device memory the plan may hold, GB (0 = the library default of 64 GiB); energies "
                         "are solved in passes that fit it")
    ap.add_argument("--bonds", action="store_true",
                    help="also return G and G< on every bond and the bond currents (the leaf extraction "
                         "keeps the bonds' far ends)")
    ap.add_argument("--half-leaves", action="store_true",
                    help="current density from half of the leaves: a checkerboard of leaves extracts the "
                         "ring around it too, the others none (useful with --leaf 2)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner even if the tuning table has an entry for this workload")
    ap.add_argument("--scattering", action="store_true",
                    help="add diagonal scattering self-energies on every node (dephasing probes, gamma = 0.05) "
                         "and solve with find_solve_scattering")
    ap.add_argument("--scattering-bonds", action="store_true",
                    help="with --scattering, also stencil-pattern scattering self-energies on every bond "
                         "(find_solve_scattering_bonds; the non-final stages then run the 32x32 wave tile)")
    ap.add_argument("--tiles", default="",
                    help="fixed wave tile per stage (one digit per stage, as reported in config.stage_tiles); "
                         "skips the autotuner")
    args = ap.parse_args()
    if args.scattering_bonds:
        args.scattering = True
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); energies "
              "would shard across GPUs with no exchange in the hot loop, but that path is not built.",
              file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_1104_0623_amd import find, inputs

    if args.serve:
        res = serve_bench(args)
        best = res["fp64"][0]
        out = {"metric": "energy-point solves/s under a Poisson request stream; p50/p99 latency",
               "value": best["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
               "steps": best["requests"], "warmup": 0, "ms_per_step": best["makespan_s"] * 1e3 / best["requests"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"serving: {args.serve_requests} requests, Poisson {args.rates or args.rate}/s, "
                                      "Nx in {32,64,128,256}, Ny in {Nx,2Nx}, 5/9-point, 1-64 energies",
                          "slots": args.slots},
               "serving": res}
        print(json.dumps(out), flush=True)
        return 0

    prob = inputs.make_preset(args.preset)
    Nx, Ny, st = prob["Nx"], prob["Ny"], prob["stencil"]
    nE = prob["energies"].size
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    E = torch.as_tensor(prob["energies"], device=dev)
    H = torch.as_tensor(prob["H"], device=dev)
    S = torch.as_tensor(prob["sigma"], device=dev)
    SL = torch.as_tensor(prob["sigma_less"], device=dev)
    dG = torch.empty((nE, Ny, Nx), dtype=torch.complex128, device=dev)
    dL = torch.empty_like(dG)
    scat, scat_np = {}, None
    if args.scattering:
        sd, sl = inputs.scattering_self_energies(Nx, Ny, nE, gamma=0.05, f=0.5, seed=0)
        scat_np = dict(sigma_d=sd, sigma_less_d=sl)
        if args.scattering_bonds:
            sb, slb = inputs.bond_scattering_self_energies(Nx, Ny, st, nE, seed=1)
            scat_np.update(sigma_b=sb, sigma_less_b=slb)
        scat = {k: torch.as_tensor(v, device=dev) for k, v in scat_np.items()}
    prec = PRECISION[args.precision]
    cmode = find.CPLX_3M if args.complex_mode == "3m" else find.CPLX_4M
    plan = find.Plan(Nx, Ny, st, leaf=args.leaf, precision=prec, complex_mode=cmode, symmetric=args.symmetric,
                     streams=args.streams, scattering=args.scattering, half_leaves=args.half_leaves,
                     workspace_budget=int(args.budget_gb * 1e9))
    plain_flops = plain_find_flops(plan)
    stream = torch.cuda.Stream()          # non-default stream (graph capture needs one)
    torch.cuda.set_stream(stream)
    tune_s = 0.0
    key = f"{Nx}x{Ny}/{st}/{args.leaf}/{args.precision}/{args.complex_mode}" + \
        {0: "", 1: "/sym", 2: "/sym2"}[args.symmetric]
    table = json.load(open(os.path.join(ROOT, "paper_1104_0623_amd", "tuning.json")))
    tiles_from = "autotune"
    if args.scattering:
        # every node carries Sigma<: the final blocks' R_K support differs from
        # the contacts-only plan's, so scattering plans have entries of their
        # own (tuned on the spot when there is none)
        key += "/scat"
    if not args.tiles and not args.autotune and not args.no_autotune and key in table:
        args.tiles, tiles_from = table[key], "tuning table"
    if args.tiles:
        plan.set_tiles([int(c) for c in args.tiles])
        tiles_from = tiles_from if tiles_from == "tuning table" else "--tiles"
    elif args.no_autotune:
        tiles_from = "default"
    else:
        # per-stage wave tiles picked by timing each configuration once on this batch
        # (a one-off plan setup, outside the timed region)
        t = time.perf_counter()
        find.autotune(plan, E, H, S, SL, dG, dL, reps=1, stream=stream)
        tune_s = time.perf_counter() - t
    tiles = plan.tiles()

    bond_out = {}
    if args.bonds:
        nb = find.n_bonds(Nx, Ny, st)
        bond_out = dict(bond_G=torch.empty((nE, nb), dtype=torch.complex128, device=dev),
                        bond_Gless=torch.empty((nE, nb), dtype=torch.complex128, device=dev),
                        bond_J=torch.empty((nE, nb), dtype=torch.float64, device=dev))

    def eager_step():
        find.solve(plan, E, H, S, SL, dG, dL, stream=stream, **bond_out, **scat)

    for _ in range(max(1, args.warmup)):
        eager_step()
    find.sync_status(plan, stream)
    # elimination launches per step, counted on one profiled eager step (a
    # captured graph replays the same launches)
    plan.set_profiling(True)
    eager_step()
    torch.cuda.synchronize()
    launches_per_step = plan.profile()[2]
    plan.set_profiling(False)
    if args.no_graph:
        # the library records a HIP event pair around every stage launch
        plan.set_profiling(True)
        step = eager_step
    else:
        # one captured hipGraph per 256-energy batch (HIP cannot time events
        # recorded inside a graph, so the replay is timed from the stream: the
        # graph holds only the stage kernels and a 1-block status fill)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            eager_step()
        torch.cuda.synchronize()

        def step():
            graph.replay()
    torch.cuda.synchronize()
    lat = []
    kms = kflops = 0.0
    nl = 0
    flops_step = plan.flops_per_energy(args.bonds) * nE
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        if args.no_graph:
            step()
            torch.cuda.synchronize()
            m, fl, n = plan.profile()   # kernel time of this step
        else:
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            step()
            ev1.record(stream)
            torch.cuda.synchronize()
            m, fl, n = ev0.elapsed_time(ev1), flops_step, 0
        lat.append(time.perf_counter() - ts)
        kms += m; kflops += fl; nl += n
    elapsed = time.perf_counter() - t0
    plan.set_profiling(False)
    find.sync_status(plan, stream)
    value = nE * args.steps / elapsed
    achieved = kflops / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    lat_ms = np.array(lat) * 1e3
    peak = PEAK[args.precision]
    out = {
        "metric": "energy-point solves/s (diag G + G<) at 128x128 mesh; p50/p99 latency",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"FIND diag G + diag G<{' + bond G, G<, J' if args.bonds else ''}, {Nx}x{Ny} mesh, "
                               f"{st}-point stencil, {nE} energies per step ({args.preset}), {args.precision}"
                               + (", diagonal scattering self-energies on every node" if args.scattering else "")
                               + (" and stencil-pattern ones on every bond" if args.scattering_bonds else "")
                               + (", leaf extraction on half of the leaves" if args.half_leaves else ""),
                   "scattering": bool(args.scattering), "scattering_bonds": bool(args.scattering_bonds),
                   "bonds": bool(args.bonds),
                   "half_leaves": bool(args.half_leaves),
                   "Nx": Nx, "Ny": Ny, "stencil": st, "energies_per_step": nE, "precision": args.precision,
                   "leaf": args.leaf, "complex_mode": args.complex_mode, "symmetric": args.symmetric, "streams": args.streams,
                   "pool_MB_per_energy": round(plan.summary()["pool_per_energy"] * 16 / 1e6, 2),
                   "plan_footprint_GB": round(plan.footprint(nE) / 1e9, 2),
                   "launch": "eager" if args.no_graph else "hipGraph replay per batch",
                   "stage_tiles": "".join(str(t) for t in tiles),
                   "stage_tiles_from": tiles_from,
                   **({"stage_tiles_note": "with bond self-energies, non-final stages whose tile is 1, 2, 3 "
                                           "or 6 run configuration 0 instead (7 where only the eight-wave form "
                                           "fits); the others as listed"}
                      if args.scattering_bonds else {}),
                   "autotune_s": round(tune_s, 3) if tiles_from == "autotune" else None},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None if args.scattering else measured_traffic(args.preset, args.precision, "".join(str(t) for t in tiles),
                                                                 args.complex_mode,
                                                                 (args.symmetric, max(1, args.streams))),
                     "kernel": "k_stage + k_final (elimination kernels, all stage launches)",
                     "timing": "HIP events per stage launch" if args.no_graph else "HIP events around each graph replay",
                     "launches_per_step": launches_per_step, "kernel_ms_per_step": kms / args.steps,
                     "algorithmic_flops_per_step": kflops / args.steps,
                     # context: the plain dense-per-front FIND's work on the same tree per
                     # step, over the same kernel time (the rate this run delivers in
                     # plain-FIND work; achieved/frac above are on the form's own count)
                     "plain_find_flops_per_step": plain_flops * nE,
                     "plain_find_equivalent_TFLOPs": plain_flops * nE * args.steps / (kms * 1e9)},
    }
    if not args.no_serve_summary and args.preset == "c3_128x128" and not args.scattering:
        # serving: continuous batching of uneven (mesh, energies) requests, p50/p99 latency
        # beside solves/s, at the configured 200 requests/s and at a rate one GPU sustains
        import argparse as _ap
        if not args.no_graph:
            del graph
        plan.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        sargs = _ap.Namespace(rates="200,4", rate=200.0, serve_requests=20, serve_precisions="fp64,mixed-gless",
                              slots=args.slots, symmetric=False)
        res = serve_bench(sargs)
        out["serving"] = {
            "workload": "20 requests per trace, Poisson arrivals, Nx in {32,64,128,256}, Ny in {Nx,2Nx}, "
                        "5/9-point, 1-64 energies each (seeded), 4 slots, general form",
            **{form: [{k: r[k] for k in ("rate_req_per_s", "solves_per_s", "p50_latency_s", "p99_latency_s",
                                         "energy_solves", "max_concurrent")} for r in runs]
               for form, runs in res.items()}}
    if args.precision != "fp64":
        # error of this result against the FP64 form of the same solve, per energy
        ref = find.Plan(Nx, Ny, st, precision=find.PREC_FP64, scattering=args.scattering)
        rG = torch.empty_like(dG); rL = torch.empty_like(dL)
        find.solve(ref, E, H, S, SL, rG, rL, stream=stream, **scat)
        find.sync_status(ref, stream)
        def nerr(x, r):
            x, r = x.reshape(nE, -1), r.reshape(nE, -1)
            return ((x - r).abs().amax(dim=1) / r.abs().amax(dim=1)).cpu().numpy()
        eg, el = nerr(dG, rG), nerr(dL, rL)
        out["mixed_error_vs_fp64"] = {"diag_G_max": float(eg.max()), "diag_Gless_max": float(el.max()),
                                      "diag_G_median": float(np.median(eg)),
                                      "diag_Gless_median": float(np.median(el)),
                                      "metric": "per energy ||x - x_fp64||_inf / ||x_fp64||_inf"}
    if not args.no_cpu_baseline and not args.scattering_bonds:
        out["cpu_baseline"] = cpu_baseline(prob, scat=scat_np)
    elif not args.no_cpu_baseline:
        # the RGF oracle takes diagonal self-energies only; the dense oracle
        # (the one that takes bond self-energies) does not reach this mesh
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
