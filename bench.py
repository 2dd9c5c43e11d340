#!/usr/bin/env python
"""Throughput of the method on one MI355X.

Workload: layered elastic box of 64 x 64 x 32 cubic cells (2.5 m), each cell
split into 6 straight 10-node tetrahedra: 1,081,665 nodes, 3,244,995 dof,
786,432 elements; Newmark-beta (beta = 1/4, gamma = 1/2), dt = 0.01 s,
Rayleigh damping 5 % at 0.1 and 2.5 Hz; bottom fixed; seeded band-limited
base acceleration (0.1 - 2.5 Hz); initial guess = Adams-Bashforth 4 plus the
regional snapshot predictor over the last 32 steps (blocks of 8^3 lattice
nodes order the nodes and shape the element patches; runs of 27 of them, in
Morton order of their centroids, are the predictor's least-squares regions);
3x3 block-Jacobi PCG to relative residual 1e-8.

One bench step = one full time step (right-hand side, predictor, PCG refine,
Newmark update) on inputs resident in HBM.  Prints ONE JSON line on stdout;
progress goes to stderr.

Other forms: --precision fp32|bf16 runs the refine as a flexible FP64 outer
PCG preconditioned by an inner FP32-arithmetic PCG (vectors FP32, or p and z
in BF16); --workload large runs the 128 x 128 x 64 cell mesh (25.6M dof,
300 steps).  The default (plain mesh, FP64) is the headline line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def ebe_pcg_bytes_per_element(n_nodes: int, n_elems: int) -> float:
    """Algorithmic HBM bytes of one fused PCG matvec launch, per element.

    Matvec (Eq. EBE) compulsory traffic: connectivity 10 x 4 B + material 4 B
    per element, and per node coordinates, p read and q written (3 x 24 B);
    the fused direction update p = z + beta p_prev adds z read and the new p
    written (2 x 24 B per node).  Node terms are spread over n_nodes/n_elems.
    """
    per_node = 5 * 24.0
    return 44.0 + per_node * n_nodes / n_elems


def cpu_baseline(wl, mesh, em, mat, fx, regions, wave, steps, gpu_iters=None):
    """The CPU oracle (BCSR block-Jacobi PCG + the same predictor) timed on host cores."""
    import numpy as np

    import oracle
    aR, bR = wl.rayleigh
    t0 = time.time()
    model = oracle.Model(mesh.coords, mesh.conn, em, mat, fx, 4 / wl.dt ** 2 + 2 * aR / wl.dt,
                         1 + 2 * bR / wl.dt)
    t_asm = time.time() - t0
    log(f"oracle assembled in {t_asm:.1f} s")
    st = oracle.Stepper(model, wl.dt, aR, bR, s=wl.s, kind=2, tol=wl.tol, regions=regions)
    iters = []
    t0 = time.time()
    for it in range(1, steps + 1):
        rec, _, _ = st.step(g=wave[it])
        iters.append(rec.iters)
    dt = time.time() - t0
    dof = 3 * mesh.n_nodes
    ms_it = dt / max(1, sum(iters)) * 1e3
    # the oracle's BCSR product alone: 3x3 FP64 block + int32 column per stored block, int64 row
    # pointer, x and y once per block row
    nnzb = int(oracle.lib().orc_nnzb(model._h))
    spmv_bytes = nnzb * (72 + 4) + mesh.n_nodes * (8 + 24 + 24)
    p = np.ones(dof)
    model.spmv("A", p)
    t1 = time.time()
    for _ in range(5):
        model.spmv("A", p)
    spmv_s = (time.time() - t1) / 5
    # PCG iterations alone (no right-hand side or predictor), on all threads and on one core
    rhs = np.random.default_rng(7).standard_normal(dof)
    rhs[np.asarray(fx).reshape(-1) != 0] = 0.0

    def pcg_ms(k):
        t = time.time()
        _, s_ = model.pcg(rhs, np.zeros(dof), tol=1e-30, max_iter=k)
        return (time.time() - t) / max(1, s_.iters) * 1e3

    n_thr = oracle.num_threads()
    pcg_all = pcg_ms(20)
    oracle.set_threads(1)
    try:
        pcg_one = pcg_ms(4)
    finally:
        oracle.set_threads(n_thr)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    note = ""
    if gpu_iters:
        # the same oracle at the timed steps' iteration count (the steps from rest need more trips)
        note = (f"; at the timed steps' {gpu_iters:.1f} iterations/step its rate would be "
                f"{dof / (gpu_iters * ms_it * 1e-3):.3g} DOF*steps/s")
    return {
        "value": dof * steps / dt,
        "unit": "DOF*steps/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"steps 1-{steps} of the same workload from rest ({np.mean(iters):.0f} PCG iterations/step, "
                   f"{ms_it:.0f} ms per iteration; BCSR assembly of {t_asm:.0f} s excluded); {dt:.1f} s wall{note}"),
        "iters_per_step": float(np.mean(iters)),
        "spmv_gbs": spmv_bytes / spmv_s / 1e9,
        "spmv_ms": spmv_s * 1e3,
        "pcg_ms_per_iteration": {"all_threads": pcg_all, "one_core": pcg_one},
        "one_core_rate_at_gpu_iters": (dof / (gpu_iters * pcg_one * 1e-3)) if gpu_iters else None,
        "host": {"cpu_model": cpu_model, "cpus_visible": os.cpu_count(), "threads_used": n_thr},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=250, help="timed time steps")
    ap.add_argument("--warmup", type=int, default=250, help="untimed time steps before the timed ones")
    ap.add_argument("--timing-every", type=int, default=32, help="bracket every n-th matvec launch with events")
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle steps in the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "ebe_pcg_traffic.txt"))
    ap.add_argument("--patch-elems", type=int, default=256, help="elements per EBE patch (1..256)")
    ap.add_argument("--region-block", type=int, default=0,
                    help="predictor regions of b^3 lattice nodes (0: the workload's, 8 = 512 nodes)")
    ap.add_argument("--region-merge", type=int, default=-1,
                    help="given regions merged per predictor region, in Morton order of their centroids "
                         "(-1: the workload's, 1 = none)")
    ap.add_argument("--energy", action="store_true",
                    help="plain/large: GPU energy over the timed steps from the amd-smi energy counter "
                         "(timed region of 4 s or more)")
    ap.add_argument("--workload", choices=["plain", "large", "learned", "ensemble"], default="plain")
    ap.add_argument("--no-graph", action="store_true", help="ensemble: enqueue PCG trips without hipGraph")
    ap.add_argument("--no-tune", action="store_true", help="ensemble: default case tiles instead of the autotuner")
    ap.add_argument("--train-seeds", type=int, default=50, help="learned: training trajectories")
    ap.add_argument("--train-steps", type=int, default=200, help="learned: steps per training trajectory")
    ap.add_argument("--train-nodes", type=int, default=4096, help="learned: sampled nodes per training step")
    ap.add_argument("--test-seeds", type=int, default=32, help="learned: test trajectories")
    ap.add_argument("--test-steps", type=int, default=200, help="learned: steps per test trajectory")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64",
                    help="fp64: plain PCG; fp32/bf16: flexible FP64 PCG with an inner low-precision PCG")
    ap.add_argument("--inner-iters", type=int, default=0, help="inner PCG trips per outer trip (0: library default)")
    ap.add_argument("--inner-tol", type=float, default=0.0, help="inner relative tolerance (0: library default)")
    ap.add_argument("--drop-tol", type=float, default=0.0,
                    help="predictor column drop threshold (0: the library's, 1e-6 for fp64 and 1e-5 for the mixed "
                         "forms, whose FP32 inner solves leave rounding noise in the snapshots)")
    ap.add_argument("--predictor", type=int, choices=[0, 1, 2], default=2,
                    help="plain/large: guess of each step (0 zero, 1 AB4, 2 AB4 + regional snapshot map)")
    ap.add_argument("--snapshots", type=int, default=0, help="plain/large: snapshot window s (0: the workload's, 32)")
    ap.add_argument("--s-min", type=int, default=0,
                    help="plain/large: column pairs before the map is used (0: the library's, 8)")
    ap.add_argument("--fixed-window", action="store_true",
                    help="plain/large: the map's guess always, the window never restarts (no AB4 guard)")
    ap.add_argument("--input", choices=["base", "surface"], default="base",
                    help="plain/large: base acceleration (default) or the paper-like surface impulses")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB device-to-device once (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_20380_amd import ebe, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "learned":
        run_learned(args)
        return
    if args.workload == "ensemble":
        run_ensemble(args)
        return
    wl = inputs.WORKLOADS[args.workload]
    prec = {"fp64": ebe.PREC_FP64, "fp32": ebe.PREC_FP32, "bf16": ebe.PREC_BF16}[args.precision]
    nt = args.warmup + args.steps
    s_win = args.snapshots or wl.s
    wl_run = inputs.Workload(wl.name, cells=wl.cells, h=wl.h, dt=wl.dt, nt=nt, s=s_win, tol=wl.tol,
                             seed=wl.seed, region_block=args.region_block or wl.region_block)
    mesh, em, mat, fx, regions, wave = wl_run.build()
    merge = args.region_merge if args.region_merge >= 0 else wl.region_merge
    dof = 3 * mesh.n_nodes
    log(f"mesh {wl.cells}: {mesh.n_nodes} nodes, {dof} dof, {mesh.n_elems} elements")
    aR, bR = wl.rayleigh
    sol = ebe.Solver(wl.dt, aR, bR, s=s_win, tol=wl.tol, patch_elems=args.patch_elems, precision=prec,
                     inner_iters=args.inner_iters, inner_tol=args.inner_tol, drop_tol=args.drop_tol,
                     predictor=args.predictor, s_min=args.s_min, fixed_window=args.fixed_window,
                     region_merge=merge)
    # per-step forcing, resident in HBM before the timed region: base acceleration (3 values
    # a step) or the paper-like surface impulses (a force vector a step)
    f_all = None
    if args.input == "surface":
        sp_nodes, sp_force = inputs.surface_impulses(mesh, wl.seed, nt, wl.dt)
        f_all = torch.zeros((nt + 1, mesh.n_nodes, 3), dtype=torch.float64, device="cuda")
        f_all[:, torch.from_numpy(sp_nodes.astype(np.int64)).cuda()] = torch.from_numpy(sp_force).cuda()
        f_all = f_all.view(nt + 1, dof)
        log(f"surface impulses at {sp_nodes.size} top nodes")

    def forcing(it):
        return (None, wave[it]) if f_all is None else (f_all[it], None)
    drop = sol.effective_config().drop_tol
    t0 = time.time()
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx, regions)
    sizes = sol.sizes()
    log(f"assembled in {time.time() - t0:.1f} s: {sizes}")

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst

    for it in range(1, args.warmup + 1):
        f, g = forcing(it)
        st = sol.step(f_ext=f, base_acc=g)
        if it % 50 == 0 or it == args.warmup:
            log(f"warmup step {it}: {st.iters} iters, res_true {st.res_true:.2e}")

    sol.set_kernel_timing(args.timing_every)
    iters, res, inner, res0, s_eff, kept = [], [], [], [], [], []
    energy = gpu_energy_reader() if args.energy else None
    torch.cuda.synchronize()
    e0 = energy() if energy else None
    t0 = time.perf_counter()
    for it in range(args.warmup + 1, nt + 1):
        f, g = forcing(it)
        st = sol.step(f_ext=f, base_acc=g)
        iters.append(st.iters)
        inner.append(st.inner_iters)
        res.append(st.res_true)
        res0.append(st.res0)
        s_eff.append(st.s_eff)
        kept.append(st.map_kept)
        if st.status != 0:
            raise RuntimeError(f"step {it} did not converge")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    e1 = energy() if energy else None
    n_timed, ebe_ms = sol.kernel_time()
    log(f"timed {args.steps} steps in {elapsed:.3f} s; mean iters {np.mean(iters):.1f}; "
        f"matvec {ebe_ms * 1e3:.1f} us over {n_timed} timed launches")

    ecfg = sol.effective_config()
    bpe = ebe_pcg_bytes_per_element(mesh.n_nodes, mesh.n_elems)
    launch_bytes = bpe * mesh.n_elems   # the timed launch is the FP64 (outer) matvec in every form
    achieved = launch_bytes / (ebe_ms * 1e-3) / 1e9 if ebe_ms > 0 else 0.0
    traffic = None
    tj = read_kv(args.traffic_file)
    if (tj.get("workload") == wl.name and tj.get("precision", "fp64") == args.precision
            and tj.get("kernel_source_sha") == kernel_source_sha()):
        traffic = float(tj["bytes_per_launch"])

    out = {
        "metric": "DOF*steps/s at rel. residual 1e-8",
        "value": dof * args.steps / elapsed,
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"f64 outer / {args.precision} inner",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": list(wl.cells), "nodes": mesh.n_nodes, "dof": dof,
                   "elements": mesh.n_elems, "dt": wl.dt, "snapshots": s_win, "tol": wl.tol,
                   "predictor": {0: "zero guess", 1: "AB4",
                                 2: "AB4 + regional snapshot map" + (", fixed window" if args.fixed_window else
                                                                     ", guarded window")}[args.predictor],
                   "s_min": ecfg.s_min, "input": ("base acceleration" if args.input == "base" else
                                                  "surface impulses (284 points)"),
                   "region_nodes": wl_run.region_block ** 3 * max(1, merge),
                   "region_merge": max(1, merge),
                   "drop_tol": drop,
                   "timed_steps": f"{args.warmup + 1}-{nt}",
                   "refine": ("block-Jacobi PCG, FP64" if args.precision == "fp64" else
                              f"flexible FP64 PCG, inner {args.precision} PCG ({ecfg.inner_iters} trips, "
                              f"tol {ecfg.inner_tol:g})")},
        "cg_iters_per_step": float(np.mean(iters)),
        "inner_iters_per_step": float(np.mean(inner)),
        "cg_iters_min_max": [int(np.min(iters)), int(np.max(iters))],
        "initial_rel_residual_geomean": float(np.exp(np.mean(np.log(np.maximum(res0, 1e-300))))),
        "snapshot_pairs_mean": float(np.mean(s_eff)),
        "map_kept_steps": int(sum(1 for k in kept if k == 1)),
        "window_restarts": int(sum(1 for k in kept if k == 0)),
        "max_true_rel_residual": float(np.max(res)),
        "ebe_matvec_hbm_gbs": achieved,
        "roofline": {"kernel": "k_ebe<PCG> (fused direction update + EBE matvec + (p,Ap))",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_note": "HBM bytes per launch from FETCH_SIZE/WRITE_SIZE, scaled by a 1 GiB copy",
                     "bytes_per_launch": launch_bytes, "mean_launch_ms": ebe_ms, "timed_launches": n_timed},
    }
    if args.energy:
        # the accumulator advances in coarse updates: only a timed region of several seconds gives a figure
        out["energy"] = None if e0 is None or e1 is None or elapsed < 4.0 else {
            "joules_per_step": (e1 - e0) / args.steps, "mean_power_w": (e1 - e0) / elapsed,
            "joules_per_mdof_step": (e1 - e0) / args.steps / (dof * 1e-6),
            "source": "amd-smi energy accumulator of this GPU, read before and after the timed steps"}
    pred_regions, _ = sol.regions()   # the predictor's regions (merged ones when region_merge > 1)
    sol.close()
    if not args.no_cpu_baseline and args.workload == "plain" and args.input == "base" and args.predictor == 2 \
            and not args.snapshots and not args.s_min and not args.fixed_window:
        log(f"CPU baseline: oracle, {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(wl_run, mesh, em, mat, fx, pred_regions, wave, args.cpu_steps,
                                           gpu_iters=float(np.mean(iters)))
    print(json.dumps(out), flush=True)


def run_learned(args):
    """Learned predictor on the 64 x 64 x 32 mesh: train on trajectories the
    solver generates (own kernels), then compare test trajectories of kind 3
    (network candidate with fallback) with the plain method (kind 2) and with
    kind 3 on a zero network (the fallback between AB4 and the snapshot guess
    alone); then kinds 2 and 3 again with the FP32 inner solve (the learned
    guess and mixed precision together)."""
    import numpy as np
    import torch

    from paper_2409_20380_amd import ebe, inputs, learn
    base = inputs.PLAIN
    steps = max(args.train_steps, args.test_steps)
    wl = inputs.Workload(base.name, cells=base.cells, h=base.h, dt=base.dt, nt=steps, s=base.s, tol=base.tol,
                         seed=base.seed, region_block=base.region_block)
    mesh, em, mat, fx, regions, _ = wl.build()
    aR, bR = wl.rayleigh
    dof = 3 * mesh.n_nodes
    sol = ebe.Solver(wl.dt, aR, bR, s=wl.s, tol=wl.tol, patch_elems=args.patch_elems)
    sol.assemble(mesh.coords, mesh.conn, em, mat, fx, regions)
    nodes = torch.from_numpy(inputs.sample_nodes(3, fx, args.train_nodes)).cuda()
    seeds = inputs.LEARN_TRAIN_SEEDS[:args.train_seeds]
    cap = len(seeds) * (args.train_steps - 4) * nodes.numel()
    t0 = time.time()
    learn.generate(sol, wl, seeds, args.train_steps, nodes, cap)
    t_gen = time.time() - t0
    n_samples = sol.samples().shape[0]
    log(f"generated {n_samples} samples from {len(seeds)} trajectories in {t_gen:.1f} s")
    t0 = time.time()
    losses = learn.train(sol, 1, [(3000, 1e-3), (2000, 3e-4), (1000, 1e-4)], 4096, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    trained, scales = sol.mlp_get()

    def run(kind, seeds_, params, solver=None):
        solver = sol if solver is None else solver
        solver.set_predictor(kind)
        if params is not None:
            solver.mlp_set(params, scales)
        its, res, picks, el = [], [], [], 0.0
        for seed in seeds_:
            w = inputs.base_wave(seed, args.test_steps, wl.dt, *wl.f_band)
            solver.reset()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for it in range(1, args.test_steps + 1):
                st = solver.step(base_acc=w[it])
                if st.status != 0:
                    raise RuntimeError(f"seed {seed} step {it} did not converge")
                its.append(st.iters); res.append(st.res_true); picks.append(st.learned)
            torch.cuda.synchronize()
            el += time.perf_counter() - t
        picks = np.array(picks)
        return dict(value=dof * args.test_steps * len(seeds_) / el, ms_per_step=el / (args.test_steps * len(seeds_)) * 1e3,
                    iters=float(np.mean(its)), max_res=float(np.max(res)),
                    pick=float((picks == 1).sum() / max(1, (picks >= 0).sum())))

    test = inputs.LEARN_TEST_SEEDS[:args.test_seeds]
    plain = run(ebe.PRED_SNAPSHOT, test, None)
    log(f"plain (kind 2): {plain}")
    sol.set_kernel_timing(args.timing_every)
    learned = run(ebe.PRED_LEARNED, test, trained)
    n_timed, ebe_ms = sol.kernel_time()
    log(f"learned (kind 3): {learned}")
    zero = run(ebe.PRED_LEARNED, test[:4], np.zeros_like(trained))
    log(f"selection only (kind 3, zero network, {min(4, len(test))} seeds): {zero}")
    sol.close()
    # the two single-case growth forms together: the trained network's guess refined by the
    # flexible FP64 PCG with the FP32 inner solve, against the same FP32 refine with the plain guess
    solm = ebe.Solver(wl.dt, aR, bR, s=wl.s, tol=wl.tol, patch_elems=args.patch_elems, precision=ebe.PREC_FP32,
                      inner_iters=args.inner_iters, inner_tol=args.inner_tol, drop_tol=args.drop_tol)
    solm.assemble(mesh.coords, mesh.conn, em, mat, fx, regions)
    inner_trips = solm.effective_config().inner_iters
    mixed_plain = run(ebe.PRED_SNAPSHOT, test, None, solm)
    log(f"plain guess, FP32 inner solve: {mixed_plain}")
    mixed_learned = run(ebe.PRED_LEARNED, test, trained, solm)
    log(f"learned guess, FP32 inner solve: {mixed_learned}")
    solm.close()
    bpe = ebe_pcg_bytes_per_element(mesh.n_nodes, mesh.n_elems)
    achieved = bpe * mesh.n_elems / (ebe_ms * 1e-3) / 1e9 if ebe_ms > 0 else 0.0
    out = {
        "metric": "DOF*steps/s at rel. residual 1e-8",
        "value": learned["value"],
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.test_steps * len(test),
        "warmup": 0,
        "ms_per_step": learned["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (network: bf16 weights, fp32 accumulate)",
        "data": "synthetic",
        "config": {"workload": "box64x64x32_learned_predictor", "cells": list(wl.cells), "dof": dof,
                   "train": f"{len(seeds)} trajectories x {args.train_steps} steps, {args.train_nodes} nodes/step, "
                            f"{n_samples} samples, 6000 Adam steps (batch 4096)",
                   "test": f"{len(test)} new waves x {args.test_steps} steps from rest",
                   "predictor": "kind 3: AB4 + network estimate of the AB4 error vs the AB4 + snapshot guess, "
                                "smaller initial residual kept"},
        "plain_value": plain["value"],
        "speedup_vs_plain": learned["value"] / plain["value"],
        "cg_iters_per_step": learned["iters"],
        "plain_cg_iters_per_step": plain["iters"],
        "learned_pick_fraction": learned["pick"],
        "selection_only": zero,
        "learned_fp32_inner": {"value": mixed_learned["value"], "ms_per_step": mixed_learned["ms_per_step"],
                               "cg_iters_per_step": mixed_learned["iters"], "max_res": mixed_learned["max_res"],
                               "speedup_vs_plain": mixed_learned["value"] / plain["value"],
                               "inner_trips": inner_trips},
        "plain_fp32_inner": {"value": mixed_plain["value"], "ms_per_step": mixed_plain["ms_per_step"],
                             "cg_iters_per_step": mixed_plain["iters"], "max_res": mixed_plain["max_res"],
                             "speedup_vs_plain": mixed_plain["value"] / plain["value"]},
        "max_true_rel_residual": max(learned["max_res"], plain["max_res"], mixed_learned["max_res"],
                                     mixed_plain["max_res"]),
        "train_seconds": {"generate": t_gen, "train": t_train},
        "final_train_loss": float(np.mean(losses[-50:])),
        "roofline": {"kernel": "k_ebe<PCG> (fused direction update + EBE matvec + (p,Ap))", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": bpe * mesh.n_elems, "mean_launch_ms": ebe_ms,
                     "timed_launches": n_timed},
    }
    print(json.dumps(out), flush=True)


def run_ensemble(args):
    """Batched ensemble: 64 cases on three meshes (16x16x8 x20, 32x32x16 x24,
    48x48x24 x20 cells), seeds 1..64, 32 snapshots, all cases advanced
    together; baseline: one case per mesh run alone on the single-case path
    over the same steps, scaled by the case counts."""
    import numpy as np
    import torch

    from paper_2409_20380_amd import ebe, inputs
    nt = args.warmup + args.steps
    dt, tol, s = inputs.PLAIN.dt, inputs.PLAIN.tol, inputs.ENSEMBLE_S
    aR, bR = inputs.PLAIN.rayleigh
    t0 = time.time()
    meshes = []
    for cells, r in inputs.ENSEMBLE:
        wl = inputs.Workload(f"box{cells[0]}x{cells[1]}x{cells[2]}", cells=cells, nt=nt, s=s)
        mesh, em, mat, fx, regions, _ = wl.build()
        meshes.append((cells, r, mesh, em, mat, fx, regions))
    C = sum(r for _, r in inputs.ENSEMBLE)
    waves = [inputs.base_wave(1 + c, nt, dt) for c in range(C)]
    dof_total = sum(3 * m[2].n_nodes * m[1] for m in meshes)
    merge = args.region_merge if args.region_merge >= 0 else inputs.ENSEMBLE_REGION_MERGE
    batch = ebe.Batch(dt, aR, bR, s=s, tol=tol, region_merge=merge)
    for cells, r, mesh, em, mat, fx, regions in meshes:
        batch.add_mesh(mesh.coords, mesh.conn, em, mat, fx, regions, r)
    t1 = time.time()
    batch.assemble(tune=not args.no_tune)
    batch.use_graph(not args.no_graph, 8)
    t_asm = time.time() - t1
    groups = [batch.group_info(g) for g in range(len(meshes))]
    log(f"ensemble: {C} cases, {dof_total} dof per step; inputs {t1 - t0:.1f} s, assemble+tune {t_asm:.1f} s; {groups}")
    G = np.zeros((nt + 1, C, 3))
    for c in range(C):
        G[:, c, :] = waves[c]
    iters = []
    for it in range(1, args.warmup + 1):
        batch.step(G[it])
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = 0.0
    for it in range(args.warmup + 1, nt + 1):
        st = batch.step(G[it])
        if any(x.status != 0 for x in st):
            raise RuntimeError(f"ensemble step {it} did not converge")
        iters.append([x.iters for x in st])
        res = max(res, max(x.res_true for x in st))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    batch.close()
    iters = np.array(iters)
    log(f"batched: {args.steps} steps in {elapsed:.2f} s; mean iters per case {iters.mean():.1f}")
    # baseline: the first case of each mesh alone on the single-case path, same steps
    seq = 0.0
    c0 = 0
    seq_detail = []
    for cells, r, mesh, em, mat, fx, regions in meshes:
        sol = ebe.Solver(dt, aR, bR, s=s, tol=tol, region_merge=merge)
        sol.assemble(mesh.coords, mesh.conn, em, mat, fx, regions)
        for it in range(1, args.warmup + 1):
            sol.step(base_acc=waves[c0][it])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for it in range(args.warmup + 1, nt + 1):
            sol.step(base_acc=waves[c0][it])
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        sol.close()
        seq += el * r
        seq_detail.append({"cells": list(cells), "ms_per_step_one_case": el / args.steps * 1e3, "cases": r})
        c0 += r
    value = dof_total * args.steps / elapsed
    out = {
        "metric": "DOF*steps/s at rel. residual 1e-8",
        "value": value,
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ensemble_64_cases_3_meshes", "meshes": [[list(c), r] for c, r in inputs.ENSEMBLE],
                   "dof_per_step": dof_total, "snapshots": s, "tol": tol, "seeds": "1-64", "region_merge": merge,
                   "graph": not args.no_graph, "tuned": not args.no_tune, "groups": groups},
        "cg_iters_per_step_per_case": float(iters.mean()),
        "max_true_rel_residual": res,
        "sequential_single_case_value": dof_total * args.steps / seq,
        "speedup_vs_sequential": seq / elapsed,
        "sequential_detail": seq_detail,
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def read_kv(path: str) -> dict:
    """key = value lines (comments with #) of a profile summary."""
    out = {}
    if os.path.exists(path):
        for line in open(path):
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                out[k.strip()] = v.strip()
    return out


def gpu_energy_reader():
    """A function returning the cumulative energy (J) of this process's GPU from the
    amd-smi library's energy accumulator, or None where it is not available."""
    try:
        import amdsmi
        import torch
        amdsmi.amdsmi_init()
        handles = amdsmi.amdsmi_get_processor_handles()
        prop = torch.cuda.get_device_properties(0)
        bdf = None
        if all(hasattr(prop, a) for a in ("pci_domain_id", "pci_bus_id", "pci_device_id")):
            bdf = f"{prop.pci_domain_id:04x}:{prop.pci_bus_id:02x}:{prop.pci_device_id:02x}.0"
        pick = [h for h in handles if bdf and amdsmi.amdsmi_get_gpu_device_bdf(h).lower() == bdf]
        if not pick and len(handles) == 1:
            pick = handles
        if not pick:
            return None
        h = pick[0]

        def read():
            e = amdsmi.amdsmi_get_energy_count(h)
            return e["energy_accumulator"] * e["counter_resolution"] * 1e-6

        read()
        return read
    except Exception as exc:   # no library, no permission, no such device: no energy figure
        log(f"energy counter not available: {exc}")
        return None


def kernel_source_sha() -> str:
    """Fingerprint of the sources the FP64 matvec kernel is built from (its
    code, the element operator and the patch layout)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "element.h", "topology.cpp"):
        with open(os.path.join(ROOT, "paper_2409_20380_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
