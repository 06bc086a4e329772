"""Benchmark: solves/sec to a 1e-8 relative residual on one MI355X.

Default workload (the learned Schur preconditioner case): a 256^3 periodic
grid with 10^4 absorbing blobs placed by random sequential addition
(minimum separation 3h), four-point kernel, uniform source f = 1, steady
diffusion-limited saddle point, to a 1e-8 relative residual.

A step is one full absorbing solve with inputs resident in device memory.
`value` is the fastest learned + FP32 solver: flexible GMRES(30) on the
whole block system with the paper's approximate-Schur preconditioner (m = 5
inner GMRES iterations, one FP32 V-cycle per product, n = 1), the inner
GMRES right-preconditioned by the trained network (weights in
paper_1306_3159_amd/weights); FP64 Krylov vectors and true FP64 residuals.
Beside it: Schur-complement GMRES(30) with inner multigrid-preconditioned CG
(learned + FP32, FP32 alone, and plain FP64: FP64 V-cycles, no learned part,
the comparison baseline), the block solver without the network in FP32 and
FP64, and the 128^3 lattice workload (8^3 blobs 16h apart, random source).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/sec at 1e-8 rel residual, learned+FP32 vs plain FP64; HBM GB/s"
HBM_PEAK_GBS = 8000.0
WEIGHTS = os.path.join(ROOT, "paper_1306_3159_amd", "weights", "precond_rsa256.npy")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rsa256_learned",
                    choices=["rsa256_learned", "lattice128_randf", "batch64", "box256"])
    ap.add_argument("--threads", type=int, default=8, help="host workers of the batch executor")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run one device copy of this many MiB (calibrates memory counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the comparison paths and the extra workload")
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--autotune", type=int, default=1,
                    help="time candidate work-group sizes of the multigrid kernels before the timed solves")
    return ap.parse_args()


# HBM bytes per launch of the finest-level FP32 Gauss-Seidel half-sweep at
# 256^3 from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (KiB per dispatch, cold
# rotating launches), scaled by what the same counters read for a 1 GiB device
# copy (FETCH_SIZE reports half the bytes read, WRITE_SIZE all bytes written).
# Valid only for the kernel source the counters were taken on.
TRAFFIC = {"source_sha256": "64f992908b027878b0cc1adce1ded5c37b01dd7bd1cd9e336be4a9e27e0f8321",
           "fetch_kib": 33813.0, "write_kib": 32768.0, "fetch_scale": 1.9999, "write_scale": 1.0}


def measured_traffic(n):
    import hashlib
    src = os.path.join(ROOT, "paper_1306_3159_amd", "csrc", "kernels_mg.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if n != 256 or TRAFFIC["source_sha256"] != digest or TRAFFIC["fetch_kib"] is None:
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"])


STEP_TIMES = {}


def timed(fn, steps, warmup):
    """Total wall time of `steps` calls after `warmup` untimed ones (each call returns once its
    solve is complete); the per-call times are kept in STEP_TIMES[fn] for the median."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    per = []
    for _ in range(steps):
        t1 = time.perf_counter()
        st = fn()
        per.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    STEP_TIMES[fn] = per
    return time.perf_counter() - t0, st


def summary(st, block=False):
    """Iteration counts of a solve: Schur GMRES with inner CG, or (block) flexible GMRES on the
    block system with inner GMRES iterations of the approximate-Schur preconditioner."""
    it = {"fgmres_iters": st["outer_iters"], "inner_gmres_iters": st["inner_iters_total"]} if block else \
        {"gmres_iters": st["outer_iters"], "inner_cg_iters": st["inner_iters_total"]}
    return {**it, "vcycles": st["vcycles"], "rel_resid": st["rel_resid"], "refinements": st["refinements"],
            "fallback": st["fallback"], "alg_bytes": st["alg_bytes"]}


# Grids up to 64^3 are launch-latency-bound and share the lock-step batched
# launches (reactive ones in the CG rounds, block-FGMRES absorbing ones in the
# V-cycle rounds); larger ones are bandwidth-bound and run on their own streams.
LOCKSTEP_MAX_CELLS = 64 ** 3
COARSE_M2 = 6   # Fourier coarse level of the headline solve: wave vectors 0 < |m|^2 <= 6 (80 columns)
HEAD_M = 3      # inner GMRES iterations of the headline solve's approximate-Schur preconditioner


def bench_batch(args, dev, rtol, steps, warmup):
    """64 uneven suspensions (grids 32..128, up to 2000 blobs, reactive/absorbing 50/50, absorbing
    ones by the block FGMRES); a step is the whole batch. value: the lock-step executor with grids
    up to 64^3 in the batched launches (reactive CG iterations in the captured CG rounds, the
    absorbing instances' V-cycles in the captured V-cycle rounds) and the larger grids on their own
    streams meanwhile. Beside it: every instance in the batched launches, the per-instance-stream
    executor, one-by-one solves, and the lock-step executor with Schur-GMRES absorbing solves (their
    inner CG iterations in the CG rounds). Returns the line's fields."""
    import torch
    import workloads as W
    from paper_1306_3159_amd import BlobRD, MIXED, SOLVER_BLOCK, SOLVER_SCHUR, solve_streams, solve_batched
    insts = W.batch_instances()

    def handles(solver):
        return [BlobRD(i.n, torch.tensor(i.q, device=dev), torch.tensor(i.kappa, device=dev), precision=MIXED,
                       rtol=rtol, stream=torch.cuda.Stream(dev),
                       saddle_solver=solver if i.kind == "absorbing" else SOLVER_SCHUR) for i in insts]

    Hs = handles(SOLVER_BLOCK)
    fs = [torch.tensor(i.f, device=dev) for i in insts]
    kinds = [1 if i.kind == "absorbing" else 0 for i in insts]
    cs = [torch.zeros_like(f) for f in fs]
    ls = [torch.zeros(i.N, dtype=torch.float64, device=dev) if k else None for i, k in zip(insts, kinds)]
    bstream = torch.cuda.Stream(dev)
    tuned = 0
    if args.autotune:
        import tempfile
        cache = os.path.join(tempfile.mkdtemp(), "tune.json")  # one timing per distinct level shape
        tuned = sum(H.autotune(reps=5, cache=cache) for H in Hs)

    def step_lockstep(cap):
        def fn():
            for c in cs:
                c.zero_()
            torch.cuda.synchronize()
            return solve_batched(Hs, kinds, fs, cs, ls, stream=bstream, lockstep_max_cells=cap, threads=args.threads)
        return fn

    def step_streams():
        for c in cs:
            c.zero_()
        torch.cuda.synchronize()
        return solve_streams(Hs, kinds, fs, cs, ls, threads=args.threads)

    ns = max(2, steps // 2)
    dt, (rc, stats) = timed(step_lockstep(LOCKSTEP_MAX_CELLS), steps, warmup)
    adt, (arc, _) = timed(step_lockstep(0), ns, 1)
    sdt, (src, _) = timed(step_streams, ns, 1)
    t1 = time.perf_counter()
    for H, k, f, c, l in zip(Hs, kinds, fs, cs, ls):
        c.zero_()
        torch.cuda.synchronize()
        if k:
            H.solve_absorbing(f, c=c, lam=l)
        else:
            H.solve_reactive(f, c=c)
    serial = time.perf_counter() - t1
    for H in Hs:
        H.close()
    Hs = handles(SOLVER_SCHUR)
    if args.autotune:
        for H in Hs:
            H.autotune(reps=5, cache=cache)
    qdt, (qrc, _) = timed(step_lockstep(LOCKSTEP_MAX_CELLS), ns, 1)
    for H in Hs:
        H.close()
    cells = sum(i.n ** 3 for i in insts)
    small = [i for i in insts if i.n ** 3 <= LOCKSTEP_MAX_CELLS]
    return {"value": len(insts) * steps / dt, "unit": "instances/s", "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * dt / steps,
            "config": {"workload": "batch64", "instances": len(insts), "total_cells": cells,
                       "total_blobs": sum(i.N for i in insts), "rtol": rtol, "absorbing_solver": "block FGMRES",
                       "executor": "lock-step batched launches (captured CG rounds, captured V-cycle rounds) for "
                                   "grids <= 64^3, own streams for larger grids",
                       "lockstep_cg_instances": sum(1 for i in small if i.kind != "absorbing"),
                       "lockstep_vcycle_instances": sum(1 for i in small if i.kind == "absorbing"),
                       "stream_threads": args.threads, "autotuned_levels": tuned},
            "rc": rc, "max_rel_resid": max(s["rel_resid"] for s in stats),
            "all_lockstep": {"instances_per_s": len(insts) * ns / adt, "rc": arc},
            "streams_executor": {"instances_per_s": len(insts) * ns / sdt, "threads": args.threads, "rc": src},
            "serial_instances_per_s": len(insts) / serial,
            "lockstep_schur_gmres": {"instances_per_s": len(insts) * ns / qdt, "rc": qrc}}


def _say(msg):
    """Progress on stderr (the one JSON line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(inst):
    """The oracle's own absorbing solve (Schur-complement GMRES(30) with inner MG-CG Poisson solves,
    FP64 V(2,2) cycles, OpenMP over z-slabs) timed end to end on the same input and tolerance on
    all host threads, once; and one full oracle Poisson solve of the same grid timed on one thread,
    which with the solve's own count of Poisson solves gives the one-core rate."""
    from oracle import iterative as it
    it.build(force=False)
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    nt = it.num_threads()
    _say(f"cpu baseline: oracle absorbing solve {inst.n}^3, {inst.N} blobs on {nt} threads")
    t0 = time.perf_counter()
    c, lam, ost = it.solve_absorbing(inst.f, inst.q, 0.0, rtol=inst.rtol, inner_rtol=1e-10)
    ts = time.perf_counter() - t0
    n_poisson = ost["iters"] + 2
    _say(f"cpu baseline: {ts:.1f} s, {ost['iters']} GMRES iterations, {ost['inner_iters']} inner CG iterations, "
         f"residual {ost['rel_resid']:.2e}; one-thread Poisson solve next")
    lbar = float(np.sum(inst.f)) / inst.N
    g = np.asarray(inst.f, dtype=np.float64) + it.spread(np.full(inst.N, -lbar), inst.q, inst.f.shape)
    it.set_num_threads(1)
    t1 = time.perf_counter()
    _, pst = it.solve_poisson(g, 0.0, rtol=1e-10)
    tp1 = time.perf_counter() - t1
    it.set_num_threads(nt)
    _say(f"cpu baseline: one-thread Poisson solve {tp1:.1f} s")
    return {"value": 1.0 / ts, "unit": "solves/s", "cores": nt, "kind": "oracle",
            "sample": f"one end-to-end oracle absorbing solve of this workload ({inst.n}^3, {inst.N} blobs, f=1, "
                      f"rtol {inst.rtol:g}, inner Poisson rtol 1e-10): {ts:.1f} s, {ost['iters']} Schur GMRES "
                      f"iterations, {ost['inner_iters']} inner CG iterations, {ost['vcycles']} V-cycles, oracle "
                      f"residual {ost['rel_resid']:.2e}; {nt} OpenMP threads of {os.cpu_count()} logical CPUs, {cpu}",
            "seconds": ts, "gmres_iters": ost["iters"], "rc": ost["rc"],
            "single_core": {"value": 1.0 / (tp1 * n_poisson), "unit": "solves/s", "cores": 1,
                            "sample": f"one full oracle Poisson solve of the same grid (its first right-hand side, "
                                      f"rtol 1e-10, {pst['inner_iters']} CG iterations) on 1 thread: {tp1:.1f} s, "
                                      f"times the {n_poisson} Poisson solves of the timed absorbing solve"}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "single-GPU build: multi-GPU sharding (z-slab decomposition) is a design note, "
                                   "not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1306_3159_amd import BlobRD, Net, MIXED, FP64, PRECOND_LEARNED, PRECOND_NONE, BOUNDARY_DIRICHLET

    dev = torch.device("cuda:0")
    rtol = 1e-8
    if args.workload == "batch64":
        b = bench_batch(args, dev, rtol, args.steps, args.warmup)
        print(json.dumps({"metric": METRIC, "value": b.pop("value"), "unit": b.pop("unit"), "n_gpus": 1,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f64 Krylov/residuals + f32 V-cycles", "data": "synthetic", **b}))
        return
    box = args.workload == "box256"
    if args.workload == "rsa256_learned":
        inst = W.learned_eval(256, 10000, index=0)
    elif box:
        inst = W.box_suspension(256, 10000)
    else:
        inst = W.cubic_lattice(random_f=True)
    q = torch.tensor(inst.q, device=dev)
    f = torch.tensor(inst.f, device=dev)

    net = None
    if args.workload == "rsa256_learned":
        net = Net(dev)
        net.set_params(torch.tensor(np.load(WEIGHTS), device=dev))
        S = BlobRD(inst.n, q, precision=MIXED, schur_precond=PRECOND_LEARNED, rtol=rtol)
        S.precond_build(net)
    elif box:
        S = BlobRD(inst.n, q, precision=MIXED, rtol=rtol, boundary=BOUNDARY_DIRICHLET, boundary_value=1.0)
    else:
        S = BlobRD(inst.n, q, precision=MIXED, rtol=rtol)
    tuning = None
    if args.autotune and not box:
        S.autotune(reps=10)
        tuning = S.get_tuning().tolist()
    learned = args.workload == "rsa256_learned"
    coarse = None
    if learned:
        # block FGMRES, approximate-Schur preconditioner whose inner GMRES is right-preconditioned by
        # the learned W inside the two-level B of the Fourier coarse level (80 columns, |m|^2 <= 6),
        # m = 3 inner iterations. W and the level are set up once per blob set, outside the timed
        # solves; the level's build is timed on its own and reported.
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K = S.coarse_build(0.0, COARSE_M2, 1e-4)
        torch.cuda.synchronize()
        coarse = {"columns": K, "m2max": COARSE_M2, "inner_rtol": 1e-4,
                  "build_ms": 1e3 * (time.perf_counter() - t0)}
        dt, st = timed(lambda: S.solve_absorbing_fgmres(f, precond="learned", m=HEAD_M, n=1, restart=30)[2],
                       args.steps, args.warmup)
    elif box:
        dt, st = timed(lambda: S.solve_absorbing_fgmres(f, precond="schur", m=5, n=1, restart=30)[2], args.steps,
                       args.warmup)
    else:
        dt, st = timed(lambda: S.solve_absorbing(f)[2], args.steps, args.warmup)
    value = args.steps / dt
    med = float(np.median(next(iter(STEP_TIMES.values())))) if len(STEP_TIMES) == 1 else None
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 Krylov/residuals + f32 V-cycles"
        + (" + bf16 network" if learned else ""), "data": "synthetic",
        "config": {"workload": args.workload, "n": inst.n, "N": inst.N, "kind": "absorbing", "rtol": rtol,
                   "kernel_w": 4, "restart": 30,
                   "path": f"block FGMRES + approximate Schur (m={HEAD_M}, n=1), inner GMRES right-preconditioned by "
                           "the learned W inside the two-level Fourier coarse level + fp32"
                   if learned else ("Dirichlet box c_inf=1: block FGMRES + approximate Schur (m=5, n=1) + fp32"
                                    if box else "Schur GMRES + inner MG-CG + fp32"),
                   "source": "f=1" if (learned or box) else "f=1+0.5N(0,1)", "seed": inst.seed},
        "solve": summary(st, block=learned or box),
        "median_ms_per_step": None if med is None else 1e3 * med,
        "tuning": tuning,
    }
    if coarse:
        out["config"]["coarse_level"] = coarse
    out["solve"]["alg_GBs"] = st["alg_bytes"] / (dt / args.steps) / 1e9

    if not args.no_extra and not box:
        n = max(2, args.steps // 2)
        P = BlobRD(inst.n, q, precision=FP64, rtol=rtol)
        if args.autotune:
            P.autotune(reps=10)
        pdt, pst = timed(lambda: P.solve_absorbing(f)[2], n, 1)
        out["plain_fp64"] = {"solver": "Schur GMRES + inner MG-CG, FP64 V-cycles, no learned part",
                             "value": n / pdt, "ms_per_step": 1e3 * pdt / n, **summary(pst)}
        out["speedup_vs_plain_fp64"] = value / out["plain_fp64"]["value"]
        if learned:
            bdt, bst = timed(lambda: P.solve_absorbing_fgmres(f, precond="schur")[2], n, 1)
            out["block_fgmres_fp64"] = {"value": n / bdt, "ms_per_step": 1e3 * bdt / n, **summary(bst, True)}
        P.close()
        if learned:
            # with the coarse level still built: the paper's m = 5, and the Schur GMRES
            bdt5, bst5 = timed(lambda: S.solve_absorbing_fgmres(f, precond="learned", m=5, n=1, restart=30)[2], n, 1)
            out["block_fgmres_learned_coarse_m5_fp32"] = {"value": n / bdt5, "ms_per_step": 1e3 * bdt5 / n,
                                                          **summary(bst5, True)}
            kdt, kst = timed(lambda: S.solve_absorbing(f)[2], n, 1)
            out["schur_gmres_learned_coarse_fp32"] = {"value": n / kdt, "ms_per_step": 1e3 * kdt / n,
                                                      "coarse_columns": coarse["columns"],
                                                      "coarse_build_ms": coarse["build_ms"], **summary(kst)}
            # and without it: W alone
            S.coarse_clear()
            wdt, wst = timed(lambda: S.solve_absorbing_fgmres(f, precond="learned", m=5, n=1, restart=30)[2], n, 1)
            out["block_fgmres_learned_fp32"] = {"value": n / wdt, "ms_per_step": 1e3 * wdt / n, **summary(wst, True)}
            sdt, sst = timed(lambda: S.solve_absorbing(f)[2], n, 1)
            out["schur_gmres_learned_fp32"] = {"value": n / sdt, "ms_per_step": 1e3 * sdt / n, **summary(sst)}
            M = BlobRD(inst.n, q, precision=MIXED, rtol=rtol)
            if args.autotune:
                M.autotune(reps=10)
            mdt, mst = timed(lambda: M.solve_absorbing(f)[2], n, 1)
            out["schur_gmres_fp32"] = {"value": n / mdt, "ms_per_step": 1e3 * mdt / n, **summary(mst)}
            cdt, cst = timed(lambda: M.solve_absorbing_fgmres(f, precond="schur")[2], n, 1)
            out["block_fgmres_fp32"] = {"value": n / cdt, "ms_per_step": 1e3 * cdt / n, **summary(cst, True)}
            M.close()
            # the three-point kernel as a throughput variant (27-cell support instead of 64)
            M3 = BlobRD(inst.n, q, precision=MIXED, rtol=rtol, kernel_w=3)
            tdt, tst = timed(lambda: M3.solve_absorbing_fgmres(f, precond="schur")[2], n, 1)
            out["block_fgmres_fp32_kernel_w3"] = {"value": n / tdt, "ms_per_step": 1e3 * tdt / n, **summary(tst, True)}
            M3.close()
            lat = W.cubic_lattice(random_f=True)
            lf = torch.tensor(lat.f, device=dev)
            L = BlobRD(lat.n, torch.tensor(lat.q, device=dev), precision=MIXED, rtol=rtol)
            ldt, lst = timed(lambda: L.solve_absorbing(lf)[2], 5, 1)
            lbdt, lbst = timed(lambda: L.solve_absorbing_fgmres(lf, precond="schur")[2], 5, 1)
            L2 = BlobRD(lat.n, torch.tensor(lat.q, device=dev), precision=FP64, rtol=rtol)
            l2dt, l2st = timed(lambda: L2.solve_absorbing(lf)[2], 5, 1)
            out["lattice128_randf"] = {"fp32_value": 5 / ldt, "plain_fp64_value": 5 / l2dt,
                                       "block_fgmres_fp32_value": 5 / lbdt, **summary(lst),
                                       "block_fgmres": summary(lbst, True)}
            L.close()
            L2.close()
            # the same suspension size in a box held at c_inf = 1 (Sec. IV.C): block FGMRES on the
            # lifted system, box multigrid kernels in FP32
            bx = W.box_suspension(inst.n, inst.N)
            Bx = BlobRD(bx.n, torch.tensor(bx.q, device=dev), precision=MIXED, rtol=rtol,
                        boundary=BOUNDARY_DIRICHLET, boundary_value=1.0)
            bf = torch.tensor(bx.f, device=dev)
            xdt, xst = timed(lambda: Bx.solve_absorbing_fgmres(bf, precond="schur")[2], n, 1)
            gms, gby = Bx.time_kernel("gs", args.kernel_reps, cold=True)
            out["dirichlet_box256_block_fgmres_fp32"] = {
                "value": n / xdt, "ms_per_step": 1e3 * xdt / n, "N": bx.N, "seed": bx.seed, **summary(xst, True),
                "gs_box_cold_us": gms * 1e3, "gs_box_cold_GBs": gby / (gms * 1e-3) / 1e9}
            Bx.close()
            # the 64 uneven suspensions of the batched workload
            _say("batch64")
            out["batch64"] = bench_batch(args, dev, rtol, 4, 1)

    # Roofline of the dominant kernel: the finest-level Gauss-Seidel half-sweep
    # (FP32), timed with HIP events on the handle's stream. Cold: back-to-back
    # launches rotating over buffer sets larger than the 256 MB Infinity Cache
    # (HBM bandwidth); warm: back-to-back launches on the same data.
    ms, by = S.time_kernel("gs", args.kernel_reps, cold=True)
    wms, _ = S.time_kernel("gs", args.kernel_reps)
    # the streaming ceiling of a launch this size: out = a + b over three arrays of the same size,
    # in the sweep's launch shape, rotating cold the same way
    pms, pby = S.time_kernel("stream", args.kernel_reps, cold=True)
    ach = by / (ms * 1e-3) / 1e9
    out["roofline"] = {"kernel": "k_gs_box_vec<float> finest level" if box else "k_gs_vec<float> finest level",
                       "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS,
                       "traffic": None if box else measured_traffic(inst.n), "avg_us": ms * 1e3, "bytes_per_launch": by,
                       "warm_avg_us": wms * 1e3, "warm_GBs": by / (wms * 1e-3) / 1e9,
                       "stream_probe": {"avg_us": pms * 1e3, "GBs": pby / (pms * 1e-3) / 1e9,
                                        "frac": pby / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                        "sweep_over_probe": (by / ms) / (pby / pms)}}
    kern = {}
    for k in ("stencil", "restrict", "prolong", "vcycle"):
        kms, kby = S.time_kernel(k, max(10, args.kernel_reps // 4))
        kern[k] = {"avg_us": kms * 1e3, "alg_GBs": kby / (kms * 1e-3) / 1e9, "bytes": kby}
    # the FP64 stencil of the Krylov vectors, cold (rotating buffer sets larger than the
    # Infinity Cache): its HBM bandwidth as a fraction of the peak
    kms, kby = S.time_kernel("stencil", args.kernel_reps, cold=True)
    kern["stencil"].update({"cold_avg_us": kms * 1e3, "cold_GBs": kby / (kms * 1e-3) / 1e9,
                            "cold_frac": kby / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS})
    # the same stencil without the CG dots, the form the block solver applies
    wms, wby = S.time_kernel("stencil_plain", max(10, args.kernel_reps // 4))
    kms, kby = S.time_kernel("stencil_plain", args.kernel_reps, cold=True)
    kern["stencil_plain"] = {"avg_us": wms * 1e3, "alg_GBs": wby / (wms * 1e-3) / 1e9, "bytes": wby,
                             "cold_avg_us": kms * 1e3, "cold_GBs": kby / (kms * 1e-3) / 1e9,
                             "cold_frac": kby / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    out["kernels"] = kern
    S.close()
    if net is not None:
        net.close()

    if not args.no_cpu_baseline and not box:
        out["cpu_baseline"] = cpu_baseline(inst)
    if args.copy_probe:
        src = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 8
    print(json.dumps(out))


if __name__ == "__main__":
    main()
