"""Train the learned Schur preconditioner on synthetic suspensions and save the weights.

Training configurations are random sequential addition (minimum separation
3h) suspensions of 10^4 blobs in a 256^3 box (smaller proxies at the same
density can be chosen with --n/--blobs). For each configuration the library computes S
sample pairs (x_s, P M P x_s) with its own multigrid-preconditioned Schur
products; training then runs the library's forward/backward kernels and
Adam. Held-out evaluation compares GMRES iterations and wall time of the
absorbing solve (f = 1, rtol 1e-8) with and without the learned part.

Usage:
  python -m paper_1306_3159_amd.train_precond --configs 500 --epochs 30 \\
      --out paper_1306_3159_amd/weights/precond_rsa.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "precond_rsa.npy")


def log(msg):
    print(msg, flush=True)


def _positions(arg):
    """Blob positions of training configuration i (seeded; runs in a worker process)."""
    import workloads as W
    i, n, blobs = arg
    return W.training_config(i, n, blobs).q


def evaluate(net, spec_list: str, dev, W, LD, MIXED, FP64):
    """Held-out absorbing solves (f = 1) with and without the network: Schur GMRES (plain FP64,
    FP32 cycles, learned, and both with the 80-column Fourier coarse level, |m|^2 <= 6) and the
    block FGMRES (diagonal, approximate Schur, learned inner, learned inner with the coarse level
    at m = 5 and m = 3)."""
    import torch
    rows = []
    for spec in spec_list.split(","):
        if not spec:
            continue
        n, N, cnt = (int(v) for v in spec.split(":"))
        for k in range(cnt):
            inst = W.learned_eval(n, N, index=100 + k) if n == 256 else W.training_config(900_000 + k, n, N)
            f = torch.ones((n, n, n), dtype=torch.float64, device=dev)
            row = {"n": n, "N": N, "seed": inst.seed}
            runs = (("plain_fp64", None, FP64, LD.gmres_iterations, {}),
                    ("mixed", None, MIXED, LD.gmres_iterations, {}),
                    ("learned_mixed", net, MIXED, LD.gmres_iterations, {}),
                    ("coarse_mixed", None, MIXED, LD.gmres_iterations, {"coarse_m2": 6}),
                    ("learned_coarse_mixed", net, MIXED, LD.gmres_iterations, {"coarse_m2": 6}),
                    ("block_diagonal_mixed", None, MIXED, LD.block_iterations, {"kind": "diagonal"}),
                    ("block_mixed", None, MIXED, LD.block_iterations, {}),
                    ("block_learned_mixed", net, MIXED, LD.block_iterations, {}),
                    ("block_learned_coarse_mixed", net, MIXED, LD.block_iterations, {"coarse_m2": 6}),
                    ("block_learned_coarse_m3_mixed", net, MIXED, LD.block_iterations, {"coarse_m2": 6, "m": 3}))
            for name, netx, prec, fn, kw in runs:
                st, dt, c, lam = fn(n, inst.q, f, netx, dev, precision=prec, **kw)
                row[name] = {"iters": st["outer_iters"], "inner_iters": st["inner_iters_total"],
                             "vcycles": st["vcycles"], "seconds": dt, "rel_resid": st["rel_resid"], "rc": st["rc"],
                             "fallback": st["fallback"]}
                if "coarse_m2" in kw:
                    row[name]["coarse_build_seconds"] = st["coarse_build_seconds"]
                log(f"eval n={n} N={N} seed={inst.seed} {name}: iters={st['outer_iters']} "
                    f"inner={st['inner_iters_total']} t={dt:.3f}s resid={st['rel_resid']:.2e}")
            rows.append(row)
    return rows


def summarize(rows):
    """Median iterations and seconds per method over the evaluated configurations."""
    out = {}
    if not rows:
        return out
    for name in [k for k in rows[0] if isinstance(rows[0][k], dict)]:
        its = [r[name]["iters"] for r in rows]
        sec = [r[name]["seconds"] for r in rows]
        out[name] = {"median_iters": float(np.median(its)), "median_seconds": float(np.median(sec)),
                     "max_rel_resid": max(r[name]["rel_resid"] for r in rows), "configs": len(rows)}
        if "coarse_build_seconds" in rows[0][name]:
            out[name]["median_coarse_build_seconds"] = float(np.median([r[name]["coarse_build_seconds"]
                                                                        for r in rows]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, default=500)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--blobs", type=int, default=10000)
    ap.add_argument("--smooth", type=float, default=0.5, help="fraction of smooth sample vectors")
    ap.add_argument("--samples", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--eval", default="256:10000:2", help="comma list of n:blobs:count held-out sets")
    ap.add_argument("--lr-final", type=float, default=None,
                    help="cosine-decay the learning rate to this value over the epochs (default: constant)")
    ap.add_argument("--workers", type=int, default=1, help="host processes generating the configurations")
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="skip training: evaluate these saved weights on the --eval sets and print the report")
    ap.add_argument("--init", default=None, metavar="WEIGHTS",
                    help="start from these saved weights instead of the seeded initial ones")
    ap.add_argument("--cycles", type=int, default=0,
                    help="train against the approximate-Schur operator with this many multigrid cycles per product "
                         "(the block preconditioner's inner operator); 0: Schur products with inner solves")
    args = ap.parse_args(argv)

    import torch
    import workloads as W
    from paper_1306_3159_amd import Net, MIXED, FP64
    from paper_1306_3159_amd import learned as LD

    dev = torch.device("cuda:0")
    t0 = time.time()
    if args.eval_only:
        net = Net(dev)
        net.set_params(torch.tensor(np.load(args.eval_only), device=dev))
        report = {"weights": args.eval_only, "eval": evaluate(net, args.eval, dev, W, LD, MIXED, FP64)}
        report["summary"] = summarize(report["eval"])
        log("REPORT " + json.dumps(report))
        return
    samples = []
    pool = None
    if args.workers > 1:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(args.workers)
        positions = pool.imap(_positions, [(i, args.n, args.blobs) for i in range(args.configs)], chunksize=4)
    else:
        positions = (_positions((i, args.n, args.blobs)) for i in range(args.configs))
    for i, q in enumerate(positions):
        samples.append(LD.harvest(args.n, q, args.samples, 1306_700_000 + i, dev, smooth_fraction=args.smooth,
                                  cycles=args.cycles))
        if (i + 1) % 50 == 0:
            log(f"harvested {i + 1}/{args.configs} configurations ({time.time() - t0:.1f}s)")
    if pool is not None:
        pool.close()
    net = Net(dev)
    init = np.load(args.init) if args.init else LD.initial_params(args.seed)
    net.set_params(torch.tensor(init, device=dev))
    hist = LD.train(net, samples, args.epochs, args.lr, args.batch, dev, seed=args.seed, log=log,
                    lr_final=args.lr_final)
    params = net.get_params().cpu().numpy()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params)
    log(f"saved {args.out}")
    report = {"configs": args.configs, "n": args.n, "blobs": args.blobs, "samples": args.samples,
              "epochs": args.epochs, "lr": args.lr, "lr_final": args.lr_final, "batch": args.batch,
              "smooth": args.smooth, "seed": args.seed, "cycles": args.cycles, "init": args.init, "loss": hist,
              "train_seconds": time.time() - t0, "eval": []}
    report["eval"] = evaluate(net, args.eval, dev, W, LD, MIXED, FP64)
    report["summary"] = summarize(report["eval"])
    log("REPORT " + json.dumps(report))


if __name__ == "__main__":
    main()
