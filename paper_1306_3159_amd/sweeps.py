"""Validation sweeps of Sec. IV on the GPU (reaction radius and effective reaction rates).

Each sweep solves single-blob periodic cells (a blob in an L^3 box is a simple-cubic array
of blobs with spacing L h) with the library and reduces the answer by the paper's formulas:

* eq. beta0_low_phi: with a uniform source s and s V = 1, the steady absorbing solution has
  mean concentration cbar and a_L = [4 pi D cbar]^{-1};
* eq. a_phi: a_L = a (1 + x + x^2), x = 2.84 a / (L h), inverted for the infinite-box radius a;
* eq. beta_P_disc: beta_P = (s a^2 / D) (1 - phi) / (3 phi) (1 + P) / cbar, phi = 4 pi a^3 / (3 V);
* eq. P_def: kappa = 4 pi D a / P for a finite reaction rate;
* eq. Omega: Omega = [(s a^2 / D)(1 - phi) / (3 phi) / cbar]^{-1}.

Sweeps: the radius at a grid node against box size (Fig. ReactionRadius left), its variation
as the blob moves off the node (right), beta_0 of cubic arrays against the fit eq.
beta_cubic, Omega(P) and beta_P at finite P (Figs. finite_P_fit, finite_P_01), the
iteration counts of the reactive steady solve of (L/4)^3 lattices against P~ (Fig.
NonSaddleGMRES; the curves are not printed, so only the counts are reported), and the far
field of one absorbing blob in a box held at c_inf (Fig. FarFieldDecay, eq. c_r_approx).

Run: python -m paper_1306_3159_amd.sweeps --out results.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, List, Sequence

import numpy as np
import torch

from .native import BlobRD, FP64, MIXED, SOLVER_BLOCK, BOUNDARY_DIRICHLET

# Values the paper prints (Sec. IV.A, IV.B).
PAPER = {"radius_node_w4": 1.27, "radius_node_w3": 0.885, "radius_average_w4": 1.255,
         "variation_w4": 0.015, "variation_w3": 0.05, "beta_cubic_b": -0.92, "beta_cubic_c": 17.4,
         "beta_lead": 1.76, "a_phi_coeff": 2.84}


def radius_extrapolated(aL: float, L: float, h: float = 1.0) -> float:
    """Solve a (1 + x + x^2) = a_L, x = 2.84 a / (L h), for a (monotone in a: bisection)."""
    lo, hi = 0.0, aL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x = PAPER["a_phi_coeff"] * mid / (L * h)
        if mid * (1.0 + x + x * x) < aL:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def beta_cubic_fit(phi: float) -> float:
    """eq. beta_cubic with the paper's fitted b and c."""
    l = PAPER["beta_lead"]
    return (1.0 + l * phi ** (1 / 3) + l ** 2 * phi ** (2 / 3) + PAPER["beta_cubic_b"] * phi
            + PAPER["beta_cubic_c"] * phi ** (4 / 3))


def _cell_mean(n: int, q, dev, w: int, kappa=None, precision=FP64, rtol=1e-10) -> float:
    """Mean concentration of the steady single-blob cell with source s = 1/V (absorbing when
    kappa is None, reactive with rate kappa otherwise). On large boxes the FP64 rounding floor
    of the residual can sit above rtol; a solve that stops there is accepted down to 1e-8,
    ample for the radii and rates (relative accuracy ~1e-6 and better)."""
    V = float(n ** 3)
    f = torch.full((n, n, n), 1.0 / V, dtype=torch.float64, device=dev)
    qt = torch.tensor(np.asarray(q, dtype=np.float64).reshape(1, 3), device=dev)
    if kappa is None:
        S = BlobRD(n, qt, kernel_w=w, precision=precision, rtol=rtol, saddle_solver=SOLVER_BLOCK, gmres_restart=10)
        c, lam, st = S.solve_absorbing(f)
    else:
        S = BlobRD(n, qt, torch.tensor([float(kappa)], dtype=torch.float64, device=dev), kernel_w=w,
                   precision=precision, rtol=rtol)
        c, st = S.solve_reactive(f)
    if st["rc"] < 0 or st["rel_resid"] > max(rtol, 1e-8):
        raise RuntimeError(f"solve did not converge: {st}")
    m = float(c.mean())
    S.close()
    return m


def radius(n: int, q, dev, w: int = 4) -> Dict[str, float]:
    """a_L and the extrapolated a of one blob at q in an n^3 box (h = D = 1). The cell's
    source is s = 1/V, so the sink absorbs s V = 1 and a_L = s V / (4 pi D cbar) = 1/(4 pi cbar)."""
    cbar = _cell_mean(n, q, dev, w)
    sV = 1.0
    aL = sV / (4.0 * math.pi * cbar)
    return {"L": n, "a_L": aL, "a": radius_extrapolated(aL, n), "cbar": cbar}


def sweep_radius_node(dev, Ls: Sequence[int] = (16, 32, 64, 128, 256), w: int = 4) -> List[dict]:
    """Fig. ReactionRadius (left): the radius of a blob at a grid node against box size."""
    return [{**radius(L, [L / 2.0] * 3, dev, w), "w": w} for L in Ls]


def sweep_translation(dev, L: int = 128, w: int = 4, fractions=(0.0, 0.25, 0.5, 0.75, 1.0),
                      directions=((1, 0, 0), (1, 1, 0), (1, 1, 1))) -> dict:
    """Fig. ReactionRadius (right): a (extrapolated) as the blob moves from a cell centre
    towards a face (1,0,0), an edge (1,1,0) or a node (1,1,1) of the cell, a fraction t of the
    way (offset t/2 per moving axis, distance delta from the centre); returns the rows and the
    relative spread (max - min) / mean."""
    rows = []
    c0 = L / 2.0 + 0.5  # a cell centre
    for d in directions:
        dv = np.asarray(d, dtype=np.float64)
        for t in fractions:
            off = 0.5 * t * dv
            r = radius(L, c0 + off, dev, w)
            rows.append({"direction": list(d), "delta": float(np.linalg.norm(off)), "a": r["a"]})
    a = np.array([r["a"] for r in rows])
    return {"w": w, "L": L, "rows": rows, "mean": float(a.mean()), "spread": float((a.max() - a.min()) / a.mean())}


def sweep_beta0_cubic(dev, ns: Sequence[int] = (8, 10, 12, 16, 24, 32, 64), w: int = 4) -> List[dict]:
    """Fig. PerDisp: beta_0 of simple-cubic arrays (one blob at a node of an n^3 cell) against
    phi, beside the fit eq. beta_cubic; a is the paper's node radius."""
    a = PAPER["radius_node_w4"] if w == 4 else PAPER["radius_node_w3"]
    out = []
    for n in ns:
        V = float(n ** 3)
        s = 1.0 / V
        phi = 4.0 * math.pi * a ** 3 / (3.0 * V)
        cbar = _cell_mean(n, [n / 2.0] * 3, dev, w)
        beta0 = s * a * a * (1.0 - phi) / (3.0 * phi) / cbar
        out.append({"n": n, "phi": phi, "beta0": beta0, "fit": beta_cubic_fit(phi)})
    return out


def sweep_finite_P(dev, n: int = 32, Ps: Sequence[float] = (0.0, 0.1, 0.3, 1.0, 3.0, 10.0), w: int = 4) -> List[dict]:
    """Figs. finite_P_fit, finite_P_01: Omega(P) and beta_P of a cubic array (one blob at a
    node of an n^3 cell) with kappa = 4 pi D a / P (eq. P_def); P = 0 is the absorbing limit."""
    a = PAPER["radius_node_w4"] if w == 4 else PAPER["radius_node_w3"]
    V = float(n ** 3)
    s = 1.0 / V
    phi = 4.0 * math.pi * a ** 3 / (3.0 * V)
    out = []
    for P in Ps:
        q = [n / 2.0] * 3
        cbar = _cell_mean(n, q, dev, w) if P == 0.0 else _cell_mean(n, q, dev, w, kappa=4.0 * math.pi * a / P)
        k = s * a * a * (1.0 - phi) / (3.0 * phi) / cbar
        out.append({"P": P, "phi": phi, "Omega": 1.0 / k, "beta_P": k * (1.0 + P)})
    return out


def sweep_reactive_convergence(dev, Ls: Sequence[int] = (32, 64, 128),
                               Ptildes: Sequence[float] = (4 * math.pi * 1e-4, 1.0, math.inf),
                               rtol: float = 1e-8) -> List[dict]:
    """Fig. NonSaddleGMRES: the steady reactive system of (L/4)^3 blobs 4 cells apart with
    P~ = 4 pi D h / kappa; multigrid-preconditioned CG iterations and V-cycles to rtol
    (kappa = 0 for P~ = inf is a pure Poisson problem with a singular operator; it is solved
    with alpha = 1/L^2 as the paper's tests do for A). The source is f = 1 + 0.5 N(0, 1)
    (seeded): a uniform source on the symmetric lattice excites only the lattice-periodic modes
    and converges in a handful of iterations whatever P~."""
    out = []
    for L in Ls:
        pts = np.arange(2.0, L, 4.0)
        q = np.stack(np.meshgrid(pts, pts, pts, indexing="ij"), -1).reshape(-1, 3)
        qt = torch.tensor(q, device=dev)
        rng = np.random.default_rng(1306_300 + L)
        f = torch.tensor(1.0 + 0.5 * rng.standard_normal((L, L, L)), device=dev)
        for Pt in Ptildes:
            kappa = 0.0 if math.isinf(Pt) else 4.0 * math.pi / Pt
            kt = torch.full((q.shape[0],), kappa, dtype=torch.float64, device=dev)
            S = BlobRD(L, qt, kt, precision=MIXED, rtol=rtol, max_iter=5000)
            alpha = 1.0 / L ** 2 if kappa == 0.0 else 0.0
            t0 = time.perf_counter()
            c, st = S.solve_reactive(f, alpha=alpha)
            torch.cuda.synchronize()
            out.append({"L": L, "blobs": int(q.shape[0]), "Ptilde": Pt, "cg_iters": st["outer_iters"],
                        "vcycles": st["vcycles"], "rel_resid": st["rel_resid"], "rc": st["rc"],
                        "seconds": time.perf_counter() - t0})
            S.close()
    return out


def _lattice(L: int, spacing: float, offset: float) -> np.ndarray:
    pts = np.arange(offset, L, spacing)
    return np.stack(np.meshgrid(pts, pts, pts, indexing="ij"), -1).reshape(-1, 3)


def _saddle_case(dev, L: int, q: np.ndarray, f: torch.Tensor, alpha: float, runs) -> dict:
    """Solve one saddle point (eq. saddle_point) by each (name, kind, m, restart) of `runs` with the block
    FGMRES (n = 1, FP64 cycles), and by the Schur-complement GMRES of the other layout."""
    qt = torch.tensor(q, device=dev)
    out = {"L": L, "blobs": int(q.shape[0]), "alpha": alpha}
    S = BlobRD(L, qt, precision=FP64, rtol=1e-8, max_iter=4000, gmres_restart=30)
    for name, kind, m, restart in runs:
        t0 = time.perf_counter()
        c, lam, st = S.solve_absorbing_fgmres(f, alpha=alpha, precond=kind, m=m, n=1, restart=restart, maxit=4000)
        torch.cuda.synchronize()
        out[name] = {"fgmres_iters": st["outer_iters"], "vcycles": st["vcycles"], "rel_resid": st["rel_resid"],
                     "rc": st["rc"], "seconds": time.perf_counter() - t0}
        print(f"[sweep]   L={L} N={q.shape[0]} alpha={alpha:g} {name}: {out[name]}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    c, lam, st = S.solve_absorbing(f, alpha=alpha)
    torch.cuda.synchronize()
    out["schur_gmres"] = {"gmres_iters": st["outer_iters"], "inner_cg_iters": st["inner_iters_total"],
                          "vcycles": st["vcycles"], "rel_resid": st["rel_resid"], "rc": st["rc"],
                          "seconds": time.perf_counter() - t0}
    print(f"[sweep]   L={L} schur_gmres: {out['schur_gmres']}", file=sys.stderr, flush=True)
    S.close()
    return out


def sweep_block_preconditioners(dev, Ls: Sequence[int] = (16, 32, 64, 128), m_L: int = 16,
                                ms: Sequence[int] = (1, 2, 3, 5, 8, 12, 16),
                                fixed_Ls: Sequence[int] = (16, 32, 64, 128, 256)) -> dict:
    """Figs. DiagonalScaling, InexactSchur, FixedNScaling (E4-E6): the block FGMRES with the diagonal
    preconditioner (n = 1, restart 200) and the approximate Schur complement (m = 5, n = 1, restart
    30) on periodic cubic arrays of absorbing blobs 4 cells apart ((L/4)^3 blobs, four-point kernel)
    with A = L^-2 I - L, beside the Schur-complement GMRES of the other layout; the approximate
    Schur complement with A = -L (null space handled as in the appendix); the m study at 16^3; and
    a fixed 64 = 4^3 blobs as L grows. The paper does not state the right-hand side: the source
    is f = 1 + 0.5 N(0, 1) (seeded), since a uniform source on a symmetric lattice excites only
    lattice-periodic modes. V-cycles count every multigrid cycle (m + 2n per outer iteration)."""
    runs = [("diagonal", "diagonal", 0, 200), ("approx_schur", "schur", 5, 30)]
    res = {"size": [], "singular": [], "m_study": None, "fixed_N": []}
    for L in Ls:
        rng = np.random.default_rng(1306_600 + L)
        f = torch.tensor(1.0 + 0.5 * rng.standard_normal((L, L, L)), device=dev)
        q = _lattice(L, 4.0, 2.0)
        res["size"].append(_saddle_case(dev, L, q, f, 1.0 / L ** 2, runs))
        res["singular"].append(_saddle_case(dev, L, q, f, 0.0, [("approx_schur", "schur", 5, 30)]))
        print(f"[sweep] block preconditioners L={L}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(1306_600 + m_L)
    f = torch.tensor(1.0 + 0.5 * rng.standard_normal((m_L, m_L, m_L)), device=dev)
    res["m_study"] = _saddle_case(dev, m_L, _lattice(m_L, 4.0, 2.0), f, 1.0 / m_L ** 2,
                                  [(f"m{m}", "schur", m, 30) for m in ms])
    for L in fixed_Ls:
        rng = np.random.default_rng(1306_700 + L)
        f = torch.tensor(1.0 + 0.5 * rng.standard_normal((L, L, L)), device=dev)
        res["fixed_N"].append(_saddle_case(dev, L, _lattice(L, L / 4.0, L / 8.0), f, 1.0 / L ** 2, runs))
        print(f"[sweep] fixed N L={L}", file=sys.stderr, flush=True)
    return res


def far_field_law(r, L: float, a: float):
    """eq. c_r_approx: c(r)/c_inf ~ L/(L - 2a) (1 - a/r), the spherical problem with c(a) = 0 and
    c(L/2) = c_inf."""
    return L / (L - 2.0 * a) * (1.0 - a / np.asarray(r, dtype=np.float64))


def sweep_far_field(dev, n: int = 96, w: int = 4, rmax_frac: float = 0.25) -> dict:
    """Fig. FarFieldDecay (E9): one absorbing blob at the centre node of an n^3 box held at
    c_inf = 1, no source (the paper's box has 100 cells per edge; the multigrid here needs an
    edge of the form 2^k times a small factor). Returns c along the +x axis and the (1,1,1)
    diagonal from the blob, the law with the position-averaged radius 1.255 h, the largest
    relative deviation from it for 3h <= r <= rmax_frac * n, and the radius a of a least-squares
    fit of c = A (1 - a/r) over the same range."""
    q = np.array([[n / 2.0] * 3])
    S = BlobRD(n, torch.tensor(q, device=dev), kernel_w=w, precision=FP64, rtol=1e-10, saddle_solver=SOLVER_BLOCK,
               boundary=BOUNDARY_DIRICHLET, boundary_value=1.0)
    c, lam, st = S.solve_absorbing(torch.zeros((n, n, n), dtype=torch.float64, device=dev))
    if st["rc"] < 0 or st["rel_resid"] > 1e-8:
        raise RuntimeError(f"solve did not converge: {st}")
    ch = c.cpu().numpy()
    S.close()
    k0 = n // 2  # cell centres k + 1/2: cell k0 sits half a cell from the blob along each axis
    ks = np.arange(k0, n)
    r_axis = np.sqrt((ks + 0.5 - n / 2.0) ** 2 + 2 * 0.25)
    c_axis = ch[k0, k0, ks]
    r_diag = np.sqrt(3.0) * (ks + 0.5 - n / 2.0)
    c_diag = ch[ks, ks, ks]
    a_paper = PAPER["radius_average_w4"] if w == 4 else PAPER["radius_node_w3"]
    r = np.concatenate([r_axis, r_diag])
    cv = np.concatenate([c_axis, c_diag])
    sel = (r >= 3.0) & (r <= rmax_frac * n)
    dev_rel = float(np.max(np.abs(cv[sel] / far_field_law(r[sel], n, a_paper) - 1.0)))
    M = np.stack([np.ones(int(sel.sum())), -1.0 / r[sel]], 1)
    (A, Aa), *_ = np.linalg.lstsq(M, cv[sel], rcond=None)
    return {"n": n, "w": w, "lambda": float(lam[0]), "r_axis": r_axis.tolist(), "c_axis": c_axis.tolist(),
            "r_diag": r_diag.tolist(), "c_diag": c_diag.tolist(), "a_paper": a_paper,
            "max_rel_dev_from_law": dev_rel, "fit_A": float(A), "fit_a": float(Aa / A),
            "fit_range": [3.0, rmax_frac * n]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="small sizes only")
    ap.add_argument("--only", default=None,
                    help="run one sweep (a result key) and replace that key in the --out file if it exists")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    t0 = time.time()
    q = args.quick
    sweeps = {
        "radius_node_w4": lambda: sweep_radius_node(dev, (16, 32) if q else (16, 32, 64, 128, 256), 4),
        "radius_node_w3": lambda: sweep_radius_node(dev, (16, 32) if q else (16, 32, 64, 128, 256), 3),
        "translation_w4": lambda: sweep_translation(dev, 32 if q else 128, 4),
        "translation_w3": lambda: sweep_translation(dev, 32 if q else 128, 3),
        "beta0_cubic": lambda: sweep_beta0_cubic(dev, (8, 16) if q else (8, 10, 12, 16, 24, 32, 64)),
        "finite_P": lambda: sweep_finite_P(dev, 16 if q else 32),
        "reactive_convergence": lambda: sweep_reactive_convergence(dev, (32,) if q else (32, 64, 128)),
        "far_field_w4": lambda: sweep_far_field(dev, 48 if q else 96, 4),
        "block_preconditioners": lambda: sweep_block_preconditioners(
            dev, (16, 32) if q else (16, 32, 64, 128), 16, (1, 3, 5, 8) if q else (1, 2, 3, 5, 8, 12, 16),
            (16, 32) if q else (16, 32, 64, 128, 256)),
    }
    if args.only is not None and args.only not in sweeps:
        raise SystemExit(f"--only must be one of {sorted(sweeps)}")
    res = {}
    if args.only and args.out and os.path.exists(args.out):
        with open(args.out) as fh:
            res = json.load(fh)
    for key, fn in sweeps.items():
        if args.only and key != args.only:
            continue
        t1 = time.time()
        res[key] = fn()
        print(f"[sweep] {key} {time.time() - t1:.1f} s", file=sys.stderr, flush=True)
    res["paper"] = PAPER
    if not args.only:
        res["seconds"] = time.time() - t0
    txt = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(txt)
    print(txt)


if __name__ == "__main__":
    main()
