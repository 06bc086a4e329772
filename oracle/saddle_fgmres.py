"""CPU FP64 oracle, part 4: the paper's own solver for the absorbing saddle point.

TEST INFRASTRUCTURE ONLY. Nothing in the product library may import, call or
link this module; only the tests, the smoke check and the benchmark's CPU
baseline use it. It shares no code with the HIP path.

The diffusion-limited system (eq. saddle_point with zeta = 1, the constraint
written J c = phi) is solved the way Sec. III.E (diffusion-limited case) and
the appendix on preconditioning the saddle-point solver describe it:

* a Krylov method on the whole block system [A, S; J, 0][c; lam] = [g; phi]:
  flexible GMRES (right preconditioned, so that the preconditioner may change
  from one application to the next; restarted; modified Gram-Schmidt);
* its preconditioner, an approximate solve of the same block system built
  from the Schur complement M = J A^{-1} S (eqs. c_exact, r_schur): a
  concentration estimate from n multigrid cycles, multipliers from either the
  single-blob diagonal M^{-1} ~ D gamma^{-1} (eq. Schur_diagonal) or m Krylov
  iterations on eq. approx_Schur with one cycle per product, then a corrected
  concentration from n more cycles started at the estimate;
* for A = -D L on the periodic grid (singular A) the appendix's extra
  handling: the mean multiplier fixed by the total source, mean-zero
  fluctuations, and the mean concentration recovered from the constraint.

The approximate inverse of A is a parameter (``ainv``), so the same steps run
with the oracle's multigrid cycles (parity with the GPU path) or with the
exact FFT inverse (the pins: with exact solves the preconditioner is an exact
inverse in the cases the paper's derivation makes exact).

Grid arrays have shape (nz, ny, nx); multipliers have length N.
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np

from . import exact as ex

# Reactive radius of a blob in units of h (Sec. IV.A): the position-averaged value of
# the four-point kernel and the three-point kernel's value at a node; the diagonal
# preconditioner takes gamma = 1/(4 pi a0).
A0_OVER_H = {4: 1.255, 3: 0.885}


class SaddleOps:
    """The blocks of the saddle-point matrix for one blob configuration."""

    def __init__(self, q, shape, alpha, D=1.0, h=1.0, w=4):
        self.q, self.shape, self.alpha, self.D, self.h, self.w = np.asarray(q, float), tuple(shape), alpha, D, h, w
        self.N = self.q.shape[0]
        self.ncell = int(np.prod(shape))

    def A(self, c):
        return ex.apply_A(c, self.alpha, self.D, self.h)

    def S(self, lam):
        return ex.spread(lam, self.q, self.shape, self.h, self.w)

    def J(self, c):
        return ex.interp(c, self.q, self.h, self.w)

    def K(self, c, lam):
        """[A, S; J, 0] [c; lam]."""
        return self.A(c) + self.S(lam), self.J(c)

    def exact_inverse(self):
        """u = A^{-1} r (the pseudo-inverse, mean-zero result, when alpha = 0)."""
        return lambda r: ex.solve_A(r, self.alpha, self.D, self.h)


def cycles_inverse(ops: SaddleOps, cycle: Callable[[np.ndarray], np.ndarray], n: int):
    """n multigrid cycles for A x = r as a stationary iteration: from a zero guess the first
    cycle is x = V r; every further cycle (or every cycle when a guess x0 is given) adds
    V (r - A x)."""
    def solve(r, x0=None):
        x = None if x0 is None else np.array(x0, dtype=float)
        for _ in range(n):
            if x is None:
                x = cycle(r)
            else:
                x = x + cycle(r - ops.A(x))
        return x
    return solve


def gmres_fixed(op: Callable[[np.ndarray], np.ndarray], b: np.ndarray, m: int) -> np.ndarray:
    """m iterations of GMRES from a zero guess (Arnoldi with modified Gram-Schmidt, no restart):
    the x in span{b, op b, ..., op^{m-1} b} that minimises |b - op x|. Stops early on an
    exact (happy) breakdown (a zero new direction)."""
    beta = float(np.linalg.norm(b))
    if beta == 0.0 or m <= 0:
        return np.zeros_like(b)
    V = [b / beta]
    Hm = np.zeros((m + 1, m))
    k = 0
    for j in range(m):
        wv = op(V[j])
        for i in range(j + 1):
            Hm[i, j] = float(np.dot(wv, V[i]))
            wv = wv - Hm[i, j] * V[i]
        Hm[j + 1, j] = float(np.linalg.norm(wv))
        k = j + 1
        if Hm[j + 1, j] == 0.0:
            break
        V.append(wv / Hm[j + 1, j])
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y = np.linalg.lstsq(Hm[:k + 1, :k], e1, rcond=None)[0]
    return sum(y[i] * V[i] for i in range(k))


def precondition(ops: SaddleOps, vg, vf, kind: str, ainv_n, ainv_1=None, m: int = 5,
                 diag: Optional[float] = None, w_apply: Optional[Callable] = None):
    """One application of the paper's saddle-point preconditioner to [vg; vf] (appendix on
    preconditioning the saddle-point solver, steps 1-5; Sec. III.E for the two variants).

    kind 'diagonal': multipliers lam~ = diag * h~ with diag = D/gamma = 4 pi a0 D by default
    (a0 from A0_OVER_H for the kernel).
    kind 'schur': m GMRES iterations on (J A1^{-1} S) lam~ = h~, A1^{-1} one cycle (ainv_1).
    kind 'learned': the same iterations right-preconditioned by an approximate inverse Schur
    complement w_apply (the learned P W P): (J A1^{-1} S W) y = h~, lam~ = W y.
    For the singular case (alpha = 0) the blob-space mean is projected out of h~, of every
    product of the inner Krylov operator and of lam~ (a mean offset of an approximate
    concentration only shifts J c by a constant, which that projection removes).
    Returns (c, lam)."""
    singular = ops.alpha == 0.0
    N, h3 = ops.N, ops.h ** 3
    proj = (lambda v: v - v.mean()) if singular else (lambda v: v)
    # 1. mean multiplier from the total source (singular A) and the concentration estimate
    lbar = h3 * float(np.sum(vg)) / N if singular else 0.0
    g_t = vg - ops.S(np.full(N, lbar))
    c_star = ainv_n(g_t)
    # 2. the Schur-complement system for the fluctuating multipliers
    h_t = proj(ops.J(c_star) - vf)
    if kind == "diagonal":
        lam_t = (4.0 * math.pi * A0_OVER_H[ops.w] * ops.h * ops.D if diag is None else diag) * h_t
    elif kind == "schur":
        lam_t = gmres_fixed(lambda v: proj(ops.J(ainv_1(ops.S(v)))), h_t, m)
    elif kind == "learned":
        y = gmres_fixed(lambda v: proj(ops.J(ainv_1(ops.S(w_apply(v))))), h_t, m)
        lam_t = w_apply(y)
    else:
        raise ValueError(kind)
    lam_t = proj(lam_t)
    # 3. corrected concentration, started from the estimate
    c_t = ainv_n(g_t - ops.S(lam_t), c_star)
    # 4. mean concentration from the constraint (singular A)
    if singular:
        c_t = c_t + float(np.mean(vf - ops.J(c_t)))
    # 5. the approximate solution
    return c_t, lam_t + lbar


def fgmres(apply_K, apply_P, bg, bf, restart=30, rtol=1e-8, maxit=1000):
    """Flexible GMRES (right preconditioned; the preconditioned directions Z are kept, so the
    preconditioner may change between applications), restarted every `restart` iterations,
    Arnoldi with modified Gram-Schmidt, from a zero initial guess. Vectors are pairs
    (grid, blobs); norms and dots run over both parts. Stops when the least-squares residual
    estimate is <= rtol |b|. Returns (xg, xf, info) with the residual estimate after every
    iteration in info['history']."""
    def dot(a, b):
        return float(np.sum(a[0] * b[0]) + np.sum(a[1] * b[1]))

    def axpy(a, x, y):
        return (y[0] + a * x[0], y[1] + a * x[1])

    bnorm = math.sqrt(dot((bg, bf), (bg, bf)))
    tol = rtol * bnorm
    x = (np.zeros_like(bg), np.zeros_like(bf))
    hist = []
    its = 0
    first = True
    while True:
        if first:
            r = (bg.copy(), bf.copy())
            first = False
        else:
            kg, kf = apply_K(*x)
            r = (bg - kg, bf - kf)
        beta = math.sqrt(dot(r, r))
        if beta <= tol or its >= maxit:
            break
        V = [(r[0] / beta, r[1] / beta)]
        Z = []
        Hm = np.zeros((restart + 1, restart))
        k = 0
        res = beta
        for j in range(restart):
            Z.append(apply_P(*V[j]))
            wv = apply_K(*Z[j])
            for i in range(j + 1):
                Hm[i, j] = dot(wv, V[i])
                wv = axpy(-Hm[i, j], V[i], wv)
            Hm[j + 1, j] = math.sqrt(dot(wv, wv))
            k = j + 1
            its += 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y = np.linalg.lstsq(Hm[:k + 1, :k], e1, rcond=None)[0]
            res = float(np.linalg.norm(e1 - Hm[:k + 1, :k] @ y))
            hist.append(res)
            if res <= tol or its >= maxit or Hm[j + 1, j] == 0.0:
                break
            V.append((wv[0] / Hm[j + 1, j], wv[1] / Hm[j + 1, j]))
        for i in range(k):
            x = axpy(y[i], Z[i], x)
        if res <= tol or its >= maxit:
            break
    return x[0], x[1], {"iters": its, "history": hist, "bnorm": bnorm}


def solve(f, q, alpha, kind="schur", m=5, n=1, restart=30, rtol=1e-8, maxit=1000, D=1.0, h=1.0, w=4,
          cycle: Optional[Callable] = None, phi=None, diag=None, w_apply=None):
    """[A, S; J, 0][c; lam] = [f; phi] by flexible GMRES with the paper's preconditioner.
    cycle: one multigrid cycle r -> V r for A (default: the exact inverse, i.e. n and the
    inner products become exact solves). Returns (c, lam, info)."""
    ops = SaddleOps(q, f.shape, alpha, D, h, w)
    cyc = ops.exact_inverse() if cycle is None else cycle
    ainv_n = cycles_inverse(ops, cyc, n)
    ainv_1 = cycles_inverse(ops, cyc, 1)
    phi = np.zeros(ops.N) if phi is None else np.asarray(phi, float)
    c, lam, info = fgmres(ops.K, lambda vg, vf: precondition(ops, vg, vf, kind, ainv_n, ainv_1, m, diag, w_apply),
                          np.asarray(f, float), phi, restart, rtol, maxit)
    return c, lam, info
