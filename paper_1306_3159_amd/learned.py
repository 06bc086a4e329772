"""Training driver of the learned Schur preconditioner (loop control only).

Samples come from the method itself: for a blob configuration and seeded
mean-zero random vectors x_s, the library computes y_s = P M P x_s with
M = J (-D L)^+ S (one multigrid-CG Poisson solve per sample,
blob_rd_schur_apply). Training then minimises
(1/S) sum_s |P W y_s - x_s|^2 / |x_s|^2 over the configurations with the
library's forward/backward kernels and Adam; W is rebuilt from the current
network for every configuration visited.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

from .native import BlobRD, Net, MIXED, PRECOND_LEARNED, PRECOND_NONE, NET_PARAMS


def initial_params(seed: int = 0) -> np.ndarray:
    """Seeded starting weights as one float32 vector in the library's parameter layout
    [W1 (64x12) | b1 | W2 (64x64) | b2 | w3 | b3]: He-scaled normal hidden layers and a
    zero output layer, so the untrained network reproduces the diagonal preconditioner."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((64, 12)) * np.sqrt(2.0 / 12)
    w2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    v = np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), np.zeros(64), np.zeros(1)])
    assert v.size == NET_PARAMS
    return v.astype(np.float32)


@dataclasses.dataclass
class Sample:
    shape: tuple
    q: np.ndarray          # (N, 3) positions
    X: torch.Tensor        # (S, N) device, mean-zero rows
    Y: torch.Tensor        # (S, N) device, Y_s = P M P X_s


def sample_vectors(q: np.ndarray, box, n_samples: int, seed: int, smooth_fraction: float = 0.5,
                   kmax2: int = 4) -> np.ndarray:
    """Seeded mean-zero blob vectors: white noise, and (for a fraction of them) smooth fields
    sum_k a_k cos(2 pi k.q/L) + b_k sin(2 pi k.q/L) over the wave vectors 0 < |k|^2 <= kmax2,
    which carry the slowly varying modes of the Schur complement."""
    rng = np.random.default_rng(seed)
    N = q.shape[0]
    X = rng.standard_normal((n_samples, N))
    n_smooth = int(round(smooth_fraction * n_samples))
    if n_smooth:
        r = int(np.floor(np.sqrt(kmax2)))
        ks = np.array([(a, b, c) for a in range(-r, r + 1) for b in range(-r, r + 1) for c in range(-r, r + 1)
                       if 0 < a * a + b * b + c * c <= kmax2], dtype=np.float64)
        ph = 2.0 * np.pi * (q / np.asarray(box, dtype=np.float64)) @ ks.T        # (N, K)
        for s in range(n_smooth):
            a = rng.standard_normal(ks.shape[0])
            b = rng.standard_normal(ks.shape[0])
            X[s] = np.cos(ph) @ a + np.sin(ph) @ b
    X -= X.mean(axis=1, keepdims=True)
    return X


def harvest(shape, q: np.ndarray, n_samples: int, seed: int, device, inner_rtol: float = 1e-8,
            precision: int = MIXED, smooth_fraction: float = 0.5, h: float = 1.0, cycles: int = 0) -> Sample:
    """Schur products of seeded sample vectors for one configuration: with inner solves to
    inner_rtol (cycles = 0), or the approximate-Schur operator with `cycles` multigrid cycles
    per product (the operator the block preconditioner's inner GMRES applies)."""
    dims = (shape,) * 3 if isinstance(shape, int) else tuple(shape)
    box = (dims[2] * h, dims[1] * h, dims[0] * h)      # (x, y, z) edges
    X = sample_vectors(q, box, n_samples, seed, smooth_fraction)
    Xd = torch.tensor(X, device=device)
    S = BlobRD(shape, torch.tensor(q, device=device), precision=precision)
    if cycles > 0:
        Y = torch.stack([S.schur_apply_cycles(Xd[s].contiguous(), 0.0, cycles) for s in range(n_samples)])
    else:
        Y = torch.stack([S.schur_apply(Xd[s], 0.0, inner_rtol) for s in range(n_samples)])
    S.close()
    return Sample(tuple(shape) if not isinstance(shape, int) else (shape,) * 3, q, Xd, Y)


def loss_and_grad(net: Net, samples: Sequence[Sample], device) -> float:
    """Accumulate the gradient over configurations into the network; returns the mean loss."""
    total = 0.0
    for smp in samples:
        S = BlobRD(smp.shape, torch.tensor(smp.q, device=device))
        S.precond_build(net)
        total += S.precond_loss_grad(net, smp.X, smp.Y)
        S.close()
    return total / max(1, len(samples))


def train(net: Net, samples: List[Sample], epochs: int, lr: float, batch: int, device, seed: int = 0,
          log: Optional[Callable[[str], None]] = None, lr_final: Optional[float] = None) -> List[float]:
    """Adam over mini-batches of configurations; returns the mean loss per epoch. With lr_final
    the step size follows a cosine from lr down to lr_final over the epochs."""
    rng = np.random.default_rng(seed)
    hist = []
    base = lr
    for ep in range(epochs):
        if lr_final is not None and epochs > 1:
            lr = lr_final + 0.5 * (base - lr_final) * (1.0 + np.cos(np.pi * ep / (epochs - 1)))
        order = rng.permutation(len(samples))
        losses = []
        t0 = time.time()
        for b0 in range(0, len(order), batch):
            net.zero_grad()
            sub = [samples[i] for i in order[b0:b0 + batch]]
            losses.append(loss_and_grad(net, sub, device))
            net.adam_step(lr)
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f} ({time.time() - t0:.1f}s)")
    return hist


def block_iterations(shape, q: np.ndarray, f: torch.Tensor, net: Optional[Net], device, rtol: float = 1e-8,
                     precision: int = MIXED, m: int = 5, kind: Optional[str] = None, coarse_m2: int = 0,
                     coarse_rtol: float = 1e-4):
    """Block FGMRES iterations and wall time of one absorbing solve with the approximate-Schur
    preconditioner, its inner GMRES preconditioned by W (net) or not (or kind = "diagonal"); with
    coarse_m2 > 0 (and a net) by the two-level B of the Fourier coarse level around W (its build
    time is returned in the stats as coarse_build_seconds, outside the solve's time)."""
    S = BlobRD(shape, torch.tensor(q, device=device), precision=precision, rtol=rtol,
               schur_precond=PRECOND_LEARNED if net is not None else PRECOND_NONE)
    if net is not None:
        S.precond_build(net)
    tb = 0.0
    if coarse_m2 > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.coarse_build(0.0, coarse_m2, coarse_rtol)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    kind = kind or ("learned" if net is not None else "schur")
    S.solve_absorbing_fgmres(f, precond=kind, m=m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, lam, st = S.solve_absorbing_fgmres(f, precond=kind, m=m)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.close()
    st["coarse_build_seconds"] = tb
    return st, dt, c, lam


def gmres_iterations(shape, q: np.ndarray, f: torch.Tensor, net: Optional[Net], device, rtol: float = 1e-8,
                     precision: int = MIXED, coarse_m2: int = 0, coarse_rtol: float = 1e-4):
    """Schur GMRES iterations and wall time of one absorbing solve, with or without W, and with
    the Fourier coarse level over 0 < |m|^2 <= coarse_m2 (0: none; its build time is returned
    in the stats as coarse_build_seconds, outside the solve's time)."""
    S = BlobRD(shape, torch.tensor(q, device=device), precision=precision, rtol=rtol,
               schur_precond=PRECOND_LEARNED if net is not None else PRECOND_NONE)
    if net is not None:
        S.precond_build(net)
    tb = 0.0
    if coarse_m2 > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.coarse_build(0.0, coarse_m2, coarse_rtol)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    c, lam, st = S.solve_absorbing(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, lam, st = S.solve_absorbing(f)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.close()
    st["coarse_build_seconds"] = tb
    return st, dt, c, lam
