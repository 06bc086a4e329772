"""Seeded synthetic inputs for the blob reaction-diffusion solves.

This module only draws inputs: blob positions, blob rates and source fields.
It contains none of the method's arithmetic (no kernels, operators or
solvers), so both the CPU oracle and the GPU path can consume it.

Units: grid spacing h = 1 and diffusion coefficient D = 1 unless a workload
says otherwise. Positions are in grid units in [0, n). Grid fields are
float64 arrays of shape (nz, ny, nx), x fastest.

Workload shapes follow the paper's test problems: cubic lattices of blobs
(Sec. III.E, blobs 4 or 16 cells apart), a single blob in a periodic box
(Sec. IV.A) and random dispersions of non-overlapping spheres (Sec. IV.C).
The paper's random packings came from an external hard-sphere code that is
not available; random sequential addition (RSA) with a minimum separation
stands in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 1306_000


def seed_for(config: int, instance: int = 0) -> int:
    return SEED_BASE + 100 * config + instance


def _min_image(d: np.ndarray, box: float) -> np.ndarray:
    return d - box * np.round(d / box)


def rsa_positions(rng: np.random.Generator, n: int, count: int, dmin: float = 3.0,
                  max_tries: int = 200_000_000) -> np.ndarray:
    """Random sequential addition in the periodic box [0, n)^3.

    Candidates are drawn uniformly; a candidate closer than ``dmin`` (minimum
    image) to an accepted point is rejected. A cell list with cells at least
    ``dmin`` wide keeps each test local.
    """
    if count == 0:
        return np.zeros((0, 3))
    ncell = max(1, int(math.floor(n / dmin)))
    csize = n / ncell
    cells: dict = {}
    out = np.empty((count, 3))
    k = 0
    tries = 0
    batch = 4096
    while k < count:
        cand = rng.uniform(0.0, n, size=(batch, 3))
        for p in cand:
            tries += 1
            if tries > max_tries:
                raise RuntimeError(f"RSA could not place {count} points (placed {k})")
            c = tuple((p // csize).astype(int) % ncell)
            ok = True
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        key = ((c[0] + dx) % ncell, (c[1] + dy) % ncell, (c[2] + dz) % ncell)
                        lst = cells.get(key)
                        if not lst:
                            continue
                        d = _min_image(out[lst] - p, float(n))
                        if np.any(np.einsum("ij,ij->i", d, d) < dmin * dmin):
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                out[k] = p
                cells.setdefault(c, []).append(k)
                k += 1
                if k == count:
                    break
    return out


def lattice_positions(n: int, spacing: int, offset: float) -> np.ndarray:
    """Simple-cubic lattice q = (spacing*i + offset) along each axis."""
    m = n // spacing
    g = np.arange(m) * spacing + offset
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)


def rsa_cap(n: int, dmin: float = 3.0, phi_excl: float = 0.25) -> int:
    """Largest blob count whose exclusion volume fraction stays below phi_excl.

    RSA of spheres of diameter dmin saturates near an excluded-volume
    fraction of about 0.38, so dense requests are capped.
    """
    v = 4.0 * math.pi * (dmin / 2.0) ** 3 / 3.0
    return int(math.floor(phi_excl * n ** 3 / v))


@dataclasses.dataclass
class Instance:
    """One suspension: a periodic n^3 grid, blobs, rates, source and solve kind."""
    name: str
    n: int
    q: np.ndarray              # (N, 3) float64, grid units
    kappa: np.ndarray          # (N,) float64
    f: np.ndarray              # (n, n, n) float64 source
    kind: str                  # "reactive" | "absorbing"
    alpha: float = 0.0
    rtol: float = 1e-8
    h: float = 1.0
    D: float = 1.0
    kernel_w: int = 4
    seed: int = 0

    @property
    def N(self) -> int:
        return int(self.q.shape[0])


def uniform_source(n: int) -> np.ndarray:
    return np.ones((n, n, n))


def random_source(rng: np.random.Generator, n: int) -> np.ndarray:
    """f = 1 + 0.5 * N(0, 1) per cell (a non-symmetric right-hand side)."""
    return 1.0 + 0.5 * rng.standard_normal((n, n, n))


def log_uniform(rng: np.random.Generator, lo: float, hi: float, size: int) -> np.ndarray:
    return 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=size)


def single_blob(n: int = 32, seed: Optional[int] = None) -> Instance:
    """32^3 grid, one blob at a uniform-random position, rate 1, f = 1 (reactive, FP64)."""
    s = seed_for(0) if seed is None else seed
    rng = np.random.default_rng(s)
    q = rng.uniform(0.0, n, size=(1, 3))
    return Instance("single_blob_32", n, q, np.ones(1), uniform_source(n), "reactive",
                    alpha=0.0, rtol=1e-10, seed=s)


def cubic_lattice(n: int = 128, spacing: int = 16, random_f: bool = False,
                  seed: Optional[int] = None) -> Instance:
    """Blobs on a simple-cubic lattice q = spacing*i + spacing/2 (cell vertices), absorbing."""
    s = seed_for(1) if seed is None else seed
    rng = np.random.default_rng(s)
    q = lattice_positions(n, spacing, spacing / 2.0)
    f = random_source(rng, n) if random_f else uniform_source(n)
    name = f"lattice{n}_s{spacing}" + ("_randf" if random_f else "")
    return Instance(name, n, q, np.zeros(q.shape[0]), f, "absorbing", rtol=1e-8, seed=s)


def disordered(n: int = 256, count: int = 20000, kind: str = "reactive",
               seed: Optional[int] = None, config: int = 2, instance: int = 0,
               dmin: float = 3.0) -> Instance:
    """RSA suspension with rates log-uniform in [1e-2, 1e2] and f = 1."""
    s = seed_for(config, instance) if seed is None else seed
    rng = np.random.default_rng(s)
    q = rsa_positions(rng, n, count, dmin)
    kappa = log_uniform(rng, 1e-2, 1e2, count)
    return Instance(f"rsa{n}_N{count}_{kind}", n, q, kappa, uniform_source(n), kind,
                    rtol=1e-8, seed=s)


BATCH_GRIDS = (32, 48, 64, 96, 128)


def batch_instances(count: int = 64, max_blobs: int = 2000, seed: Optional[int] = None
                    ) -> List[Instance]:
    """Uneven independent suspensions for batched solves.

    Grid edge drawn from {32, 48, 64, 96, 128}; blob count uniform in
    [1, max_blobs] and capped so RSA with d_min = 3 stays feasible; kind is
    reactive or absorbing with probability 1/2.
    """
    out = []
    for i in range(count):
        s = seed_for(3, i) if seed is None else seed + i
        rng = np.random.default_rng(s)
        n = int(rng.choice(BATCH_GRIDS))
        want = int(rng.integers(1, max_blobs + 1))
        N = min(want, rsa_cap(n))
        kind = "absorbing" if rng.random() < 0.5 else "reactive"
        q = rsa_positions(rng, n, N)
        kappa = log_uniform(rng, 1e-2, 1e2, N)
        out.append(Instance(f"batch{i}_n{n}_N{N}_{kind}", n, q, kappa, uniform_source(n), kind,
                            rtol=1e-8, seed=s))
    return out


def learned_eval(n: int = 256, count: int = 10000, index: int = 0) -> Instance:
    s = seed_for(4, index)
    rng = np.random.default_rng(s)
    q = rsa_positions(rng, n, count)
    return Instance(f"rsa{n}_N{count}_absorbing", n, q, np.zeros(count), uniform_source(n),
                    "absorbing", rtol=1e-8, seed=s)


def box_suspension(n: int = 256, count: int = 10000, margin: float = 3.0, index: int = 0) -> Instance:
    """RSA suspension in a box whose faces hold c = c_inf (the setting of Sec. IV.C): blobs at
    least `margin` cells inside every face and 3 cells apart, absorbing, f = 1. The points are
    drawn by periodic RSA in the inner cube [margin, n - margin)^3; its minimum-image test is
    stricter than the plain distance, so the separation holds in the box as well."""
    s = seed_for(5, index)
    rng = np.random.default_rng(s)
    q = margin + rsa_positions(rng, int(round(n - 2 * margin)), count)
    return Instance(f"box{n}_N{count}_absorbing", n, q, np.zeros(count), uniform_source(n), "absorbing",
                    rtol=1e-8, seed=s)


def training_config(index: int, n: int = 128, count: int = 1250) -> Instance:
    """Training suspensions for the learned preconditioner (same density as 256^3/10^4)."""
    s = 1306_500_000 + index
    rng = np.random.default_rng(s)
    q = rsa_positions(rng, n, count)
    return Instance(f"train{index}_n{n}_N{count}", n, q, np.zeros(count), uniform_source(n),
                    "absorbing", rtol=1e-8, seed=s)


def random_grid(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape)
