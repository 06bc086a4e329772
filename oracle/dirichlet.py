"""CPU FP64 oracle, part 5: the blob model in a box with the concentration held on its faces.

TEST INFRASTRUCTURE ONLY. Nothing in the product library may import, call or
link this module; only the tests use it. It shares no code with the HIP path.

The paper's single-blob tests place a blob in a cubic box with c = c_inf on the
boundary (Sec. IV.C, eq. c_r_approx, Fig. FarFieldDecay). On the cell-centred
grid the face value is the mean of a boundary cell and its mirror ghost, so the
7-point Laplacian at a boundary cell takes the ghost value 2 c_b - c.

Writing c = c_b + u removes the boundary value: L_{c_b}(c_b + u) = L_0 u, where
L_0 uses the ghost -u (homogeneous faces), and a blob whose kernel support lies
inside the box has J 1 = 1. So

  reactive   (alpha I - D L_0 + S kappa J) u = f - alpha c_b - c_b S kappa,
  absorbing  [alpha I - D L_0, S; J, 0][u; lam] = [f - alpha c_b; -c_b],

with alpha I - D L_0 invertible for every alpha >= 0 (no null space), and
diagonalised by the type-II discrete sine transform: the modes
sin(pi m (k + 1/2) / n), m = 1..n, have L_0-eigenvalues -(4/h^2) sin^2(pi m / (2n)).

Grid arrays have shape (nz, ny, nx), x fastest; blob positions (N, 3) are (x, y, z)
and must keep their kernel support inside the box (the spreading and averaging of
exact.py then see no wrap).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from . import exact as ex


def laplacian0(u: np.ndarray, h: float = 1.0) -> np.ndarray:
    """7-point Laplacian with homogeneous faces: the ghost beyond a face is -u of the cell."""
    out = -6.0 * u
    for ax in range(3):
        lo = np.concatenate([-np.take(u, [0], axis=ax), np.take(u, range(u.shape[ax] - 1), axis=ax)], axis=ax)
        hi = np.concatenate([np.take(u, range(1, u.shape[ax]), axis=ax), -np.take(u, [u.shape[ax] - 1], axis=ax)],
                            axis=ax)
        out = out + lo + hi
    return out / (h * h)


def laplacian_box(c: np.ndarray, c_b: float, h: float = 1.0) -> np.ndarray:
    """7-point Laplacian with the face value c_b: ghost 2 c_b - c."""
    out = -6.0 * c
    for ax in range(3):
        n = c.shape[ax]
        lo = np.concatenate([2 * c_b - np.take(c, [0], axis=ax), np.take(c, range(n - 1), axis=ax)], axis=ax)
        hi = np.concatenate([np.take(c, range(1, n), axis=ax), 2 * c_b - np.take(c, [n - 1], axis=ax)], axis=ax)
        out = out + lo + hi
    return out / (h * h)


def dense_laplacian0(shape, h: float = 1.0) -> np.ndarray:
    """L_0 as a dense matrix, built cell by cell (a missing neighbour adds -1 to the diagonal)."""
    nz, ny, nx = shape
    M = nz * ny * nx
    L = np.zeros((M, M))
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                row = (kz * ny + ky) * nx + kx
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    z, y, x = kz + dz, ky + dy, kx + dx
                    L[row, row] -= 1.0 / h ** 2
                    if 0 <= z < nz and 0 <= y < ny and 0 <= x < nx:
                        L[row, (z * ny + y) * nx + x] += 1.0 / h ** 2
                    else:
                        L[row, row] -= 1.0 / h ** 2
    return L


def boundary_faces(shape) -> np.ndarray:
    """Number of box faces each cell touches (0 inside, 1 on a face, 2 on an edge, 3 at a corner)."""
    out = np.zeros(shape)
    for ax in range(3):
        idx = np.arange(shape[ax])
        edge = ((idx == 0).astype(float) + (idx == shape[ax] - 1).astype(float))
        sh = [1, 1, 1]
        sh[ax] = shape[ax]
        out = out + edge.reshape(sh)
    return out


def symbol0(shape, alpha: float, D: float, h: float) -> np.ndarray:
    """Eigenvalues of alpha I - D L_0 on the DST-II modes m = 1..n per axis."""
    parts = []
    for n in shape:
        parts.append(np.sin(np.pi * np.arange(1, n + 1) / (2 * n)) ** 2)
    sz, sy, sx = parts
    return alpha + (4.0 * D / h ** 2) * (sz[:, None, None] + sy[None, :, None] + sx[None, None, :])


def solve_A0(g: np.ndarray, alpha: float, D: float = 1.0, h: float = 1.0) -> np.ndarray:
    """u = (alpha I - D L_0)^{-1} g by the type-II sine transform."""
    return sfft.idstn(sfft.dstn(g, type=2) / symbol0(g.shape, alpha, D, h), type=2)


def apply_A0(u, alpha, D=1.0, h=1.0):
    return alpha * u - D * laplacian0(u, h)


def schur_matrix0(q, shape, alpha, D=1.0, h=1.0, w=4) -> np.ndarray:
    """G = J (alpha I - D L_0)^{-1} S, one sine-transform solve per column."""
    N = q.shape[0]
    G = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        G[:, j] = ex.interp(solve_A0(ex.spread(e, q, shape, h, w), alpha, D, h), q, h, w)
    return G


def solve_reactive_box(f, q, kappa, alpha, c_b, D=1.0, h=1.0, w=4):
    """(alpha I - D L_{c_b} + S kappa J) c = f by the lifting c = c_b + u and the N x N blob
    system (I + K G) mu = K J A0^{-1} g' (mu = kappa J u). Returns (c, mu)."""
    shape = f.shape
    N = q.shape[0]
    g = f - alpha * c_b - c_b * ex.spread(kappa, q, shape, h, w)
    G = schur_matrix0(q, shape, alpha, D, h, w)
    K = np.diag(kappa)
    mu = np.linalg.solve(np.eye(N) + K @ G, kappa * ex.interp(solve_A0(g, alpha, D, h), q, h, w))
    return c_b + solve_A0(g - ex.spread(mu, q, shape, h, w), alpha, D, h), mu


def solve_absorbing_box(f, q, alpha, c_b, D=1.0, h=1.0, w=4):
    """[alpha I - D L_{c_b}, S; J, 0][c; lam] = [f; 0] by the lifting c = c_b + u:
    G lam = J A0^{-1} g' + c_b, u = A0^{-1}(g' - S lam). Returns (c, lam)."""
    shape = f.shape
    g = f - alpha * c_b
    G = schur_matrix0(q, shape, alpha, D, h, w)
    lam = np.linalg.solve(G, ex.interp(solve_A0(g, alpha, D, h), q, h, w) + c_b)
    return c_b + solve_A0(g - ex.spread(lam, q, shape, h, w), alpha, D, h), lam


# Residuals relative to the right-hand side of the lifted system (the boundary value
# moved to the right; with f = 0 the boundary value alone drives the problem).


def reactive_residual_box(c, f, q, kappa, alpha, c_b, D=1.0, h=1.0, w=4) -> float:
    """|| f - B c || / || f - alpha c_b - c_b S kappa ||, B with the face value c_b."""
    r = f - (alpha * c - D * laplacian_box(c, c_b, h) + ex.spread(kappa * ex.interp(c, q, h, w), q, c.shape, h, w))
    den = f - alpha * c_b - c_b * ex.spread(kappa, q, c.shape, h, w)
    return float(np.linalg.norm(r) / np.linalg.norm(den))


def absorbing_residual_box(c, lam, f, q, alpha, c_b, D=1.0, h=1.0, w=4) -> float:
    """|| [f - A c - S lam; -J c] || / || [f - alpha c_b; -c_b] || with A = alpha I - D L_{c_b}."""
    r1 = f - (alpha * c - D * laplacian_box(c, c_b, h)) - ex.spread(lam, q, c.shape, h, w)
    r2 = -ex.interp(c, q, h, w)
    N = q.shape[0]
    den = math.sqrt(float(np.sum((f - alpha * c_b) ** 2)) + N * c_b * c_b)
    return math.sqrt(float(np.sum(r1 * r1) + np.sum(r2 * r2))) / den
