"""CPU FP64 oracle, part 6: a Fourier coarse level for the Schur preconditioner.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline); shares no
code with the HIP path.

The paper preconditions the Schur complement M = J A^+ S of the absorbing
saddle-point system (eq. r_schur) with a diagonal approximation of M^{-1}
(eq. Schur_diagonal, Sec. III.E); the learned preconditioner W adds
short-ranged pair terms to that diagonal. Both are local: the slowly varying
modes of M, whose eigenvalues grow like (N/V) / (D |k|^2) for long waves,
are left to the Krylov method. This part adds a coarse level spanned by the
lowest Fourier modes of the blob set,

    Z = [cos(k.q_i) - mean, sin(k.q_i) - mean]  for k = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z),

over the integer wave vectors 0 < |m|^2 <= m2max (one of each +-m pair), and
combines it with W by the balancing two-level form (Mandel 1993; the "BNN"
form of Tang, Nabben, Vuik and Erlangga 2009):

    B = Q + (I - Q M) W (I - M Q),   Q = Z E^{-1} Z^T,   E = Z^T M Z.

B solves the coarse modes exactly (B M Z = Z), leaves the residual
M B r - r orthogonal to the coarse space, and keeps an exact W exact. The
paper has no coarse level; this is an extension of its Schur preconditioner.
At alpha = 0 (periodic, Appendix A) M and W act on mean-zero vectors
(M -> P M P, W -> P W P); the mean-free columns of Z keep B mean-free.
"""
from __future__ import annotations

from typing import Callable, Sequence, Union

import numpy as np


def wave_vectors(m2max: int) -> np.ndarray:
    """Integer wave vectors m = (m_x, m_y, m_z) with 0 < |m|^2 <= m2max, one of each pair
    +-m (the one whose first nonzero component is positive); (count, 3) int array."""
    r = int(np.floor(np.sqrt(max(m2max, 0))))
    out = []
    for mx in range(-r, r + 1):
        for my in range(-r, r + 1):
            for mz in range(-r, r + 1):
                m2 = mx * mx + my * my + mz * mz
                if m2 == 0 or m2 > m2max:
                    continue
                first = mx if mx != 0 else (my if my != 0 else mz)
                if first > 0:
                    out.append((mx, my, mz))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def basis(q: np.ndarray, shape: Sequence[int], h: float = 1.0, m2max: int = 3) -> np.ndarray:
    """The coarse basis Z (N, K): for each wave vector the columns cos(k.q) and sin(k.q),
    each with its mean over the blobs removed. shape is (nz, ny, nx); q is (N, 3) (x, y, z)."""
    nz, ny, nx = shape
    L = np.array([nx * h, ny * h, nz * h], dtype=np.float64)
    m = wave_vectors(m2max).astype(np.float64)
    k = 2.0 * np.pi * m / L[None, :]                 # (K/2, 3)
    ph = np.asarray(q, dtype=np.float64) @ k.T       # (N, K/2)
    Z = np.empty((q.shape[0], 2 * m.shape[0]))
    Z[:, 0::2] = np.cos(ph)
    Z[:, 1::2] = np.sin(ph)
    return Z - Z.mean(axis=0, keepdims=True)


def two_level(M: np.ndarray, Z: np.ndarray, W: Union[np.ndarray, Callable[[np.ndarray], np.ndarray]]
              ) -> np.ndarray:
    """The dense balancing preconditioner B = Q + (I - Q M) W (I - M Q) with Q = Z E^{-1} Z^T
    and E = Z^T M Z (symmetrised); W a matrix or a function applied to the columns of a matrix.
    M is the Schur operator the solve uses (P M P at alpha = 0)."""
    N = M.shape[0]
    E = Z.T @ M @ Z
    E = 0.5 * (E + E.T)
    Q = Z @ np.linalg.solve(E, Z.T)
    I = np.eye(N)
    right = I - M @ Q
    Wr = W @ right if isinstance(W, np.ndarray) else W(right)
    return Q + (I - Q @ M) @ Wr


def two_level_operator(apply_M: Callable[[np.ndarray], np.ndarray], Z: np.ndarray,
                       apply_W: Callable[[np.ndarray], np.ndarray]) -> Callable[[np.ndarray], np.ndarray]:
    """The same balancing form without forming M: M enters through its products with the
    K columns of Z (taken once) and with one more vector per application. Returns r -> B r,
    evaluated in the order of the definition: a = E^{-1} Z^T r, w = W (r - M Z a),
    z = w + Z (a - E^{-1} Z^T M w) (M symmetric, so Z^T M w = (M Z)^T w is not used)."""
    MZ = np.column_stack([apply_M(Z[:, k]) for k in range(Z.shape[1])])
    E = Z.T @ MZ
    E = 0.5 * (E + E.T)

    def apply(r: np.ndarray) -> np.ndarray:
        a = np.linalg.solve(E, Z.T @ r)
        w = apply_W(r - MZ @ a)
        return w + Z @ (a - np.linalg.solve(E, Z.T @ apply_M(w)))
    return apply


def projector(N: int) -> np.ndarray:
    """P = I - 1 1^T / N (Appendix A's null-space projection)."""
    return np.eye(N) - np.full((N, N), 1.0 / N)
