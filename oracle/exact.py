"""CPU FP64 oracle, part 1: the definitions and exact solves.

TEST INFRASTRUCTURE ONLY. Nothing in the product library may import, call or
link this module; only the tests, the smoke check and the benchmark's CPU
baseline use it. It shares no code with the HIP path.

Everything here is the plain definition of what the blob method computes
(arXiv:1306.3159, "Reaction-diffusion with minimally-resolved blobs"),
written out in float64 NumPy:

* the Peskin kernels phi_3 and phi_4 and the tensor-product weights
  (Sec. III.A, eq. tensor_product; moment conditions eq. JS_invariance);
* local averaging J and spreading S = dV_f^{-1} J^T (Sec. III.A);
* the (2d+1)-point periodic cell-centred Laplacian L (Sec. III.A);
* the reactive operator B = alpha I - D L + S kappa J (eqs. unsteady_system,
  steady_state) and the saddle-point system (eq. saddle_point with
  zeta = 1, xi = 1/dV_f);
* exact solves: the FFT diagonalises alpha I - D L on a periodic grid, and
  the blob coupling is eliminated with a dense N x N (bordered) system,
  the Schur-complement route of eqs. c_exact and r_schur with the periodic
  null-space handling of Appendix A.

Units: positions and grid in physical units with cell k centred at
(k + 1/2) h. Grid arrays have shape (nz, ny, nx), x fastest. Blob
positions are (N, 3) arrays ordered (x, y, z).
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Kernels (Sec. III.A). The paper states the moment conditions and the blob
# volumes (dV = 2^d h^d for phi_3, (8/3)^d h^d for phi_4) but not the
# formulas; these are the published forms it cites: phi_4 from Peskin's
# 2002 review, phi_3 from Roma, Peskin and Berger (1999).
# ---------------------------------------------------------------------------


def phi4(r):
    """Peskin's four-point kernel, support [-2, 2] in units of h."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    x = a[m1]
    out[m1] = (3.0 - 2.0 * x + np.sqrt(np.maximum(1.0 + 4.0 * x - 4.0 * x * x, 0.0))) / 8.0
    x = a[m2]
    out[m2] = (5.0 - 2.0 * x - np.sqrt(np.maximum(-7.0 + 12.0 * x - 4.0 * x * x, 0.0))) / 8.0
    return out


def phi3(r):
    """Three-point kernel of Roma, Peskin and Berger, support [-3/2, 3/2] in units of h."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 0.5
    m2 = (a > 0.5) & (a < 1.5)
    x = a[m1]
    out[m1] = (1.0 + np.sqrt(np.maximum(1.0 - 3.0 * x * x, 0.0))) / 3.0
    x = a[m2]
    out[m2] = (5.0 - 3.0 * x - np.sqrt(np.maximum(1.0 - 3.0 * (1.0 - x) ** 2, 0.0))) / 6.0
    return out


def kernel(w: int):
    if w == 4:
        return phi4
    if w == 3:
        return phi3
    raise ValueError("kernel width must be 3 or 4")


def blob_volume_factor(w: int) -> float:
    """Per-axis sum of phi^2 (Sec. III.A): 3/8 for phi_4, 1/2 for phi_3."""
    return {4: 3.0 / 8.0, 3: 0.5}[w]


# ---------------------------------------------------------------------------
# Weights, J and S (Sec. III.A).
# ---------------------------------------------------------------------------


def axis_weights(qa: float, n: int, h: float, w: int) -> np.ndarray:
    """1-D weights phi_w((q - r_k)/h) for all n cells of one periodic axis.

    r_k = (k + 1/2) h; the separation is taken as the nearest periodic image.
    """
    k = np.arange(n)
    d = (qa - (k + 0.5) * h) / h
    d = d - n * np.round(d / n)
    return kernel(w)(d)


def blob_stencil(q: np.ndarray, shape: Tuple[int, int, int], h: float, w: int):
    """Nonzero support of one blob: index arrays (iz, iy, ix) and the 3-D weights.

    The 3-D weight is the tensor product of the three axis weights
    (eq. tensor_product).
    """
    nz, ny, nx = shape
    wx = axis_weights(q[0], nx, h, w)
    wy = axis_weights(q[1], ny, h, w)
    wz = axis_weights(q[2], nz, h, w)
    ix = np.nonzero(wx)[0]
    iy = np.nonzero(wy)[0]
    iz = np.nonzero(wz)[0]
    W = wz[iz][:, None, None] * wy[iy][None, :, None] * wx[ix][None, None, :]
    return iz, iy, ix, W


def interp(c: np.ndarray, q: np.ndarray, h: float = 1.0, w: int = 4) -> np.ndarray:
    """Local averaging J: (J c)_i = sum_k phi_w(q_i - r_k) c_k."""
    out = np.zeros(q.shape[0])
    for i in range(q.shape[0]):
        iz, iy, ix, W = blob_stencil(q[i], c.shape, h, w)
        out[i] = np.sum(W * c[np.ix_(iz, iy, ix)])
    return out


def spread(lam: np.ndarray, q: np.ndarray, shape, h: float = 1.0, w: int = 4) -> np.ndarray:
    """Spreading S = dV_f^{-1} J^T with dV_f = h^3: (S lam)_k = h^-3 sum_i phi_w(q_i - r_k) lam_i."""
    out = np.zeros(shape)
    for i in range(q.shape[0]):
        iz, iy, ix, W = blob_stencil(q[i], shape, h, w)
        out[np.ix_(iz, iy, ix)] += W * lam[i] / h ** 3
    return out


def dense_J(q: np.ndarray, shape, h: float = 1.0, w: int = 4) -> np.ndarray:
    """J as a dense N x n_cells matrix, built entry by entry from the kernel."""
    nz, ny, nx = shape
    J = np.zeros((q.shape[0], nz * ny * nx))
    for i in range(q.shape[0]):
        wx = axis_weights(q[i, 0], nx, h, w)
        wy = axis_weights(q[i, 1], ny, h, w)
        wz = axis_weights(q[i, 2], nz, h, w)
        for kz in range(nz):
            for ky in range(ny):
                for kx in range(nx):
                    J[i, (kz * ny + ky) * nx + kx] = wz[kz] * wy[ky] * wx[kx]
    return J


# ---------------------------------------------------------------------------
# Laplacian and operators (Sec. III.A, III.B).
# ---------------------------------------------------------------------------


def laplacian(c: np.ndarray, h: float = 1.0) -> np.ndarray:
    """Standard 7-point cell-centred Laplacian with periodic wrap."""
    out = -6.0 * c
    for ax in range(3):
        out = out + np.roll(c, 1, axis=ax) + np.roll(c, -1, axis=ax)
    return out / (h * h)


def dense_laplacian(shape, h: float = 1.0) -> np.ndarray:
    """The 7-point periodic Laplacian as a dense matrix, built cell by cell."""
    nz, ny, nx = shape
    M = nz * ny * nx
    L = np.zeros((M, M))
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                row = (kz * ny + ky) * nx + kx
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    col = (((kz + dz) % nz) * ny + (ky + dy) % ny) * nx + (kx + dx) % nx
                    L[row, col] += 1.0 / h ** 2
                    L[row, row] -= 1.0 / h ** 2
    return L


def apply_A(c: np.ndarray, alpha: float, D: float = 1.0, h: float = 1.0) -> np.ndarray:
    """A c = alpha c - D L c (eq. Helmholtz with alpha = 1/dt)."""
    return alpha * c - D * laplacian(c, h)


def apply_B(c, q, kappa, alpha, D=1.0, h=1.0, w=4):
    """B c = (alpha I - D L + S kappa J) c (eqs. unsteady_system, steady_state)."""
    return apply_A(c, alpha, D, h) + spread(kappa * interp(c, q, h, w), q, c.shape, h, w)


# ---------------------------------------------------------------------------
# Exact periodic Helmholtz / Poisson solve by FFT.
# ---------------------------------------------------------------------------


def helmholtz_symbol(shape, alpha: float, D: float, h: float) -> np.ndarray:
    """Eigenvalues of alpha I - D L on the periodic grid: alpha + (4D/h^2) sum sin^2(pi m / n)."""
    nz, ny, nx = shape
    sz = np.sin(np.pi * np.arange(nz) / nz) ** 2
    sy = np.sin(np.pi * np.arange(ny) / ny) ** 2
    sx = np.sin(np.pi * np.arange(nx) / nx) ** 2
    return alpha + (4.0 * D / h ** 2) * (sz[:, None, None] + sy[None, :, None] + sx[None, None, :])


def solve_A(g: np.ndarray, alpha: float, D: float = 1.0, h: float = 1.0) -> np.ndarray:
    """u = (alpha I - D L)^{-1} g; for alpha = 0 the pseudo-inverse (mean-zero result)."""
    lam = helmholtz_symbol(g.shape, alpha, D, h)
    gh = np.fft.fftn(g)
    if alpha == 0.0:
        lam = lam.copy()
        lam[0, 0, 0] = 1.0
        gh[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(gh / lam))


def schur_matrix(q, shape, alpha, D=1.0, h=1.0, w=4) -> np.ndarray:
    """G = J A^+ S (eq. r_schur's M with zeta = xi = 1), one FFT solve per column."""
    N = q.shape[0]
    G = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        G[:, j] = interp(solve_A(spread(e, q, shape, h, w), alpha, D, h), q, h, w)
    return G


# ---------------------------------------------------------------------------
# Exact reactive solve: (alpha I - D L + S kappa J) c = f.
# With mu = kappa J c the blob sink strengths, c = A^+ (f - S mu) + cbar e.
# ---------------------------------------------------------------------------


def solve_reactive(f, q, kappa, alpha, D=1.0, h=1.0, w=4, G=None):
    """Exact reactive solution via the N x N (bordered) blob system.

    alpha > 0: (I + K G) mu = K J A^{-1} f, c = A^{-1}(f - S mu).
    alpha = 0 (periodic, Appendix A): the sink total is fixed by the source,
    sum(mu) = h^3 sum(f); c = (-D L)^+ (f - S mu) + cbar with
    [I + K G, -K 1; 1^T, 0] [mu; cbar] = [K J (-DL)^+ f; h^3 sum f].
    Returns (c, mu).
    """
    N = q.shape[0]
    shape = f.shape
    if G is None:
        G = schur_matrix(q, shape, alpha, D, h, w)
    K = np.diag(kappa)
    rhs = kappa * interp(solve_A(f, alpha, D, h), q, h, w)
    if alpha > 0.0:
        mu = np.linalg.solve(np.eye(N) + K @ G, rhs)
        c = solve_A(f - spread(mu, q, shape, h, w), alpha, D, h)
        return c, mu
    if np.sum(kappa) <= 0.0:
        raise ValueError("steady reactive problem with zero total rate is singular")
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = np.eye(N) + K @ G
    M[:N, N] = -kappa
    M[N, :N] = 1.0
    b = np.concatenate([rhs, [h ** 3 * np.sum(f)]])
    sol = np.linalg.solve(M, b)
    mu, cbar = sol[:N], sol[N]
    c = solve_A(f - spread(mu, q, shape, h, w), 0.0, D, h) + cbar
    return c, mu


# ---------------------------------------------------------------------------
# Exact absorbing (diffusion-limited) solve: [A, S; J, 0][c; lam] = [f; phi].
# ---------------------------------------------------------------------------


def solve_absorbing(f, q, alpha, D=1.0, h=1.0, w=4, phi=None, G=None):
    """Exact saddle-point solution (eqs. saddle_point, c_exact, r_schur; Appendix A).

    alpha > 0: G lam = J A^{-1} f - phi, c = A^{-1}(f - S lam).
    alpha = 0 (periodic): sum(lam) = h^3 sum(f) (solvability, Appendix A) and
    c = (-DL)^+(f - S lam) + cbar with
    [G, -1; 1^T, 0][lam; cbar] = [J (-DL)^+ f - phi; h^3 sum f].
    Returns (c, lam).
    """
    N = q.shape[0]
    shape = f.shape
    if N == 0:
        raise ValueError("absorbing problem needs at least one blob")
    if phi is None:
        phi = np.zeros(N)
    if G is None:
        G = schur_matrix(q, shape, alpha, D, h, w)
    rhs = interp(solve_A(f, alpha, D, h), q, h, w) - phi
    if alpha > 0.0:
        lam = np.linalg.solve(G, rhs)
        return solve_A(f - spread(lam, q, shape, h, w), alpha, D, h), lam
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = G
    M[:N, N] = -1.0
    M[N, :N] = 1.0
    sol = np.linalg.lstsq(M, np.concatenate([rhs, [h ** 3 * np.sum(f)]]), rcond=None)[0]
    lam, cbar = sol[:N], sol[N]
    c = solve_A(f - spread(lam, q, shape, h, w), 0.0, D, h) + cbar
    return c, lam


def step(c_old, f, q, kappa, dt, D=1.0, h=1.0, w=4, G=None):
    """One backward-Euler step (eq. c_np1): B c^{n+1} = c^n/dt + f with alpha = 1/dt."""
    return solve_reactive(f + c_old / dt, q, kappa, 1.0 / dt, D, h, w, G)[0]


def step_absorbing(c_old, f, q, dt, D=1.0, h=1.0, w=4, G=None):
    """One backward-Euler step of a diffusion-limited suspension (eq. c_np1 without the
    reaction term; the sinks are the multipliers of eq. saddle_point with A = I/dt - D L,
    the finite-dt case of Sec. III.C, so A is invertible):
    [A, S; J, 0][c^{n+1}; lam] = [c^n/dt + f; 0]. Returns (c^{n+1}, lam)."""
    return solve_absorbing(f + c_old / dt, q, 1.0 / dt, D, h, w, G=G)


# ---------------------------------------------------------------------------
# Residuals (the paper does not define one; unweighted 2-norms).
# ---------------------------------------------------------------------------


def reactive_residual(c, f, q, kappa, alpha, D=1.0, h=1.0, w=4) -> float:
    r = f - apply_B(c, q, kappa, alpha, D, h, w)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def absorbing_residual(c, lam, f, q, alpha, D=1.0, h=1.0, w=4, phi=None) -> float:
    """|| [f - A c - S lam; phi - J c] || / || [f; phi] ||."""
    if phi is None:
        phi = np.zeros(q.shape[0])
    r1 = f - apply_A(c, alpha, D, h) - spread(lam, q, c.shape, h, w)
    r2 = phi - interp(c, q, h, w)
    num = math.sqrt(float(np.sum(r1 * r1) + np.sum(r2 * r2)))
    den = math.sqrt(float(np.sum(f * f) + np.sum(phi * phi)))
    return num / den


# ---------------------------------------------------------------------------
# Reaction radius (Sec. IV.A).
# ---------------------------------------------------------------------------


def radius_from_mean(cbar: float, s: float, V: float, D: float = 1.0) -> float:
    """a_L = s V / (4 pi D cbar) (eq. beta0_low_phi): the one sink absorbs the whole source
    s V at the Smoluchowski rate 4 pi D a_L cbar, so a_L does not depend on the source."""
    return s * V / (4.0 * math.pi * D * cbar)


def radius_extrapolated(aL: float, L: float) -> float:
    """Invert a_L = a (1 + x + x^2), x = 2.84 a / L (eq. a_phi) for a."""
    lo, hi = 0.0, aL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x = 2.84 * mid / L
        if mid * (1.0 + x + x * x) < aL:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def gamma_single_blob(q, shape, D=1.0, h=1.0, w=4) -> float:
    """gamma = J (-D L)^+ S 1 for one blob (the diagonal of eq. Schur_diagonal, sign flipped)."""
    return float(interp(solve_A(spread(np.ones(1), q[None, :], shape, h, w), 0.0, D, h),
                        q[None, :], h, w)[0])
