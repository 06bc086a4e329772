"""Pins for the oracle of the blob model in a box with a fixed face value (Sec. IV.C).

The sine-transform solves are checked against dense matrices built cell by cell, the
lifting c = c_b + u against the inhomogeneous system assembled directly, and the single
absorbing blob against the paper's far-field law (eq. c_r_approx).
"""
import numpy as np
import pytest

from oracle import dirichlet as dr
from oracle import exact as ex


def _setup(seed, shape=(6, 8, 10)):
    rng = np.random.default_rng(seed)
    return rng, shape, rng.standard_normal(shape)


def test_laplacian0_matches_dense_and_spectrum():
    """L_0 (ghost -u) applied by shifts equals the cell-by-cell matrix; the matrix's spectrum
    is the sine-transform symbol (an independent check of the eigenvalues used by solve_A0)."""
    rng, shape, u = _setup(81)
    L = dr.dense_laplacian0(shape, 0.7)
    assert np.max(np.abs(L @ u.ravel() - dr.laplacian0(u, 0.7).ravel())) < 1e-12
    assert np.allclose(L, L.T)
    ev = np.sort(np.linalg.eigvalsh(-L))
    sym = np.sort(dr.symbol0(shape, 0.0, 1.0, 0.7).ravel())
    assert np.max(np.abs(ev - sym)) < 1e-11 * sym.max()


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_solve_A0_matches_dense(alpha):
    """alpha I - D L_0 is invertible even for alpha = 0 (no null space with fixed faces)."""
    rng, shape, g = _setup(82)
    D, h = 1.3, 0.9
    A = alpha * np.eye(g.size) - D * dr.dense_laplacian0(shape, h)
    ref = np.linalg.solve(A, g.ravel())
    assert np.max(np.abs(dr.solve_A0(g, alpha, D, h).ravel() - ref)) < 1e-11 * np.max(np.abs(ref))


def test_face_value_lifting():
    """The ghost 2 c_b - c makes L_{c_b}(c_b + u) = L_0 u, so a constant c_b is harmonic."""
    rng, shape, u = _setup(83)
    assert np.max(np.abs(dr.laplacian_box(2.5 + u, 2.5) - dr.laplacian0(u))) < 1e-12
    assert np.max(np.abs(dr.laplacian_box(np.full(shape, 2.5), 2.5))) < 1e-12


def _dense_box(alpha, c_b, kappa=None):
    """The inhomogeneous system assembled directly: the face value enters the right side as
    2 D c_b / h^2 per face a boundary cell touches."""
    rng = np.random.default_rng(84)
    n = 10
    shape = (n, n, n)
    q = np.array([[4.3, 5.1, 4.8], [6.2, 3.9, 5.7]])
    f = 1.0 + 0.5 * rng.standard_normal(shape)
    Jd = ex.dense_J(q, shape)
    A = alpha * np.eye(n ** 3) - dr.dense_laplacian0(shape)
    rhs = f.ravel() + 2.0 * c_b * dr.boundary_faces(shape).ravel()
    return q, f, Jd, A, rhs


@pytest.mark.parametrize("alpha", [0.0, 0.4])
def test_reactive_box_matches_dense(alpha):
    kappa = np.array([0.7, 25.0])
    q, f, Jd, A, rhs = _dense_box(alpha, 1.7)
    ref = np.linalg.solve(A + Jd.T @ np.diag(kappa) @ Jd, rhs)
    c, mu = dr.solve_reactive_box(f, q, kappa, alpha, 1.7)
    assert np.max(np.abs(c.ravel() - ref)) < 1e-10 * np.max(np.abs(ref))
    assert dr.reactive_residual_box(c, f, q, kappa, alpha, 1.7) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 0.4])
def test_absorbing_box_matches_dense(alpha):
    q, f, Jd, A, rhs = _dense_box(alpha, 1.7)
    N = q.shape[0]
    M = np.block([[A, Jd.T], [Jd, np.zeros((N, N))]])
    ref = np.linalg.solve(M, np.concatenate([rhs, np.zeros(N)]))
    c, lam = dr.solve_absorbing_box(f, q, alpha, 1.7)
    assert np.max(np.abs(c.ravel() - ref[:-N])) < 1e-10 * np.max(np.abs(ref[:-N]))
    assert np.max(np.abs(lam - ref[-N:])) < 1e-10 * np.max(np.abs(ref[-N:]))
    assert dr.absorbing_residual_box(c, lam, f, q, alpha, 1.7) < 1e-12


def test_single_blob_far_field():
    """Sec. IV.C, eq. c_r_approx: an absorbing blob at the centre of a box held at c_inf,
    no source: c(r)/c_inf ~ L/(L - 2a) (1 - a/r) with a = 1.255 h (loose: 1 %)."""
    n = 64
    q = np.array([[32.0, 32.0, 32.0]])
    c, lam = dr.solve_absorbing_box(np.zeros((n, n, n)), q, 0.0, 1.0)
    a = 1.255
    for k in (38, 42, 48, 56):
        r = k + 0.5 - 32.0
        assert c[31, 31, k] == pytest.approx(n / (n - 2 * a) * (1 - a / r), rel=0.01)
    assert lam[0] > 0.0
