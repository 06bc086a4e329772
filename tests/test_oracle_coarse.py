"""Pins for the Fourier coarse level of the Schur preconditioner (oracle/coarse.py).

The balancing form is pinned by what it must do for any W (solve the coarse modes exactly,
leave residuals orthogonal to the coarse space, keep an exact W exact, reduce to the exact
inverse when the coarse space is everything) and the basis by Fourier analysis on a blob
lattice, where the modes are orthogonal and are eigenvectors of the exact Schur matrix."""
import numpy as np
import pytest

from oracle import coarse as CO
from oracle import exact as ex
import workloads as W


def test_wave_vector_counts_are_half_the_sums_of_three_squares():
    # r3(n), the number of integer points with |m|^2 = n: 6, 12, 8, 6, 24, 24 for n = 1..6
    r3 = [6, 12, 8, 6, 24, 24]
    for m2max in range(1, 7):
        m = CO.wave_vectors(m2max)
        assert m.shape[0] == sum(r3[:m2max]) // 2
        s = {tuple(v) for v in m}
        assert len(s) == m.shape[0]
        assert not any(tuple(-v) in s for v in m)
        assert np.all((m * m).sum(1) <= m2max) and np.all((m * m).sum(1) > 0)
    assert CO.wave_vectors(0).shape == (0, 3)


def _lattice(n, p, offset):
    a = n / p
    g = (np.arange(p) * a)[:, None] + np.asarray(offset)[None, :]
    x, y, z = np.meshgrid(g[:, 0], g[:, 1], g[:, 2], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1)


@pytest.mark.parametrize("alpha", [0.0, 0.37])
def test_lattice_modes_are_orthogonal_eigenvectors_of_the_schur_matrix(alpha):
    """Blobs on a 4^3 lattice of a 16^3 grid, all at the same offset within their cell: the
    Schur matrix commutes with the lattice shifts, so each cos/sin column is an eigenvector,
    and the columns are orthogonal with Z^T Z = (N/2) I below the lattice's Nyquist limit."""
    n, p = 16, 4
    q = _lattice(n, p, (0.3, 1.7, 2.45))
    N = q.shape[0]
    Z = CO.basis(q, (n, n, n), 1.0, 3)
    assert Z.shape == (N, 26)
    assert np.allclose(Z.T @ Z, 0.5 * N * np.eye(26), atol=1e-10)
    G = ex.schur_matrix(q, (n, n, n), alpha)
    MZ = G @ Z
    mu = np.einsum("ik,ik->k", Z, MZ) / (0.5 * N)
    assert np.allclose(MZ, Z * mu[None, :], atol=1e-10 * np.abs(mu).max())
    assert np.allclose(mu[0::2], mu[1::2], rtol=1e-10)       # cos and sin share an eigenvalue
    # long waves feel the mean-field Green's function: mu falls as |m|^2 grows
    m2 = (CO.wave_vectors(3) ** 2).sum(1)
    assert mu[0::2][m2 == 1].min() > mu[0::2][m2 == 2].max() > mu[0::2][m2 == 2].min() > mu[0::2][m2 == 3].max()


def _config(alpha, N=30, n=16, seed=5):
    rng = np.random.default_rng(seed)
    q = W.rsa_positions(rng, n, N, 3.0)
    G = ex.schur_matrix(q, (n, n, n), alpha)
    if alpha == 0.0:
        P = CO.projector(N)
        return q, P @ G @ P, P
    return q, G, np.eye(N)


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_balancing_solves_the_coarse_modes_for_any_w(alpha):
    n = 16
    q, M, P = _config(alpha)
    N = q.shape[0]
    Z = CO.basis(q, (n, n, n), 1.0, 2)
    rng = np.random.default_rng(7)
    Wm = P @ rng.standard_normal((N, N)) @ P                  # any W, not even symmetric
    B = CO.two_level(M, Z, Wm)
    assert np.allclose(B @ M @ Z, Z, atol=1e-9)
    R = Z.T @ (M @ B - np.eye(N))                             # residuals orthogonal to the coarse space
    assert np.abs(R).max() < 1e-9 * np.abs(Z).max() * N
    # the callable form of W gives the same matrix
    assert np.allclose(CO.two_level(M, Z, lambda X: Wm @ X), B, atol=1e-12)
    if alpha == 0.0:
        one = np.ones(N)
        assert np.abs(B @ one).max() < 1e-10 and np.abs(one @ B).max() < 1e-10


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_balancing_keeps_an_exact_w_exact(alpha):
    n = 16
    q, M, P = _config(alpha)
    Minv = np.linalg.pinv(M, rcond=1e-12)
    Z = CO.basis(q, (n, n, n), 1.0, 3)
    assert np.allclose(CO.two_level(M, Z, Minv), Minv, atol=1e-9 * np.abs(Minv).max())


def test_full_coarse_space_is_the_exact_inverse():
    """Seven blobs and the six modes with |m|^2 = 1: the mean-free columns span all of
    range(P), so B = (P M P)^+ whatever W is."""
    n = 16
    q, M, P = _config(0.0, N=7, seed=11)
    Z = CO.basis(q, (n, n, n), 1.0, 1)
    assert Z.shape == (7, 6) and np.linalg.matrix_rank(Z) == 6
    rng = np.random.default_rng(3)
    for Wm in (np.zeros((7, 7)), P @ rng.standard_normal((7, 7)) @ P):
        assert np.allclose(CO.two_level(M, Z, Wm), np.linalg.pinv(M, rcond=1e-12), atol=1e-9)


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_matrix_free_form_is_the_dense_form(alpha):
    """two_level_operator (M only through products) against two_level on the dense matrix;
    a W that is not symmetric, so swapped roles of the two projections would show."""
    n = 16
    q, M, P = _config(alpha)
    N = q.shape[0]
    Z = CO.basis(q, (n, n, n), 1.0, 3)
    rng = np.random.default_rng(13)
    Wm = P @ rng.standard_normal((N, N)) @ P
    B = CO.two_level(M, Z, Wm)
    op = CO.two_level_operator(lambda v: M @ v, Z, lambda v: Wm @ v)
    for _ in range(3):
        r = rng.standard_normal(N)
        assert np.allclose(op(r), B @ r, atol=1e-10 * np.abs(B).max() * np.abs(r).max())


def test_plausible_mistakes_break_a_pin():
    """Swapping the two projections, or keeping the column means, fails the pins above."""
    n = 16
    q, M, P = _config(0.0)
    N = q.shape[0]
    Z = CO.basis(q, (n, n, n), 1.0, 2)
    rng = np.random.default_rng(9)
    Wm = P @ rng.standard_normal((N, N)) @ P
    E = Z.T @ M @ Z
    Q = Z @ np.linalg.solve(0.5 * (E + E.T), Z.T)
    I = np.eye(N)
    swapped = Q + (I - M @ Q) @ Wm @ (I - Q @ M)
    assert not np.allclose(swapped @ M @ Z, Z, atol=1e-6)
    Zm = Z + 0.3                                               # columns with a mean
    assert np.abs(CO.two_level(M, Zm, Wm) @ np.ones(N)).max() > 1e-3
