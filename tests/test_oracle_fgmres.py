"""Pins for the oracle of the paper's own saddle-point solver (flexible GMRES with the
diagonal and approximate-Schur preconditioners, Sec. III.E diffusion-limited case and the
appendix on preconditioning the saddle-point solver).

The preconditioner is pinned where the paper's derivation makes it exact (exact inner
solves), FGMRES against the minimal-residual property computed by brute force, and the
whole solver against the dense exact saddle solution.
"""
import math

import numpy as np
import pytest

from oracle import exact as ex
from oracle import iterative as it
from oracle import saddle_fgmres as fg
import workloads as W


def _setup(n, N, alpha, seed, h=1.0, D=1.0):
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    q = W.rsa_positions(rng, n * h, N, 3.0 * h) if N > 1 else rng.uniform(0, n * h, (1, 3))
    ops = fg.SaddleOps(q, shape, alpha, D, h)
    vg = rng.standard_normal(shape)
    vf = rng.standard_normal(N)
    return rng, ops, vg, vf


def _residual(ops, c, lam, vg, vf):
    kg, kf = ops.K(c, lam)
    num = math.sqrt(np.sum((kg - vg) ** 2) + np.sum((kf - vf) ** 2))
    return num / math.sqrt(np.sum(vg ** 2) + np.sum(vf ** 2))


@pytest.mark.parametrize("kind", ["diagonal", "schur"])
def test_precond_exact_for_one_blob_singular(kind):
    """A = -D L, one blob, exact inverses: the mean multiplier is fixed by the total source,
    the fluctuation space is empty, and the mean concentration comes from the constraint, so
    the preconditioner solves the block system exactly whatever gamma is."""
    rng, ops, vg, vf = _setup(8, 1, 0.0, 31, h=0.9, D=1.4)
    Ai = ops.exact_inverse()
    inv = fg.cycles_inverse(ops, Ai, 1)
    c, lam = fg.precondition(ops, vg, vf, kind, inv, inv, m=3, diag=123.0)
    assert _residual(ops, c, lam, vg, vf) < 1e-12


def test_precond_diagonal_exact_for_one_blob_with_exact_gamma():
    """A invertible, one blob: the Schur complement is the scalar M_11, so the diagonal variant
    with D/gamma replaced by 1/M_11 (eq. Schur_diagonal made exact) is an exact solve."""
    rng, ops, vg, vf = _setup(8, 1, 0.3, 32)
    M11 = ex.schur_matrix(ops.q, ops.shape, 0.3)[0, 0]
    inv = fg.cycles_inverse(ops, ops.exact_inverse(), 1)
    c, lam = fg.precondition(ops, vg, vf, "diagonal", inv, inv, diag=1.0 / M11)
    assert _residual(ops, c, lam, vg, vf) < 1e-12
    # any other constant is not exact
    c, lam = fg.precondition(ops, vg, vf, "diagonal", inv, inv, diag=0.5 / M11)
    assert _residual(ops, c, lam, vg, vf) > 1e-3


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_precond_schur_exact_with_enough_inner_iterations(alpha):
    """Approximate-Schur variant with exact inner solves and as many inner GMRES iterations as
    the multiplier space has dimensions (N, or N - 1 mean-zero fluctuations for A = -D L):
    eq. approx_Schur is then solved exactly, and the preconditioner is an exact inverse of the
    block system (the paper's eqs. c_exact and r_schur)."""
    rng, ops, vg, vf = _setup(12, 5, alpha, 33)
    inv = fg.cycles_inverse(ops, ops.exact_inverse(), 1)
    c, lam = fg.precondition(ops, vg, vf, "schur", inv, inv, m=5 if alpha > 0 else 4)
    assert _residual(ops, c, lam, vg, vf) < 1e-10
    c2, lam2 = fg.precondition(ops, vg, vf, "schur", inv, inv, m=2)
    assert _residual(ops, c2, lam2, vg, vf) > 1e-6  # truncated inner solve is approximate


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_precond_learned_exact_with_exact_schur_inverse(alpha):
    """Learned variant: when W is the exact inverse of the (projected) Schur complement, one
    inner iteration solves eq. approx_Schur (the preconditioned operator is the identity on
    the multiplier space) and, with exact inner solves, the preconditioner is exact."""
    rng, ops, vg, vf = _setup(12, 5, alpha, 38)
    G = ex.schur_matrix(ops.q, ops.shape, alpha)
    if alpha == 0.0:
        P = np.eye(5) - 1.0 / 5
        Winv = np.linalg.pinv(P @ G @ P)
    else:
        Winv = np.linalg.inv(G)
    inv = fg.cycles_inverse(ops, ops.exact_inverse(), 1)
    c, lam = fg.precondition(ops, vg, vf, "learned", inv, inv, m=1, w_apply=lambda v: Winv @ v)
    assert _residual(ops, c, lam, vg, vf) < 1e-10
    # a poor W needs more inner iterations
    c, lam = fg.precondition(ops, vg, vf, "learned", inv, inv, m=1, w_apply=lambda v: 3.0 * v - v.mean())
    assert _residual(ops, c, lam, vg, vf) > 1e-6


def test_gmres_fixed_is_minimal_residual():
    """gmres_fixed: the minimiser over the Krylov space, by brute force (QR of the explicit
    Krylov matrix and least squares)."""
    rng = np.random.default_rng(34)
    n = 12
    B = rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n)
    for m in (1, 3, 6):
        x = fg.gmres_fixed(lambda v: B @ v, b, m)
        K = np.column_stack([np.linalg.matrix_power(B, k) @ b for k in range(m)])
        Q, _ = np.linalg.qr(K)
        y = np.linalg.lstsq(B @ Q, b, rcond=None)[0]
        assert np.linalg.norm(b - B @ x) == pytest.approx(np.linalg.norm(b - B @ Q @ y), rel=1e-9)
    x = fg.gmres_fixed(lambda v: B @ v, b, n)
    assert np.linalg.norm(B @ x - b) < 1e-10 * np.linalg.norm(b)


def test_fgmres_minimal_residual_history():
    """With a fixed linear preconditioner P, FGMRES's estimate after k iterations is
    min |b - K P y| over the Krylov space of K P (brute force on the assembled matrices)."""
    rng, ops, vg, vf = _setup(8, 2, 0.3, 35)
    ncell, N = ops.ncell, ops.N
    Jd = ex.dense_J(ops.q, ops.shape)
    A = 0.3 * np.eye(ncell) - ex.dense_laplacian(ops.shape)
    K = np.block([[A, Jd.T], [Jd, np.zeros((N, N))]])
    P = np.diag(1.0 / np.concatenate([np.full(ncell, 6.3), np.full(N, 0.7)]))

    def app(M):
        def f(g, l):
            y = M @ np.concatenate([g.ravel(), l])
            return y[:ncell].reshape(ops.shape), y[ncell:]
        return f

    _, _, info = fg.fgmres(app(K), app(P), vg, vf, restart=40, rtol=1e-14, maxit=6)
    b = np.concatenate([vg.ravel(), vf])
    KP = K @ P
    for k in range(1, 7):
        Kr = np.column_stack([np.linalg.matrix_power(KP, i) @ b for i in range(k)])
        Q, _ = np.linalg.qr(Kr)
        y = np.linalg.lstsq(KP @ Q, b, rcond=None)[0]
        assert info["history"][k - 1] == pytest.approx(np.linalg.norm(b - KP @ Q @ y), rel=1e-8)


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 16 ** 2])
@pytest.mark.parametrize("kind", ["diagonal", "schur"])
def test_fgmres_with_multigrid_reaches_exact_solution(alpha, kind):
    """The solver with the oracle's multigrid V(2,2) cycles (n = 1, m = 5; A = L^-2 I - L as in
    the paper's tests, and the steady A = -L with the null-space handling) converges to the
    dense exact saddle solution, and the true residual of its answer matches its estimate."""
    rng = np.random.default_rng(36)
    n = 16
    q = np.stack(np.meshgrid(*[np.arange(2.0, n, 8.0)] * 3, indexing="ij"), -1).reshape(-1, 3)
    q = q + rng.uniform(-0.5, 0.5, q.shape)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    cyc = lambda r: it.vcycle(r, alpha)
    c, lam, info = fg.solve(f, q, alpha, kind=kind, rtol=1e-9, restart=30, cycle=cyc)
    ce, le = ex.solve_absorbing(f, q, alpha)
    assert np.linalg.norm(c - ce) / np.linalg.norm(ce) < 1e-8
    assert np.linalg.norm(lam - le) / np.linalg.norm(le) < 1e-8
    ops = fg.SaddleOps(q, f.shape, alpha)
    true = _residual(ops, c, lam, f, np.zeros(len(q)))
    assert true <= 1e-9
    # the flexible form keeps the estimate equal to the true residual of x0 + Z y
    assert true == pytest.approx(info["history"][-1] / info["bnorm"], rel=1e-3)


def test_fgmres_exact_preconditioner_converges_in_one_iteration():
    rng = np.random.default_rng(37)
    n = 12
    q = W.rsa_positions(rng, n, 4, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    c, lam, info = fg.solve(f, q, 0.2, kind="schur", m=4, rtol=1e-10)
    assert info["iters"] == 1
    ce, le = ex.solve_absorbing(f, q, 0.2)
    assert np.linalg.norm(c - ce) / np.linalg.norm(ce) < 1e-10


def test_outer_iterations_set_by_the_concentration_cycles():
    """The approximate-Schur preconditioner (appendix on preconditioning; eq. approx_Schur) with
    one V-cycle per approximate Poisson solve: at the 256^3 / 10^4 blob density (20 blobs in
    32^3), m = 5 inner GMRES iterations already solve the one-cycle Schur system as well as m = N
    does, and right-preconditioning them by the exact inverse Schur complement (the best any
    learned W can be) leaves the outer FGMRES count unchanged; only more concentration cycles
    (n = 2) lower it. This bounds what a better W can gain in the block solver."""
    rng = np.random.default_rng(100)
    n, N = 32, 20
    q = W.rsa_positions(rng, n, N, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    cyc = lambda r: it.vcycle(r, 0.0)
    G = ex.schur_matrix(q, (n, n, n), 0.0)
    P = np.eye(N) - 1.0 / N
    Minv = np.linalg.pinv(P @ G @ P)
    its = {}
    for name, kw in (("m5", dict(kind="schur", m=5)), ("mN", dict(kind="schur", m=N)),
                     ("exactW", dict(kind="learned", m=5, w_apply=lambda v: P @ (Minv @ (P @ v)))),
                     ("n2", dict(kind="schur", m=5, n=2))):
        c, lam, info = fg.solve(f, q, 0.0, cycle=cyc, **kw)
        assert ex.absorbing_residual(c, lam, f, q, 0.0) <= 1e-8
        its[name] = info["iters"]
    assert its["m5"] == its["mN"] == its["exactW"], its
    assert its["n2"] < its["m5"], its
