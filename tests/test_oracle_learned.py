"""Pins for the learned-preconditioner oracle (oracle/learned.py)."""
import math

import numpy as np
import pytest

from oracle import learned as LN
import workloads as W


def test_bf16_rounding_matches_torch():
    """Round-to-nearest-even float32 -> bfloat16, checked against torch's conversion."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 10.0 ** rng.uniform(-6, 6, 5000),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0], np.float32)]).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(LN.bf16_round(a), ref)
    assert LN.bf16_round(np.array([1.0 + 2 ** -8], np.float32))[0] == 1.0       # tie -> even


def test_pair_list_matches_periodic_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(1)
    n = 40
    q = W.rsa_positions(rng, n, 300, 3.0)
    ptr, col = LN.pair_list(q, (n, n, n))
    tree = cKDTree(q, boxsize=n)
    ref = tree.query_ball_point(q, LN.RC - 1e-12)
    for i in range(q.shape[0]):
        assert sorted(ref[i]) == list(col[ptr[i]:ptr[i + 1]])
    # symmetric pattern, self included
    pairs = {(i, j) for i in range(q.shape[0]) for j in col[ptr[i]:ptr[i + 1]]}
    assert all((j, i) in pairs for (i, j) in pairs)
    assert all((i, i) in pairs for i in range(q.shape[0]))


def test_features_antisymmetric_and_bounded():
    rng = np.random.default_rng(2)
    n = 32
    q = rng.uniform(-5, n + 5, (50, 3))
    i = rng.integers(0, 50, 200)
    j = rng.integers(0, 50, 200)
    nu = LN.neighbour_counts(q, (n, n, n))
    a = LN.features(q, (n, n, n), i, j, nu)
    b = LN.features(q, (n, n, n), j, i, nu)
    assert a.shape[1] == LN.NFEAT == 12
    assert np.allclose(a[:, :3], -b[:, :3], atol=1e-15)
    assert np.allclose(a[:, 3], b[:, 3])
    assert np.all((a[:, 4:10] >= 0) & (a[:, 4:10] < 1))
    assert np.allclose(a[:, 4:7], b[:, 7:10])
    assert np.array_equal(a[:, 10], b[:, 11]) and np.array_equal(a[:, 10], 0.25 * nu[i])
    assert np.all(a[:, 3] <= math.sqrt(3) * n / 2 / LN.RC + 1e-12)


def test_neighbour_counts_match_a_periodic_kdtree():
    """nu_i = other blobs within r_c / 2 (minimum image): against scipy's periodic KD-tree, and
    every pair counted from both ends."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(8)
    n = 40
    q = W.rsa_positions(rng, n, 400, 3.0)
    nu = LN.neighbour_counts(q, (n, n, n))
    tree = cKDTree(q % n, boxsize=n)
    ref = np.array([len(x) - 1 for x in tree.query_ball_point(q % n, 0.5 * LN.RC - 1e-12)])
    assert np.array_equal(nu, ref)
    assert nu.sum() == 2 * len(tree.query_pairs(0.5 * LN.RC - 1e-12))
    assert nu.max() > 0


def test_untrained_network_is_the_diagonal_preconditioner():
    """Zero output layer: W = D h 4 pi a0 I, the diagonal approximation of eq. Schur_diagonal."""
    rng = np.random.default_rng(3)
    n = 32
    q = W.rsa_positions(rng, n, 60, 3.0)
    p = LN.rounded(LN.init_params(0))
    ptr, col, val, _ = LN.assemble(p, q, (n, n, n), h=1.0, D=2.0)
    row = np.repeat(np.arange(60), np.diff(ptr))
    assert np.allclose(val[row == col], 2.0 * 4 * math.pi * LN.A0)
    assert np.all(val[row != col] == 0.0)


def test_assembled_matrix_symmetric():
    rng = np.random.default_rng(4)
    n = 32
    q = W.rsa_positions(rng, n, 80, 3.0)
    p = LN.init_params(5)
    p["w3"] = rng.standard_normal(64).astype(np.float32)
    p["b3"] = np.array([0.3], np.float32)
    ptr, col, val, _ = LN.assemble(LN.rounded(p), q, (n, n, n))
    Wd = np.zeros((80, 80))
    for i in range(80):
        Wd[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
    assert np.allclose(Wd, Wd.T, rtol=0, atol=1e-12)


def test_gradient_matches_finite_differences():
    """Analytic backprop of the solve-pair loss against central differences (float64 weights)."""
    rng = np.random.default_rng(6)
    n = 24
    N = 30
    q = W.rsa_positions(rng, n, N, 3.0)
    p = LN.init_params(7)
    p["w3"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
    p["b3"] = np.array([0.05], np.float32)
    p64 = {k: np.asarray(v, np.float64) for k, v in p.items()}
    Xs = rng.standard_normal((3, N))
    Xs -= Xs.mean(1, keepdims=True)
    Ys = rng.standard_normal((3, N)) * 0.05
    loss, grads = LN.loss_and_grad(p64, q, (n, n, n), Xs, Ys, round_weights=False)
    eps = 1e-6
    for k, idx in (("W1", (3, 2)), ("W1", (10, 7)), ("b1", (5,)), ("W2", (4, 9)), ("W2", (63, 0)),
                   ("b2", (11,)), ("w3", (17,)), ("b3", (0,))):
        pp = {kk: vv.copy() for kk, vv in p64.items()}
        pm = {kk: vv.copy() for kk, vv in p64.items()}
        pp[k][idx] += eps
        pm[k][idx] -= eps
        lp, _ = LN.loss_and_grad(pp, q, (n, n, n), Xs, Ys, want_grad=False, round_weights=False)
        lm, _ = LN.loss_and_grad(pm, q, (n, n, n), Xs, Ys, want_grad=False, round_weights=False)
        fd = (lp - lm) / (2 * eps)
        assert grads[k][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_adam_first_step_moves_by_lr_times_sign():
    """Kingma and Ba: with bias correction the first step is lr * g / |g| (up to eps)."""
    p = {k: v.copy() for k, v in LN.init_params(8).items()}
    rng = np.random.default_rng(9)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    st = {}
    out = LN.adam_step(p, g, st, lr=1e-3)
    for k in LN.PARAM_ORDER:
        assert np.allclose(out[k].astype(np.float64), p[k].astype(np.float64) - 1e-3 * np.sign(g[k]), atol=1e-6)
    assert st["t"] == 1


def test_matrix_unit_model_within_bf16_of_fp64():
    """The matrix-unit model (bf16 operands in every network product) stays within the bf16
    rounding bound of the float64 network, which is pinned by finite differences above: W and
    every gradient tensor agree to 1e-2 (bf16 keeps 8 significand bits, 2^-9 relative), W stays
    exactly symmetric, and the model does differ from float64 (its roundings take effect)."""
    rng = np.random.default_rng(10)
    n, N = 32, 90
    q = W.rsa_positions(rng, n, N, 3.0)
    p = LN.init_params(11)
    p["b1"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
    p["w3"] = (0.3 * rng.standard_normal(64)).astype(np.float32)
    p["b3"] = np.array([0.2], np.float32)
    Xs = rng.standard_normal((3, N))
    Xs -= Xs.mean(1, keepdims=True)
    Ys = 0.05 * rng.standard_normal((3, N))
    l64, g64 = LN.loss_and_grad(p, q, (n, n, n), Xs, Ys)
    lmu, gmu = LN.loss_and_grad(p, q, (n, n, n), Xs, Ys, mfma_operands=True)
    assert lmu == pytest.approx(l64, rel=1e-2)
    for k in LN.PARAM_ORDER:
        d = np.linalg.norm(gmu[k] - g64[k]) / np.linalg.norm(g64[k])
        assert d <= 1e-2, (k, d)
    assert any(not np.array_equal(gmu[k], g64[k]) for k in ("W1", "W2"))
    ptr, col, v64, _ = LN.assemble(LN.rounded(p), q, (n, n, n))
    _, _, vmu, _ = LN.assemble(LN.rounded(p), q, (n, n, n), mfma_operands=True)
    diag = (np.repeat(np.arange(N), np.diff(ptr)) == col) * 4 * math.pi * LN.A0
    assert 0 < np.linalg.norm(vmu - v64) <= 1e-2 * np.linalg.norm(v64 - diag)
    Wd = np.zeros((N, N))
    for i in range(N):
        Wd[i, col[ptr[i]:ptr[i + 1]]] = vmu[ptr[i]:ptr[i + 1]]
    assert np.array_equal(Wd, Wd.T)
