"""CPU FP64 oracle, part 3: the learned pairwise Schur preconditioner.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline); shares no
code with the HIP path.

The paper preconditions the Schur complement M = J A^+ S (eq. r_schur) with
the diagonal approximation M^{-1} ~ chi gamma^{-1} I, gamma ~ (4 pi a)^{-1}
(eq. Schur_diagonal, Sec. III.E). The learned preconditioner keeps that
diagonal and adds a short-ranged pairwise correction produced by a small
network, symmetric by construction:

    W_ij = D h [ delta_ij 4 pi a0 / h + (g(i, j) + g(j, i)) / 2 ],   |q_j - q_i| < r_c,

with a0 = 1.255 h (the position-averaged reactive radius of Sec. IV.A),
r_c = 12 h, minimum-image separations, and

    x(i, j) = [d / r_c (3), |d| / r_c, frac(q_i/h - 1/2) (3), frac(q_j/h - 1/2) (3),
               nu_i / 4, nu_j / 4]
    g = w3 . silu(W2 silu(W1 x + b1) + b2) + b3,   widths 12 -> 64 -> 64 -> 1,

where nu_i counts the other blobs within r_c / 2 of blob i (minimum image): the
pair's surroundings, which set how strongly its neighbours shield it.

The weights W1, W2, w3 are used rounded to bfloat16 (round to nearest even);
biases and all arithmetic here are float64. The preconditioner applied to a
Schur residual r is z = P W P r with P = I - 1 1^T / N (periodic null space,
Appendix A).

Training minimises, over sample pairs (x_s, y_s = P M P x_s) produced by the
method's own Schur operator,

    loss = (1/S) sum_s || P W y_s - x_s ||^2 / || x_s ||^2,

with Adam (Kingma and Ba, 2015) on float32 master weights.

Two arithmetic models of the same network. The default evaluates everything in
float64 on the bf16-rounded weights. With mfma_operands=True the oracle also
rounds to bfloat16 every operand that a bf16 matrix-unit product takes: the
features (layer 1) and the first hidden activations (layer 2) in the forward
pass, and the pre-activation gradients of layers 2 and 1 where they enter the
products of the backward pass (d h1 = d a2 W2, the W2 and W1 gradients). The
products and all sums stay float64; the rounding is treated as identity when
differentiating (as the hardware path does).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

RC = 12.0
WIDTH = 64
NFEAT = 12
NU_SCALE = 0.25  # the neighbour counts enter as nu / 4
A0 = 1.255   # reactive radius of a four-point blob, in units of h


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    """Seeded float32 initial weights: scaled normal hidden layers, zero output layer
    (so the untrained preconditioner is exactly the diagonal of eq. Schur_diagonal)."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": (rng.standard_normal((WIDTH, NFEAT)) * math.sqrt(2.0 / NFEAT)).astype(np.float32),
        "b1": np.zeros(WIDTH, np.float32),
        "W2": (rng.standard_normal((WIDTH, WIDTH)) * math.sqrt(2.0 / WIDTH)).astype(np.float32),
        "b2": np.zeros(WIDTH, np.float32),
        "w3": np.zeros(WIDTH, np.float32),
        "b3": np.zeros(1, np.float32),
    }
    return p


PARAM_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in PARAM_ORDER])


def unflatten(v: np.ndarray) -> Dict[str, np.ndarray]:
    shapes = {"W1": (WIDTH, NFEAT), "b1": (WIDTH,), "W2": (WIDTH, WIDTH), "b2": (WIDTH,), "w3": (WIDTH,),
              "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n], np.float32).reshape(shapes[k])
        o += n
    return out


def n_params() -> int:
    return WIDTH * NFEAT + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH + 1


# ---------------------------------------------------------------- pairs and features
def wrap_positions(q: np.ndarray, n, h: float = 1.0) -> np.ndarray:
    box = np.asarray(n, dtype=np.float64) * h
    return q - box * np.floor(q / box)


def pair_list(q: np.ndarray, n, h: float = 1.0, rc: float = RC) -> Tuple[np.ndarray, np.ndarray]:
    """All ordered pairs (i, j), j = i included, with minimum-image |q_j - q_i| < rc.

    Returned in CSR form (row pointer, column indices with columns ascending)."""
    box = np.asarray(n, dtype=np.float64) * h
    N = q.shape[0]
    rows = []
    for i in range(N):
        d = q - q[i]
        d -= box * np.round(d / box)
        r2 = np.einsum("ij,ij->i", d, d)
        rows.append(np.nonzero(r2 < rc * rc)[0])
    ptr = np.zeros(N + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    return ptr, np.concatenate(rows) if rows else np.zeros(0, np.int64)


def neighbour_counts(q: np.ndarray, n, h: float = 1.0, rc: float = RC) -> np.ndarray:
    """nu_i: the number of blobs j != i with minimum-image |q_j - q_i| < rc / 2."""
    box = np.asarray(n, dtype=np.float64) * h
    qw = wrap_positions(q, n, h)
    N = q.shape[0]
    nu = np.zeros(N)
    for i in range(N):
        d = qw - qw[i]
        d -= box * np.round(d / box)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        nu[i] = np.count_nonzero(r < 0.5 * rc) - 1
    return nu


def features(q: np.ndarray, n, i: np.ndarray, j: np.ndarray, nu: np.ndarray, h: float = 1.0,
             rc: float = RC) -> np.ndarray:
    box = np.asarray(n, dtype=np.float64) * h
    qw = wrap_positions(q, n, h)
    d = qw[j] - qw[i]
    d -= box * np.round(d / box)
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    si = qw[i] / h - 0.5
    sj = qw[j] / h - 0.5
    fi = si - np.floor(si)
    fj = sj - np.floor(sj)
    return np.concatenate([d / rc, (r / rc)[:, None], fi, fj, NU_SCALE * nu[i][:, None], NU_SCALE * nu[j][:, None]],
                          axis=1)


# ---------------------------------------------------------------- network
def silu(t):
    return t / (1.0 + np.exp(-t))


def dsilu(t):
    s = 1.0 / (1.0 + np.exp(-t))
    return s * (1.0 + t * (1.0 - s))


def rounded(p: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """Weights as the network uses them: W1, W2, w3 in bfloat16, biases float32."""
    out = {}
    for k in PARAM_ORDER:
        out[k] = bf16_round(p[k]) if k in ("W1", "W2", "w3") else np.asarray(p[k], np.float64)
    return out


def _operand(a, mfma_operands):
    """A matrix-product operand: bfloat16-rounded in the matrix-unit model, else as is."""
    return bf16_round(a) if mfma_operands else a


def forward(p: Dict[str, np.ndarray], X: np.ndarray, mfma_operands: bool = False):
    """g for each feature row of X (float64), with the cache needed by backward."""
    Xo = _operand(X, mfma_operands)
    a1 = Xo @ p["W1"].T + p["b1"]
    h1 = _operand(silu(a1), mfma_operands)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(a2)
    g = h2 @ p["w3"] + p["b3"][0]
    return g, (Xo, a1, h1, a2, h2, mfma_operands)


def backward(p, cache, dg):
    X, a1, h1, a2, h2, mfma_operands = cache
    grads = {"w3": h2.T @ dg, "b3": np.array([dg.sum()])}
    da2 = np.outer(dg, p["w3"]) * dsilu(a2)
    grads["b2"] = da2.sum(0)
    da2o = _operand(da2, mfma_operands)
    grads["W2"] = da2o.T @ h1
    da1 = (da2o @ p["W2"]) * dsilu(a1)
    grads["b1"] = da1.sum(0)
    grads["W1"] = _operand(da1, mfma_operands).T @ X
    return grads


def assemble(p_rounded, q, n, h=1.0, D=1.0, rc=RC, mfma_operands=False):
    """CSR of W: (ptr, col, val, cache) with val_ij = D h (diag + (g_ij + g_ji)/2)."""
    ptr, col = pair_list(q, n, h, rc)
    row = np.repeat(np.arange(q.shape[0]), np.diff(ptr))
    nu = neighbour_counts(q, n, h, rc)
    X = np.concatenate([features(q, n, row, col, nu, h, rc), features(q, n, col, row, nu, h, rc)])
    g, cache = forward(p_rounded, X, mfma_operands)
    m = row.size
    val = D * h * (0.5 * (g[:m] + g[m:]) + (row == col) * 4.0 * math.pi * A0)
    return ptr, col, val, (row, cache, m)


def spmv(ptr, col, val, x):
    y = np.zeros(ptr.size - 1)
    for i in range(ptr.size - 1):
        y[i] = np.dot(val[ptr[i]:ptr[i + 1]], x[col[ptr[i]:ptr[i + 1]]])
    return y


def project(v):
    return v - v.mean()


def apply(ptr, col, val, r):
    """z = P W P r."""
    return project(spmv(ptr, col, val, project(r)))


def loss_and_grad(params: Dict[str, np.ndarray], q, n, X_s: np.ndarray, Y_s: np.ndarray, h=1.0, D=1.0,
                  rc=RC, want_grad=True, round_weights=True, mfma_operands=False):
    """loss = (1/S) sum_s |P W y_s - x_s|^2 / |x_s|^2 and its gradient w.r.t. the
    float32 master parameters (the rounding to bfloat16 is treated as identity;
    round_weights=False evaluates everything with unrounded float64 weights;
    mfma_operands selects the matrix-unit model of the module docstring)."""
    pr = rounded(params) if round_weights else {k: np.asarray(params[k], np.float64) for k in PARAM_ORDER}
    ptr, col, val, (row, cache, m) = assemble(pr, q, n, h, D, rc, mfma_operands)
    S = X_s.shape[0]
    loss = 0.0
    GW = np.zeros(val.size)
    for s in range(S):
        x, y = X_s[s], Y_s[s]
        res = apply(ptr, col, val, y) - x
        nx2 = float(np.dot(x, x))
        loss += float(np.dot(res, res)) / nx2 / S
        # d loss / d val_e for e = (i, j): (2/(S |x|^2)) (P res)_i (P y)_j
        yp = project(y)
        rp = project(res)
        GW += (2.0 / (S * nx2)) * rp[row] * yp[col]
    if not want_grad:
        return loss, None
    dg_ij = D * h * 0.5 * GW
    dg = np.concatenate([dg_ij, dg_ij])
    grads = backward(pr, cache, dg)
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) of float32 master weights."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k in PARAM_ORDER:
        g = np.asarray(grads[k], np.float64)
        m = beta1 * state.get("m_" + k, np.zeros_like(g)) + (1 - beta1) * g
        v = beta2 * state.get("v_" + k, np.zeros_like(g)) + (1 - beta2) * g * g
        state["m_" + k], state["v_" + k] = m, v
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        out[k] = (np.asarray(params[k], np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return out
