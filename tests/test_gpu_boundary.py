"""The batch handle and the handle-owned learned network of the C ABI (blob_rd_create_batch,
blob_rd_solve_batch, blob_rd_precond_set_weights / get_weights / train_step), through the
ctypes binding, against the oracle and against the equivalent explicit calls."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact as ex
from oracle import learned as LN
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1306_3159_amd import native
    native.load_library()
    return torch.device("cuda:0")


def T(a, dev, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)


def rand_params(seed):
    rng = np.random.default_rng(seed)
    p = LN.init_params(seed)
    p["b1"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
    p["b2"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
    p["w3"] = (0.05 * rng.standard_normal(64)).astype(np.float32)
    p["b3"] = np.array([0.02], np.float32)
    return p


def test_set_weights_builds_the_same_w(dev):
    """set_weights on a learned handle gives bitwise the W of precond_build with a network holding
    the same parameters, and get_weights returns the blob that was set."""
    _say("set_weights")
    from paper_1306_3159_amd import BlobRD, Net, PRECOND_LEARNED, weights_blob, blob_params
    rng = np.random.default_rng(31)
    n, N = 48, 120
    q = W.rsa_positions(rng, n, N, 3.0)
    p = rand_params(32)
    blob = weights_blob(LN.flatten(p))
    A = BlobRD(n, T(q, dev), schur_precond=PRECOND_LEARNED)
    # the untrained own network is the paper's diagonal preconditioner
    _, col0, val0 = (t.cpu().numpy() for t in A.precond_csr())
    ptr0 = A.precond_csr()[0].cpu().numpy()
    row0 = np.repeat(np.arange(N), np.diff(ptr0))
    assert np.allclose(val0[row0 == col0], 4 * math.pi * LN.A0, rtol=1e-15) and np.all(val0[row0 != col0] == 0)
    A.precond_set_weights(blob)
    assert A.precond_get_weights() == blob
    net = Net(dev)
    net.set_params(T(blob_params(blob), dev, torch.float32))
    B = BlobRD(n, T(q, dev))
    B.precond_build(net)
    for a, b in zip(A.precond_csr(), B.precond_csr()):
        assert torch.equal(a, b)
    # the oracle's matrix-unit model of the same network
    optr, ocol, oval, _ = LN.assemble(LN.rounded(LN.unflatten(blob_params(blob))), q, (n, n, n), mfma_operands=True)
    ptr, col, val = (t.cpu().numpy() for t in A.precond_csr())
    assert np.array_equal(ptr, optr) and np.array_equal(col, ocol)
    diag = (np.repeat(np.arange(N), np.diff(optr)) == ocol) * 4 * math.pi * LN.A0
    from test_gpu_learned import w_matches_model
    w_matches_model(val, oval, diag)
    for S in (A, B):
        S.close()
    net.close()


def test_train_step(dev):
    """One train_step on the handle's own network: the loss is the oracle's, the update is the
    explicit path's (zero_grad, loss_grad, Adam) bit for bit, the first Adam step moves every
    weight with a clear gradient by lr against the oracle gradient's sign, and W follows."""
    _say("train_step")
    from paper_1306_3159_amd import BlobRD, Net, PRECOND_LEARNED, weights_blob, blob_params
    rng = np.random.default_rng(33)
    n, N, Sm, lr = 48, 150, 4, 1e-3
    q = W.rsa_positions(rng, n, N, 3.0)
    p = rand_params(34)
    blob = weights_blob(LN.flatten(p))
    p0 = blob_params(blob)
    X = rng.standard_normal((Sm, N))
    X -= X.mean(1, keepdims=True)
    Y = 0.05 * rng.standard_normal((Sm, N))
    A = BlobRD(n, T(q, dev), schur_precond=PRECOND_LEARNED)
    A.precond_set_weights(blob)
    loss = A.precond_train_step(T(X, dev), T(Y, dev), lr)
    loss_o, g_o = LN.loss_and_grad(LN.unflatten(p0), q, (n, n, n), X, Y)
    assert loss == pytest.approx(loss_o, rel=1e-3)
    # explicit path on a separate network with the same masters
    net = Net(dev)
    net.set_params(T(p0, dev, torch.float32))
    B = BlobRD(n, T(q, dev))
    B.precond_build(net)
    net.zero_grad()
    B.precond_loss_grad(net, T(X, dev), T(Y, dev))
    net.adam_step(lr)
    p1 = net.get_params().cpu().numpy()
    assert A.precond_get_weights() == weights_blob(p1)
    g = LN.flatten(g_o).astype(np.float64)
    clear = np.abs(g) > 1e-3 * np.abs(g).max()
    step = (p1.astype(np.float64) - p0.astype(np.float64))
    assert np.allclose(step[clear], -lr * np.sign(g[clear]), rtol=1e-3, atol=1e-7)
    # the handle's W is now the updated network's
    B.precond_build(net)
    for a, b in zip(A.precond_csr(), B.precond_csr()):
        assert torch.equal(a, b)
    for S in (A, B):
        S.close()
    net.close()


def test_own_network_errors(dev):
    """Handles without their own network refuse the calls; a wrong blob size is refused."""
    _say("own network errors")
    from paper_1306_3159_amd import BlobRD, BlobRDError, PRECOND_LEARNED, weights_blob
    rng = np.random.default_rng(35)
    q = W.rsa_positions(rng, 32, 20, 3.0)
    S = BlobRD(32, T(q, dev))
    with pytest.raises(BlobRDError):
        S.precond_set_weights(weights_blob(LN.flatten(LN.init_params(0))))
    S.close()
    S = BlobRD(32, T(q, dev), schur_precond=PRECOND_LEARNED)
    with pytest.raises(BlobRDError):
        S.precond_set_weights(b"\0" * 100)
    S.close()


def test_learned_handle_solves_with_set_weights(dev):
    """A block-learned handle given the committed weights by set_weights solves the absorbing
    system to the oracle's 1e-8 without falling back."""
    _say("learned handle solve")
    import os
    from paper_1306_3159_amd import BlobRD, MIXED, SOLVER_BLOCK_LEARNED, weights_blob
    rng = np.random.default_rng(36)
    n, N = 64, 156
    q = W.rsa_positions(rng, n, N, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1306_3159_amd",
                         "weights", "precond_rsa256.npy")
    S = BlobRD(n, T(q, dev), precision=MIXED, saddle_solver=SOLVER_BLOCK_LEARNED, rtol=1e-8)
    S.precond_set_weights(weights_blob(np.load(wpath)))
    c, lam, st = S.solve_absorbing(T(f, dev))
    assert st["rc"] == 0 and st["fallback"] == 0, st
    assert ex.absorbing_residual(c.cpu().numpy(), lam.cpu().numpy(), f, q, 0.0) <= 1e-8
    S.close()


def test_batch_handle(dev):
    """blob_rd_create_batch + blob_rd_solve_batch on uneven reactive and absorbing instances
    (Schur and block solvers, both precisions' members kept to one precision per batch): every
    answer meets 1e-8 by the oracle's residual, and equals the member solved alone."""
    _say("batch handle")
    from paper_1306_3159_amd import Batch, MIXED, SOLVER_BLOCK
    specs, inst = [], []
    for k, (n, N, kind, solver) in enumerate([(32, 60, 0, 0), (48, 200, 1, SOLVER_BLOCK), (64, 300, 0, 0),
                                              (32, 20, 1, 0), (96, 400, 1, SOLVER_BLOCK), (48, 90, 0, 0)]):
        rng = np.random.default_rng(4700 + k)
        q = W.rsa_positions(rng, n, N, 3.0)
        kap = W.log_uniform(rng, 1e-2, 1e2, N)
        f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
        specs.append(dict(shape=n, q=T(q, dev), kappa=T(kap, dev), precision=MIXED, kind=kind,
                          saddle_solver=solver))
        inst.append((n, q, kap, kind, f))
    B = Batch(specs)
    fs = [T(f, dev) for *_, f in inst]
    cs = [torch.zeros_like(f) for f in fs]
    ls = [torch.zeros(q.shape[0], dtype=torch.float64, device=dev) if kind else None for _, q, _, kind, _ in inst]
    rc, stats = B.solve(fs, cs, ls)
    assert rc == 0, stats
    for (n, q, kap, kind, f), c, l, m in zip(inst, cs, ls, B.members):
        if kind == 0:
            assert ex.reactive_residual(c.cpu().numpy(), f, q, kap, 0.0) <= 1e-8
            c2, st = m.solve_reactive(T(f, dev))
            assert torch.equal(c, c2)
        else:
            assert ex.absorbing_residual(c.cpu().numpy(), l.cpu().numpy(), f, q, 0.0) <= 1e-8
            c2, l2, st = m.solve_absorbing(T(f, dev))
            assert torch.equal(c, c2) and torch.equal(l, l2)
    B.close()
