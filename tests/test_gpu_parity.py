"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances: FP64 paths match the oracle to ~1e-12 relative element by element
(operators, one V-cycle) and to 1e-10 relative for solves; mixed-precision
solves (FP32 V-cycles under FP64 CG, refinement) reach the 1e-8 relative
residual and match the FP64 solution to ~1e-8 (solution error is bounded by
the condition number times the residual).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact as ex
from oracle import iterative as it
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


def T(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def H(t):
    return t.detach().cpu().numpy()


def make(dev, shape, q, kappa=None, **kw):
    from paper_1306_3159_amd import BlobRD
    return BlobRD(shape, T(q, dev), None if kappa is None else T(kappa, dev), **kw)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ operators
CASES = [((32, 32, 32), 40, 1.0, 4), ((24, 24, 24), 30, 0.7, 4), ((20, 20, 20), 25, 1.0, 4),
         ((16, 32, 24), 20, 1.0, 4), ((48, 48, 48), 60, 1.0, 3), ((8, 8, 8), 3, 1.0, 4)]


@pytest.mark.parametrize("shape,N,h,w", CASES)
def test_interp_spread_apply_parity(dev, shape, N, h, w):
    _say("interp/spread/apply", shape, N, h, w)
    rng = np.random.default_rng(100 + N)
    nz, ny, nx = shape
    q = rng.uniform(-2.0, 2.0 + nx * h, size=(N, 3)) * np.array([1.0, ny / nx, nz / nx])
    kappa = W.log_uniform(rng, 1e-2, 1e2, N)
    c = rng.standard_normal(shape)
    lam = rng.standard_normal(N)
    S = make(dev, shape, q, kappa, h=h, kernel_w=w)
    qw = q.copy()  # oracle uses the nearest periodic image itself
    jc = H(S.interp(T(c, dev)))
    assert np.max(np.abs(jc - ex.interp(c, qw, h, w))) < 1e-13 * max(1, np.abs(jc).max())
    sl = H(S.spread(T(lam, dev)))
    ref = ex.spread(lam, qw, shape, h, w)
    assert np.max(np.abs(sl - ref)) < 1e-13 * np.abs(ref).max()
    for alpha in (0.0, 0.37):
        y = H(S.apply(T(c, dev), alpha, True))
        refy = ex.apply_B(c, qw, kappa, alpha, 1.0, h, w)
        assert np.max(np.abs(y - refy)) < 1e-12 * np.abs(refy).max()
    S.close()


# The densest batch suspensions (RSA capped at an excluded-volume fraction of 1/4: 579 blobs on
# 32^3, 1955 on 48^3) put about 9 and 18 blobs in each 8^3 tile, so a tile's 27-tile neighbourhood
# holds 250-500 candidates and the spread plan stages them in LDS over several passes.
DENSE = [(32, 579, 4), (32, 579, 3), (48, 1955, 4), (48, 1955, 3)]


@pytest.mark.parametrize("n,N,w", DENSE)
def test_interp_spread_apply_parity_dense(dev, n, N, w):
    _say("interp/spread/apply dense", n, N, w)
    assert N == W.rsa_cap(n)
    rng = np.random.default_rng(700 + N + w)
    q = W.rsa_positions(rng, n, N, 3.0)
    # candidates of the busiest 8^3 tile (blobs whose base cell lies in it or its 26 neighbours)
    # exceed the 128 that one LDS staging pass holds
    nt = n // 8
    tiles = (np.floor(q - 0.5).astype(int) % n) // 8
    cnt = np.zeros((nt,) * 3, int)
    np.add.at(cnt, (tiles[:, 2], tiles[:, 1], tiles[:, 0]), 1)
    cand = sum(np.roll(cnt, (a, b, c), (0, 1, 2)) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1))
    assert cand.max() > 128
    kappa = W.log_uniform(rng, 1e-2, 1e2, N)
    shape = (n, n, n)
    c = rng.standard_normal(shape)
    lam = rng.standard_normal(N)
    S = make(dev, shape, q, kappa, kernel_w=w)
    jc = H(S.interp(T(c, dev)))
    assert np.max(np.abs(jc - ex.interp(c, q, 1.0, w))) < 1e-13 * max(1, np.abs(jc).max())
    sl = H(S.spread(T(lam, dev)))
    ref = ex.spread(lam, q, shape, 1.0, w)
    assert np.max(np.abs(sl - ref)) < 1e-13 * np.abs(ref).max()
    for alpha in (0.0, 0.37):
        y = H(S.apply(T(c, dev), alpha, True))
        refy = ex.apply_B(c, q, kappa, alpha, 1.0, 1.0, w)
        assert np.max(np.abs(y - refy)) < 1e-12 * np.abs(refy).max()
    S.close()


# ------------------------------------------------------------------ multigrid
@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 48, 48), (16, 32, 24), (64, 64, 64)])
@pytest.mark.parametrize("alpha", [0.0, 2.0])
def test_vcycle_parity_fp64(dev, shape, alpha):
    _say("vcycle fp64", shape, alpha)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(shape)
    if alpha == 0.0:
        r -= r.mean()
    S = make(dev, shape, np.zeros((0, 3)))
    z = H(S.vcycle(T(r, dev), alpha))
    zr = it.vcycle(r, alpha)
    assert np.max(np.abs(z - zr)) < 1e-12 * np.abs(zr).max()
    S.close()


@pytest.mark.parametrize("alpha", [0.0, 2.0])
@pytest.mark.parametrize("shape", [(64, 64, 64), (48, 48, 48), (24, 40, 56)])
def test_vcycle_parity_mixed(dev, alpha, shape):
    """FP32 V-cycle against the FP64 oracle cycle. 64^3 and 48^3 run the vector forms of every
    per-level kernel (the four-row-block restriction included); on 24 x 40 x 56 the second
    level has 14-cell rows, so its correction and restriction take the one-cell forms."""
    _say("vcycle mixed", alpha, shape)
    rng = np.random.default_rng(8)
    r = rng.standard_normal(shape)
    if alpha == 0.0:
        r -= r.mean()
    from paper_1306_3159_amd import MIXED
    S = make(dev, shape, np.zeros((0, 3)), precision=MIXED)
    z = H(S.vcycle(T(r, dev), alpha))
    zr = it.vcycle(r, alpha)
    assert rel(z, zr) < 2e-6
    # element by element: a local slip in one of the ragged one-cell forms would pass the norm
    # check; 1e-5 of the field's largest value is about 100 FP32 units in the last place
    assert np.max(np.abs(z - zr)) < 1e-5 * np.abs(zr).max()
    S.close()


# ------------------------------------------------------------------ reactive
@pytest.mark.parametrize("prec", [0, 1])
def test_single_blob_reactive(dev, prec):
    """32^3, one blob at a seeded position, kappa = 1, f = 1, steady (alpha = 0)."""
    inst = W.single_blob()
    _say("single blob reactive", prec)
    S = make(dev, inst.n, inst.q, inst.kappa, precision=prec, rtol=inst.rtol if prec == 0 else 1e-8)
    c, st = S.solve_reactive(T(inst.f, dev))
    c = H(c)
    assert st["rc"] == 0, st
    ce, mu = ex.solve_reactive(inst.f, inst.q, inst.kappa, 0.0)
    tol = 1e-10 if prec == 0 else 1e-8
    assert ex.reactive_residual(c, inst.f, inst.q, inst.kappa, 0.0) <= tol
    assert rel(c, ce) < tol
    # closed form: mean(c) = V (1/kappa + gamma / D)
    gam = ex.gamma_single_blob(inst.q[0], (32, 32, 32))
    assert c.mean() == pytest.approx(32 ** 3 * (1.0 + gam), rel=tol)
    S.close()


@pytest.mark.parametrize("alpha", [0.0, 0.5])
@pytest.mark.parametrize("prec", [0, 1])
def test_reactive_many_blobs(dev, alpha, prec):
    _say("reactive many", alpha, prec)
    rng = np.random.default_rng(31)
    n = 32
    q = W.rsa_positions(rng, n, 40, 3.0)
    kappa = W.log_uniform(rng, 1e-2, 1e2, 40)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    S = make(dev, n, q, kappa, precision=prec, rtol=1e-10 if prec == 0 else 1e-8)
    c, st = S.solve_reactive(T(f, dev), alpha=alpha)
    c = H(c)
    assert st["rc"] == 0, st
    ce, _ = ex.solve_reactive(f, q, kappa, alpha)
    tol = 1e-10 if prec == 0 else 1e-8
    assert ex.reactive_residual(c, f, q, kappa, alpha) <= tol
    assert rel(c, ce) < 10 * tol
    S.close()


# ------------------------------------------------------------------ absorbing
@pytest.mark.parametrize("alpha", [0.0, 0.25])
@pytest.mark.parametrize("prec", [0, 1])
def test_absorbing_small(dev, alpha, prec):
    _say("absorbing small", alpha, prec)
    rng = np.random.default_rng(41)
    n = 32
    q = W.rsa_positions(rng, n, 30, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    S = make(dev, n, q, precision=prec, rtol=1e-10 if prec == 0 else 1e-8)
    c, lam, st = S.solve_absorbing(T(f, dev), alpha=alpha)
    c, lam = H(c), H(lam)
    assert st["rc"] == 0, st
    ce, le = ex.solve_absorbing(f, q, alpha)
    tol = 1e-10 if prec == 0 else 1e-8
    assert ex.absorbing_residual(c, lam, f, q, alpha) <= tol
    assert rel(lam, le) < 100 * tol
    assert rel(c, ce) < 100 * tol
    if alpha == 0.0:
        assert lam.sum() == pytest.approx(f.sum(), rel=1e-12)
    S.close()


def test_single_absorbing_blob_radius(dev):
    """Sec. IV.A: single absorbing blob at a node with s = 1/V: a ~ 1.27 h (four-point)."""
    n = 64
    V = float(n ** 3)
    q = np.array([[32.0, 32.0, 32.0]])
    _say("radius", n)
    S = make(dev, n, q, rtol=1e-10)
    c, lam, st = S.solve_absorbing(T(np.full((n, n, n), 1.0 / V), dev))
    c = H(c)
    a = ex.radius_extrapolated(ex.radius_from_mean(c.mean(), 1.0 / V, V), n)
    assert a == pytest.approx(1.27, rel=0.01)
    assert H(lam)[0] == pytest.approx(1.0, rel=1e-12)
    S.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_lattice_128_uniform_source(dev, prec):
    """128^3 grid, 8^3 blobs 16h apart at cell vertices, f = 1: lam_i = 16^3 and c equals
    the one-cell (16^3) solution tiled 8 times per axis."""
    inst = W.cubic_lattice()
    _say("lattice128", prec)
    S = make(dev, inst.n, inst.q, precision=prec, rtol=1e-8)
    c, lam, st = S.solve_absorbing(T(inst.f, dev))
    assert st["rc"] == 0, st
    c, lam = H(c), H(lam)
    c1, _ = ex.solve_absorbing(np.ones((16, 16, 16)), np.array([[8.0, 8.0, 8.0]]), 0.0)
    tiled = np.tile(c1, (8, 8, 8))
    assert np.max(np.abs(lam - 4096.0)) < 1e-8 * 4096
    assert rel(c, tiled) < 1e-8
    assert st["rel_resid"] <= 1e-8
    S.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_lattice_128_random_source(dev, prec):
    """Same lattice, random source: the Schur GMRES does real work. Checked through the
    oracle's FP64 saddle residual at full size and sampled against the oracle solve."""
    inst = W.cubic_lattice(random_f=True)
    _say("lattice128 random f", prec)
    S = make(dev, inst.n, inst.q, precision=prec, rtol=1e-8)
    c, lam, st = S.solve_absorbing(T(inst.f, dev))
    assert st["rc"] == 0, st
    c, lam = H(c), H(lam)
    r = ex.absorbing_residual(c, lam, inst.f, inst.q, 0.0)
    assert r <= 1e-8
    assert lam.sum() == pytest.approx(inst.f.sum(), rel=1e-12)
    S.close()


# ------------------------------------------------------------------ time stepping
def test_backward_euler_steps(dev):
    _say("BE steps")
    rng = np.random.default_rng(51)
    n = 32
    q = W.rsa_positions(rng, n, 20, 3.0)
    kappa = W.log_uniform(rng, 1e-2, 1e2, 20)
    f = np.ones((n, n, n))
    S = make(dev, n, q, kappa, rtol=1e-11)
    c = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    ce = np.zeros((n, n, n))
    G = ex.schur_matrix(q, (n, n, n), 2.0)
    for k in range(3):
        st = S.step(T(f, dev), c, 0.5)
        assert st["rc"] == 0
        ce = ex.step(ce, f, q, kappa, 0.5, G=G)
    assert rel(H(c), ce) < 1e-10
    S.close()


@pytest.mark.parametrize("prec,solver", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_absorbing_steps(dev, prec, solver):
    """Backward-Euler steps of an absorbing suspension (A = I/dt - D L, J c = 0) against the
    oracle's exact steps, with GMRES warm-started from the previous step's multipliers; a cold
    start reaches the same answer within the tolerance."""
    _say("absorbing steps", prec, solver)
    rng = np.random.default_rng(53)
    n, dt = 32, 0.5
    q = W.rsa_positions(rng, n, 30, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    tol = 1e-10 if prec == 0 else 1e-8
    S = make(dev, n, q, precision=prec, rtol=tol, saddle_solver=solver)
    G = ex.schur_matrix(q, (n, n, n), 1.0 / dt)
    c = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    lam = torch.zeros(30, dtype=torch.float64, device=dev)
    ce = np.zeros((n, n, n))
    ft = T(f, dev)
    for k in range(3):
        c_old = c.clone()
        st = S.step_absorbing(ft, c, lam, dt, warm=k > 0)
        assert st["rc"] == 0 and st["rel_resid"] <= tol, (k, st)
        g = f + H(c_old) / dt
        assert ex.absorbing_residual(H(c), H(lam), g, q, 1.0 / dt) <= tol
        ce, le = ex.step_absorbing(ce, f, q, dt, G=G)
        assert rel(H(c), ce) < 100 * tol
        assert rel(H(lam), le) < 100 * tol
        if k == 2:
            c_cold, lam_cold = c_old.clone(), torch.zeros_like(lam)
            st_cold = S.step_absorbing(ft, c_cold, lam_cold, dt, warm=False)
            assert st_cold["rc"] == 0
            assert rel(H(c_cold), H(c)) < 100 * tol and rel(H(lam_cold), H(lam)) < 100 * tol
            print("warm", st["outer_iters"], "cold", st_cold["outer_iters"], flush=True)
            assert st["outer_iters"] <= st_cold["outer_iters"]
    S.close()


def test_absorbing_step_errors(dev):
    _say("absorbing step errors")
    from paper_1306_3159_amd import BlobRDError
    rng = np.random.default_rng(54)
    S = make(dev, 16, W.rsa_positions(rng, 16, 3, 3.0))
    f = torch.ones((16, 16, 16), dtype=torch.float64, device=dev)
    c = torch.zeros_like(f)
    lam = torch.zeros(3, dtype=torch.float64, device=dev)
    for dt in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(BlobRDError):
            S.step_absorbing(f, c, lam, dt)
    with pytest.raises(ValueError):
        S.step_absorbing(f, c, torch.zeros(4, dtype=torch.float64, device=dev), 0.5)
    S.close()
    S0 = make(dev, 16, np.zeros((0, 3)))
    with pytest.raises(BlobRDError):
        S0.step_absorbing(f, c, torch.zeros(0, dtype=torch.float64, device=dev), 0.5)
    S0.close()


# ------------------------------------------------------------------ errors, determinism
def test_error_codes(dev):
    _say("errors")
    from paper_1306_3159_amd import BlobRD, BlobRDError
    with pytest.raises(BlobRDError) as e:
        BlobRD((36, 36, 36), T(np.zeros((1, 3)), dev))
    assert e.value.code == -1
    S = make(dev, 16, np.array([[3.0, 4.0, 5.0]]))       # kappa missing -> zero rates
    with pytest.raises(BlobRDError) as e:
        S.solve_reactive(T(np.ones((16, 16, 16)), dev))
    assert e.value.code == -4
    S.close()
    S = make(dev, 16, np.zeros((0, 3)))
    with pytest.raises(BlobRDError) as e:
        S.solve_absorbing(T(np.ones((16, 16, 16)), dev))
    assert e.value.code == -1
    S.close()


def test_bitwise_deterministic(dev):
    _say("determinism")
    rng = np.random.default_rng(61)
    n = 32
    q = W.rsa_positions(rng, n, 50, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    outs = []
    for _ in range(2):
        S = make(dev, n, q, precision=1)
        c, lam, st = S.solve_absorbing(T(f, dev))
        outs.append((H(c), H(lam)))
        S.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_graph_replay_matches_eager(dev, monkeypatch):
    """CG iterations replayed from captured HIP graphs give bitwise the same answers as
    eager launches; several solves in a row (graph replays with eager work between)."""
    _say("graphs vs eager")
    rng = np.random.default_rng(71)
    n = 32
    q = W.rsa_positions(rng, n, 40, 3.0)
    kappa = W.log_uniform(rng, 1e-2, 1e2, 40)
    fs = [1.0 + 0.5 * rng.standard_normal((n, n, n)) for _ in range(3)]
    res = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("BLOB_RD_GRAPHS", mode)
        S = make(dev, n, q, kappa, precision=1)
        outs = []
        for f in fs:
            c, lam, st = S.solve_absorbing(T(f, dev))
            cr, st2 = S.solve_reactive(T(f, dev))
            outs.append((H(c), H(lam), H(cr)))
        res[mode] = outs
        S.close()
    for a, b in zip(res["1"], res["0"]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_batch_matches_solo(dev):
    """Uneven instances (grids 32/48/64, reactive and absorbing) solved concurrently on
    their own streams give bitwise the results of solving each alone."""
    _say("batch")
    from paper_1306_3159_amd import BlobRD, solve_streams
    specs = [(32, 60, 0), (48, 200, 1), (64, 300, 0), (32, 20, 1), (48, 90, 0), (64, 150, 1)]
    inst = []
    for k, (n, N, kind) in enumerate(specs):
        rng = np.random.default_rng(800 + k)
        q = W.rsa_positions(rng, n, N, 3.0)
        kap = W.log_uniform(rng, 1e-2, 1e2, N)
        inst.append((n, q, kap, kind))

    def handles():
        out = []
        for n, q, kap, kind in inst:
            out.append(make(dev, n, q, kap, precision=1, stream=torch.cuda.Stream(dev)))
        return out

    solo = []
    for S, (n, q, kap, kind) in zip(handles(), inst):
        f = T(np.ones((n, n, n)), dev)
        torch.cuda.synchronize()
        if kind == 0:
            c, st = S.solve_reactive(f)
            solo.append((H(c), None))
        else:
            c, lam, st = S.solve_absorbing(f)
            solo.append((H(c), H(lam)))
        assert st["rc"] == 0
        S.close()
    Hs = handles()
    fs = [T(np.ones((n, n, n)), dev) for n, _, _, _ in inst]
    cs = [torch.zeros((n, n, n), dtype=torch.float64, device=dev) for n, _, _, _ in inst]
    ls = [torch.zeros(q.shape[0], dtype=torch.float64, device=dev) if kind else None for _, q, _, kind in inst]
    torch.cuda.synchronize()
    rc, stats = solve_streams(Hs, [k for *_, k in inst], fs, cs, ls, threads=4)
    assert rc == 0, stats
    for (c0, l0), c, l in zip(solo, cs, ls):
        assert np.array_equal(H(c), c0)
        if l0 is not None:
            assert np.array_equal(H(l), l0)
    for S in Hs:
        S.close()


@pytest.fixture(scope="module")
def rsa256():
    return W.disordered(kind="reactive")


def test_rsa256_reactive_full_size(dev, rsa256):
    """256^3, 2e4 RSA blobs, kappa log-uniform in [1e-2, 1e2], f = 1: steady reactive solve
    (FP32 V-cycles, FP64 CG) checked by the oracle's FP64 residual at full size."""
    inst = rsa256
    _say("rsa256 reactive")
    S = make(dev, inst.n, inst.q, inst.kappa, precision=1, rtol=1e-8)
    c, st = S.solve_reactive(T(inst.f, dev))
    assert st["rc"] == 0, st
    print("rsa256 reactive", st, flush=True)
    assert ex.reactive_residual(H(c), inst.f, inst.q, inst.kappa, 0.0) <= 1e-8
    S.close()


def test_rsa256_absorbing_full_size(dev, rsa256):
    inst = rsa256
    _say("rsa256 absorbing")
    S = make(dev, inst.n, inst.q, precision=1, rtol=1e-8)
    c, lam, st = S.solve_absorbing(T(inst.f, dev))
    assert st["rc"] == 0, st
    print("rsa256 absorbing", st, flush=True)
    c, lam = H(c), H(lam)
    assert ex.absorbing_residual(c, lam, inst.f, inst.q, 0.0) <= 1e-8
    assert lam.sum() == pytest.approx(inst.f.sum(), rel=1e-12)
    S.close()


def test_rsa256_learned_block_fgmres_full_size(dev):
    """The learned + FP32 headline solve at full size: 256^3, 10^4 RSA blobs, f = 1, the
    committed network weights, block FGMRES(30) with the approximate-Schur preconditioner
    (m = 5, n = 1) whose inner GMRES is right-preconditioned by W, FP32 V-cycles. The oracle's
    FP64 saddle residual of the answer meets 1e-8, the multipliers carry the whole source
    (sum(lam) = h^3 sum(f), Appendix A) and the network was used (no fallback)."""
    import os
    from paper_1306_3159_amd import BlobRD, Net, MIXED, PRECOND_LEARNED
    inst = W.learned_eval(256, 10000, index=0)
    _say("rsa256 learned block FGMRES", inst.seed)
    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1306_3159_amd",
                         "weights", "precond_rsa256.npy")
    net = Net(dev)
    net.set_params(torch.tensor(np.load(wpath), device=dev))
    S = BlobRD(inst.n, T(inst.q, dev), precision=MIXED, schur_precond=PRECOND_LEARNED, rtol=1e-8)
    S.precond_build(net)
    c, lam, st = S.solve_absorbing_fgmres(T(inst.f, dev), precond="learned", m=5, n=1, restart=30)
    print("rsa256 learned block FGMRES", st, flush=True)
    assert st["rc"] == 0 and st["fallback"] == 0, st
    c, lam = H(c), H(lam)
    assert ex.absorbing_residual(c, lam, inst.f, inst.q, 0.0) <= 1e-8
    assert lam.sum() == pytest.approx(inst.f.sum(), rel=1e-12)
    S.close()
    net.close()


def test_rsa256_backward_euler(dev, rsa256):
    """Backward-Euler steps dt = 0.5 from c = 0: every step meets 1e-8 (oracle residual on
    the first two steps) and the total reactant grows monotonically toward steady state."""
    inst = rsa256
    _say("rsa256 BE")
    S = make(dev, inst.n, inst.q, inst.kappa, precision=1, rtol=1e-8)
    c = torch.zeros((inst.n,) * 3, dtype=torch.float64, device=dev)
    f = T(inst.f, dev)
    prev = None
    totals = []
    for k in range(20):
        if k < 2:
            prev = H(c)
        st = S.step(f, c, 0.5)
        assert st["rc"] == 0 and st["rel_resid"] <= 1e-8, (k, st)
        if k < 2:
            g = inst.f + prev / 0.5
            assert ex.reactive_residual(H(c), g, inst.q, inst.kappa, 2.0) <= 1e-8
        totals.append(float(c.sum()))
    assert all(b > a for a, b in zip(totals, totals[1:]))
    S.close()


@pytest.mark.parametrize("solver", [0, 1])
def test_rsa256_absorbing_steps(dev, rsa256, solver):
    """Absorbing suspension at full size (256^3, 2e4 RSA blobs), five backward-Euler steps
    dt = 0.5 from c = 0 with warm-started multipliers: every step meets 1e-8, the first is
    checked by the oracle's FP64 saddle residual, every step keeps the discrete mass balance
    h^3 sum(c1 - c0)/dt = h^3 sum(f) - sum(lam) up to its residual, and the warm starts need
    no more Krylov iterations than the cold first step (Schur GMRES, or the block FGMRES
    started from c^n and the previous multipliers)."""
    inst = rsa256
    _say("rsa256 absorbing steps", solver)
    n, dt = inst.n, 0.5
    S = make(dev, n, inst.q, precision=1, rtol=1e-8, saddle_solver=solver)
    c = torch.zeros((n,) * 3, dtype=torch.float64, device=dev)
    lam = torch.zeros(inst.q.shape[0], dtype=torch.float64, device=dev)
    f = T(inst.f, dev)
    fsum = float(f.sum())
    iters = []
    for k in range(5):
        c_old = c.clone()
        st = S.step_absorbing(f, c, lam, dt, warm=k > 0)
        assert st["rc"] == 0 and st["rel_resid"] <= 1e-8, (k, st)
        iters.append(st["outer_iters"])
        gnorm = float(torch.linalg.vector_norm(f + c_old / dt))
        balance = float((c - c_old).sum()) / dt - (fsum - float(lam.sum()))
        assert abs(balance) <= 1e-8 * gnorm * math.sqrt(c.numel()), (k, balance)
        if k == 0:
            assert ex.absorbing_residual(H(c), H(lam), inst.f, inst.q, 1.0 / dt) <= 1e-8
    print("rsa256 absorbing steps, GMRES iterations", iters, flush=True)
    assert max(iters[1:]) <= iters[0]
    S.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_blocked_levels_bitwise(dev, monkeypatch, prec):
    """The temporally blocked launches of the coarser per-level levels (pre-smoothing, residual and
    restriction in one launch; correction and post-smoothing in another) give bitwise the results of
    the per-step launches: one V-cycle and a whole absorbing solve."""
    _say("blocked levels, prec", prec)
    rng = np.random.default_rng(91)
    n = 128
    q = W.rsa_positions(rng, n, 300, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    r = rng.standard_normal((n, n, n))
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("BLOB_RD_BLOCKED", mode)
        S = make(dev, n, q, precision=prec)
        z = H(S.vcycle(T(r, dev), 0.0))
        c, lam, st = S.solve_absorbing(T(f, dev))
        assert st["rc"] == 0
        out[mode] = (z, H(c), H(lam))
        S.close()
    for a, b in zip(out["1"], out["0"]):
        assert np.array_equal(a, b)
