"""GPU parity of the paper's own saddle-point solver (flexible GMRES on the block system with
the diagonal and approximate-Schur preconditioners) against the oracle, through the C ABI.

One preconditioner application is compared element by element with the oracle's steps run on
the oracle's own V(2,2) cycles (FP64 handle: the cycles agree to ~1e-12, so 1e-9 covers the
m = 5 inner GMRES iterations; mixed handle: FP32 cycles, 1e-4). Whole solves are compared with
the dense exact saddle solution and with the oracle solver's iteration counts.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact as ex
from oracle import iterative as it
from oracle import saddle_fgmres as fg
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make(dev, n, q, **kw):
    from paper_1306_3159_amd import BlobRD
    return BlobRD(n, T(q, dev), **kw)


def lattice(n, spacing, rng, jitter=0.0):
    pts = np.arange(spacing / 2.0, n, spacing)
    q = np.stack(np.meshgrid(pts, pts, pts, indexing="ij"), -1).reshape(-1, 3)
    return q + rng.uniform(-jitter, jitter, q.shape)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["diagonal", "schur"])
@pytest.mark.parametrize("alpha", [0.0, 1.0 / 32 ** 2])
def test_precond_parity(dev, alpha, kind, prec):
    _say("saddle precond", alpha, kind, prec)
    rng = np.random.default_rng(71)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    vg = rng.standard_normal((n, n, n))
    vf = rng.standard_normal(N)
    S = make(dev, n, q, precision=prec)
    zg, zl = S.saddle_precond(T(vg, dev), T(vf, dev), alpha=alpha, precond=kind, m=5, n=1)
    ops = fg.SaddleOps(q, (n, n, n), alpha)
    inv = fg.cycles_inverse(ops, lambda r: it.vcycle(r, alpha), 1)
    cg, cl = fg.precondition(ops, vg, vf, kind, inv, inv, m=5)
    tol = 1e-9 if prec == 0 else 1e-4
    assert rel(H(zg), cg) < tol
    assert rel(H(zl), cl) < tol
    # two cycles per approximate solve
    zg2, zl2 = S.saddle_precond(T(vg, dev), T(vf, dev), alpha=alpha, precond=kind, m=5, n=2)
    inv2 = fg.cycles_inverse(ops, lambda r: it.vcycle(r, alpha), 2)
    cg2, cl2 = fg.precondition(ops, vg, vf, kind, inv2, inv, m=5)
    assert rel(H(zg2), cg2) < tol
    assert rel(H(zl2), cl2) < tol
    S.close()


@pytest.mark.parametrize("kind", ["diagonal", "schur"])
@pytest.mark.parametrize("alpha", [0.0, 1.0 / 32 ** 2])
def test_fgmres_solve_matches_oracle(dev, alpha, kind):
    """FP64 handle: the exact saddle solution to the tolerance, and the oracle solver's iteration
    count (same arithmetic up to rounding order). Mixed handle: the same solution at 1e-8."""
    _say("fgmres solve", alpha, kind)
    rng = np.random.default_rng(72)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    ce, le = ex.solve_absorbing(f, q, alpha)
    _, _, info = fg.solve(f, q, alpha, kind=kind, rtol=1e-10, cycle=lambda r: it.vcycle(r, alpha))
    for prec, tol in ((0, 1e-10), (1, 1e-8)):
        S = make(dev, n, q, precision=prec, rtol=tol)
        c, lam, st = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond=kind)
        assert st["rc"] == 0, st
        c, lam = H(c), H(lam)
        assert st["rel_resid"] <= tol
        assert ex.absorbing_residual(c, lam, f, q, alpha) <= 1.01 * tol
        assert rel(c, ce) < 100 * tol and rel(lam, le) < 100 * tol
        print("prec", prec, kind, "alpha", alpha, "FGMRES", st["outer_iters"], "oracle", info["iters"],
              "cycles", st["vcycles"], flush=True)
        if prec == 0:
            assert abs(st["outer_iters"] - info["iters"]) <= 1
        S.close()


@pytest.mark.parametrize("kind", ["diagonal", "schur"])
def test_fgmres_second_gram_schmidt_pass(dev, kind, monkeypatch):
    """The classical Gram-Schmidt of the block FGMRES re-orthogonalises a new basis vector when the
    projection removed most of it; forcing that second pass on every vector (BLOB_RD_FG_REORTH=1)
    gives the same iterations and the same solution to the tolerance, and still the oracle's
    iteration count."""
    _say("fgmres second pass", kind)
    rng = np.random.default_rng(74)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    alpha = 1.0 / n ** 2
    _, _, info = fg.solve(f, q, alpha, kind=kind, rtol=1e-10, cycle=lambda r: it.vcycle(r, alpha))
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("BLOB_RD_FG_REORTH", mode)
        S = make(dev, n, q, precision=0, rtol=1e-10)
        c, lam, st = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond=kind)
        assert st["rc"] == 0 and st["rel_resid"] <= 1e-10, st
        assert abs(st["outer_iters"] - info["iters"]) <= 1
        out[mode] = (H(c), H(lam), st)
        S.close()
    assert out["0"][2]["outer_iters"] == out["1"][2]["outer_iters"]
    assert rel(out["1"][0], out["0"][0]) < 1e-9 and rel(out["1"][1], out["0"][1]) < 1e-9


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 32 ** 2])
def test_fgmres_steps_issued_ahead(dev, alpha, monkeypatch):
    """Arnoldi steps issued before the host has read the previous step's residual estimate:
    never (BLOB_RD_FG_AHEAD=0), when the contraction predicts no convergence (1, the default) and
    always (2, so the step that converges always has one more behind it, issued past
    convergence). The extra step must change nothing the solution update reads: bitwise the
    same solution, the same counts, and the exact solution to the tolerance."""
    _say("fgmres steps ahead", alpha)
    rng = np.random.default_rng(75)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    ce, le = ex.solve_absorbing(f, q, alpha)
    out = {}
    for mode in ("0", "1", "2"):
        monkeypatch.setenv("BLOB_RD_FG_AHEAD", mode)
        for prec, tol in ((0, 1e-10), (1, 1e-8)):
            S = make(dev, n, q, precision=prec, rtol=tol)
            c, lam, st = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond="schur")
            assert st["rc"] == 0 and st["rel_resid"] <= tol, st
            c, lam = H(c), H(lam)
            assert rel(c, ce) < 100 * tol and rel(lam, le) < 100 * tol
            out[(mode, prec)] = (c, lam, st["outer_iters"], st["vcycles"], st["inner_iters_total"], st["alg_bytes"])
            S.close()
    for prec in (0, 1):
        ref = out[("0", prec)]
        for mode in ("1", "2"):
            got = out[(mode, prec)]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
            assert got[2:] == ref[2:]


@pytest.mark.parametrize("alpha", [0.0, 0.05])
def test_fgmres_non_cubic_grid_matches_oracle(dev, alpha):
    """A 24 x 32 x 40 box (nz, ny, nx) with h = 0.7: half-rows of 20 cells, so the split-layout
    steps of the block preconditioner (its FP32 concentration estimate, the residual entry, the
    sum back to FP64) run their general forms on rows that are not powers of two. The exact
    saddle solution (FFT Schur matrix) to 1e-10 in FP64 and 1e-8 mixed, with the oracle's
    residual."""
    _say("fgmres non-cubic", alpha)
    shape, h = (24, 32, 40), 0.7
    rng = np.random.default_rng(76)
    N = 25
    nz, ny, nx = shape
    L = np.array([nx, ny, nz]) * h
    q = []
    while len(q) < N:
        p = rng.uniform(0.0, 1.0, 3) * L
        if all(np.linalg.norm((p - o + 0.5 * L) % L - 0.5 * L) >= 3.0 * h for o in q):
            q.append(p)
    q = np.array(q)
    f = 1.0 + 0.5 * rng.standard_normal(shape)
    ce, le = ex.solve_absorbing(f, q, alpha, h=h)
    from paper_1306_3159_amd import BlobRD
    for prec, tol in ((0, 1e-10), (1, 1e-8)):
        S = BlobRD(shape, T(q, dev), h=h, precision=prec, rtol=tol)
        c, lam, st = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond="schur")
        assert st["rc"] == 0 and st["rel_resid"] <= tol, st
        c, lam = H(c), H(lam)
        assert ex.absorbing_residual(c, lam, f, q, alpha, h=h) <= 1.01 * tol
        assert rel(c, ce) < 100 * tol and rel(lam, le) < 100 * tol
        S.close()


def test_fgmres_fixed_blob_count_lattice(dev):
    """The paper's fixed-N test (64 = 4^3 blobs on a lattice, A = L^-2 I - L) at L = 64 with both
    preconditioners: converges, and the oracle's FP64 residual agrees at full size."""
    _say("fgmres lattice 64")
    rng = np.random.default_rng(73)
    n = 64
    q = lattice(n, 16.0, rng)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    alpha = 1.0 / n ** 2
    S = make(dev, n, q, precision=1, rtol=1e-8)
    for kind in ("diagonal", "schur"):
        c, lam, st = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond=kind, restart=200 if kind == "diagonal"
                                              else 30)
        assert st["rc"] == 0, st
        print(kind, st, flush=True)
        assert ex.absorbing_residual(H(c), H(lam), f, q, alpha) <= 1e-8
    S.close()


def test_fgmres_errors_and_limits(dev):
    _say("fgmres errors")
    from paper_1306_3159_amd import BlobRDError
    rng = np.random.default_rng(74)
    n = 16
    q = W.rsa_positions(rng, n, 5, 3.0)
    f = T(1.0 + 0.5 * rng.standard_normal((n, n, n)), dev)
    S = make(dev, n, q, rtol=1e-10)
    c, lam, st = S.solve_absorbing_fgmres(f, precond="diagonal", maxit=2)
    assert st["rc"] == 1 and st["outer_iters"] == 2  # not converged, reported
    with pytest.raises(BlobRDError):
        S.solve_absorbing_fgmres(f, m=31)  # above the handle's GMRES restart length
    with pytest.raises(BlobRDError):
        S.solve_absorbing_fgmres(f, alpha=-1.0)
    with pytest.raises(BlobRDError):
        S.saddle_precond(f, torch.zeros(5, dtype=torch.float64, device=dev), n=65)
    with pytest.raises(ValueError):
        S.solve_absorbing_fgmres(f, restart=2000)
    lib = S._lib
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    from paper_1306_3159_amd.native import Stats, _saddle_opts, _ptr
    import ctypes
    o = _saddle_opts()
    cc = torch.zeros_like(f)
    ll = torch.zeros(5, dtype=torch.float64, device=dev)
    rc = lib.blob_rd_solve_absorbing_fgmres(S._h, 0.0, ctypes.byref(o), _ptr(f), _ptr(cc), _ptr(ll), _ptr(ws), 1024,
                                            ctypes.byref(Stats()))
    assert rc == -2  # workspace too small
    S.close()


def _net(dev, p):
    from paper_1306_3159_amd import Net
    from oracle import learned as LN
    net = Net(dev)
    net.set_params(torch.as_tensor(LN.flatten(p), dtype=torch.float32, device=dev))
    return net


@pytest.mark.parametrize("trained", [False, True])
def test_precond_parity_learned(dev, trained):
    """Learned variant (inner GMRES right-preconditioned by P W P). Untrained network: W is
    exactly the diagonal of eq. Schur_diagonal on both sides, so the FP64 handle matches the
    oracle to 1e-9. Random weights: the oracle's W is its matrix-unit model of the network
    (bf16 operands in every product), which the GPU's W matches to float32 accumulation
    except for rare bf16 rounding flips (one bf16 step of one hidden unit in a few entries);
    the preconditioner output then agrees to 1e-3."""
    _say("saddle precond learned", trained)
    from oracle import learned as LN
    from paper_1306_3159_amd import PRECOND_LEARNED
    rng = np.random.default_rng(75)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    vg = rng.standard_normal((n, n, n))
    vf = rng.standard_normal(N)
    p = LN.init_params(5)
    if trained:
        p["b1"] = (0.1 * rng.standard_normal(64)).astype(np.float32)
        p["w3"] = (0.05 * rng.standard_normal(64)).astype(np.float32)
    net = _net(dev, p)
    S = make(dev, n, q, precision=0, schur_precond=PRECOND_LEARNED)
    S.precond_build(net)
    zg, zl = S.saddle_precond(T(vg, dev), T(vf, dev), alpha=0.0, precond="learned", m=4)
    ptr, col, val, _ = LN.assemble(LN.rounded(p), q, n, mfma_operands=True)
    ops = fg.SaddleOps(q, (n, n, n), 0.0)
    inv = fg.cycles_inverse(ops, lambda r: it.vcycle(r, 0.0), 1)
    cg, cl = fg.precondition(ops, vg, vf, "learned", inv, inv, m=4, w_apply=lambda v: LN.apply(ptr, col, val, v))
    tol = 1e-3 if trained else 1e-9
    assert rel(H(zg), cg) < tol and rel(H(zl), cl) < tol
    S.close()
    net.close()


def test_fgmres_learned_solve_and_fallback(dev):
    """Learned block preconditioner: the solve reaches the tolerance and the exact answer; for
    alpha > 0 (the network approximates the steady Schur complement) and on a handle without a
    built W it falls back to the plain approximate-Schur variant and says so."""
    _say("fgmres learned solve")
    from oracle import learned as LN
    from paper_1306_3159_amd import PRECOND_LEARNED
    rng = np.random.default_rng(76)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    p = LN.init_params(6)
    p["w3"] = (0.05 * rng.standard_normal(64)).astype(np.float32)
    net = _net(dev, p)
    S = make(dev, n, q, precision=1, schur_precond=PRECOND_LEARNED, rtol=1e-8)
    S.precond_build(net)
    for alpha in (0.0, 1.0 / n ** 2):
        ce, le = ex.solve_absorbing(f, q, alpha)
        c, lam, st = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond="learned")
        assert st["rc"] == 0 and st["fallback"] == (1 if alpha > 0 else 0), st
        assert ex.absorbing_residual(H(c), H(lam), f, q, alpha) <= 1e-8
        assert rel(H(lam), le) < 1e-6
    S.close()
    S2 = make(dev, n, q, precision=1, rtol=1e-8)
    c, lam, st = S2.solve_absorbing_fgmres(T(f, dev), precond="learned")
    assert st["rc"] == 0 and st["fallback"] == 1
    S2.close()
    net.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_schur_apply_cycles_parity(dev, prec):
    """The approximate-Schur operator P J A_n^{-1} S P (n multigrid cycles) against the oracle's
    steps on its own cycles."""
    _say("schur apply cycles", prec)
    rng = np.random.default_rng(77)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    x = rng.standard_normal(N)
    S = make(dev, n, q, precision=prec)
    ops = fg.SaddleOps(q, (n, n, n), 0.0)
    xp = x - x.mean()
    for cyc in (1, 2):
        y = H(S.schur_apply_cycles(T(x, dev), 0.0, cyc))
        inv = fg.cycles_inverse(ops, lambda r: it.vcycle(r, 0.0), cyc)
        ref = ops.J(inv(ops.S(xp)))
        ref -= ref.mean()
        assert rel(y, ref) < (1e-10 if prec == 0 else 1e-5)
    S.close()


def test_fgmres_stops_at_rounding_floor(dev):
    """A tolerance below the FP64 rounding floor of the residual ends after two restarts that
    do not reduce it, reported as not converged with the floor as the residual."""
    _say("fgmres rounding floor")
    n = 16
    q = np.array([[8.0, 8.0, 8.0]])
    f = torch.full((n, n, n), 1.0 / n ** 3, dtype=torch.float64, device=dev)
    S = make(dev, n, q, rtol=1e-17)
    c, lam, st = S.solve_absorbing_fgmres(f, precond="schur", restart=10)
    assert st["rc"] == 1 and st["outer_iters"] < 200, st
    assert st["rel_resid"] < 1e-12
    S.close()


@pytest.mark.parametrize("kind", ["diagonal", "schur"])
def test_fgmres_three_point_kernel(dev, kind):
    """The three-point kernel (27-cell support): preconditioner parity with the oracle and the
    exact saddle solution."""
    _say("fgmres w=3", kind)
    rng = np.random.default_rng(78)
    n, N = 32, 30
    q = W.rsa_positions(rng, n, N, 3.0)
    vg = rng.standard_normal((n, n, n))
    vf = rng.standard_normal(N)
    f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
    S = make(dev, n, q, precision=0, kernel_w=3, rtol=1e-10)
    zg, zl = S.saddle_precond(T(vg, dev), T(vf, dev), alpha=0.0, precond=kind)
    ops = fg.SaddleOps(q, (n, n, n), 0.0, w=3)
    inv = fg.cycles_inverse(ops, lambda r: it.vcycle(r, 0.0), 1)
    cg, cl = fg.precondition(ops, vg, vf, kind, inv, inv, m=5)
    assert rel(H(zg), cg) < 1e-9 and rel(H(zl), cl) < 1e-9
    c, lam, st = S.solve_absorbing_fgmres(T(f, dev), precond=kind)
    assert st["rc"] == 0, st
    ce, le = ex.solve_absorbing(f, q, 0.0, w=3)
    assert rel(H(c), ce) < 1e-8 and rel(H(lam), le) < 1e-8
    S.close()


@pytest.mark.parametrize("prec,precond", [(1, "schur"), (0, "diagonal"), (1, "learned")])
def test_fgmres_graph_replays_match_eager(dev, monkeypatch, prec, precond):
    """The block FGMRES replays each Arnoldi step as a captured HIP graph: three solves in a row
    with different right sides (eager work and synchronisations between the replays) give
    bitwise the answers, iteration counts and residuals of a handle that never captures."""
    _say("fgmres graphs vs eager", prec, precond)
    from oracle import learned as LN
    from paper_1306_3159_amd import PRECOND_LEARNED
    rng = np.random.default_rng(78)
    n, N = 48, 60
    q = W.rsa_positions(rng, n, N, 3.0)
    p = LN.init_params(9)
    p["w3"] = (0.05 * rng.standard_normal(64)).astype(np.float32)
    net = _net(dev, p)
    hs = []
    for mode in ("1", "0"):
        monkeypatch.setenv("BLOB_RD_GRAPHS", mode)
        S = make(dev, n, q, precision=prec, rtol=1e-8, schur_precond=PRECOND_LEARNED)
        S.precond_build(net)
        hs.append(S)
    for rep in range(3):
        f = T(1.0 + 0.5 * rng.standard_normal((n, n, n)), dev)
        (cg, lg, sg), (ce, le, se) = (S.solve_absorbing_fgmres(f, precond=precond) for S in hs)
        assert sg["rc"] == 0 and se["rc"] == 0
        assert torch.equal(cg, ce) and torch.equal(lg, le), rep
        assert sg["outer_iters"] == se["outer_iters"] and sg["rel_resid"] == se["rel_resid"]
        assert sg["vcycles"] == se["vcycles"] and sg["inner_iters_total"] == se["inner_iters_total"]
        assert sg["alg_bytes"] == pytest.approx(se["alg_bytes"], rel=1e-12)
        torch.cuda.synchronize()
    for S in hs:
        S.close()
    net.close()
