"""GPU parity of the Dirichlet-box path (Sec. IV.C: a box whose faces hold c = c_inf) with the
oracle, through the C ABI.

The oracle solves the lifted systems exactly (sine transform + dense N x N blob systems); the
library solves them by multigrid CG (reactive) and the block FGMRES (absorbing) to rtol 1e-10,
so solutions agree to ~1e-8 relative. Operators agree to rounding. The single-blob far field is
checked against the oracle and against eq. c_r_approx (E9; the paper's box has 100 cells per
edge, here 96 so that the multigrid coarsens to 3^3), and the negative concentration inside the
kernel of an absorbing blob (E2).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dirichlet as dr
from oracle import exact as ex

pytestmark = pytest.mark.gpu

CB = 1.7


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


def box(dev, shape, q, kappa=None, cb=CB, **kw):
    from paper_1306_3159_amd import BlobRD, BOUNDARY_DIRICHLET
    return BlobRD(shape, T(q, dev), None if kappa is None else T(kappa, dev), boundary=BOUNDARY_DIRICHLET,
                  boundary_value=cb, **kw)


def inner_blobs(rng, shape, n):
    """n blob positions (x, y, z) at least 3h inside every face of a (nz, ny, nx) box."""
    nz, ny, nx = shape
    lo = np.array([3.0, 3.0, 3.0])
    hi = np.array([nx - 3.0, ny - 3.0, nz - 3.0])
    return lo + rng.uniform(0.0, 1.0, (n, 3)) * (hi - lo)


SHAPE = (16, 24, 32)  # (nz, ny, nx): levels 32x24x16 -> 16x12x8 -> 8x6x4


def test_box_apply(dev):
    """alpha I - D L_0 (+ S kappa J) with homogeneous faces, to rounding."""
    rng = np.random.default_rng(1306_501)
    q = 0.8 * inner_blobs(rng, SHAPE, 5)  # h = 0.8
    kappa = 10 ** rng.uniform(-1, 1, 5)
    x = rng.standard_normal(SHAPE)
    S = box(dev, (SHAPE[0], SHAPE[1], SHAPE[2]), q, kappa, h=0.8, D=1.3)
    _say("box apply", SHAPE)
    y0 = H(S.apply(T(x, dev), alpha=0.3, with_blobs=False))
    ref0 = dr.apply_A0(x, 0.3, 1.3, 0.8)
    assert rel(y0, ref0) < 1e-14
    y1 = H(S.apply(T(x, dev), alpha=0.3, with_blobs=True))
    ref1 = ref0 + ex.spread(kappa * ex.interp(x, q, 0.8, 4), q, SHAPE, 0.8, 4)
    assert rel(y1, ref1) < 1e-13
    S.close()


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_box_vcycle_symmetric_and_contracting(dev, alpha):
    """The V-cycle preconditions CG, so it must be symmetric; one cycle on the box operator
    cuts the residual several times."""
    from paper_1306_3159_amd import FP64
    rng = np.random.default_rng(1306_502)
    S = box(dev, SHAPE, inner_blobs(rng, SHAPE, 2), precision=FP64)
    a, b = rng.standard_normal(SHAPE), rng.standard_normal(SHAPE)
    _say("box vcycle", SHAPE, alpha)
    Va, Vb = H(S.vcycle(T(a, dev), alpha)), H(S.vcycle(T(b, dev), alpha))
    assert abs(np.sum(Va * b) - np.sum(a * Vb)) < 1e-12 * abs(np.sum(Va * b))
    r = a - dr.apply_A0(Va, alpha)
    assert np.linalg.norm(r) < 0.2 * np.linalg.norm(a)
    S.close()


def test_box_poisson_no_blobs(dev):
    """-D L_{c_b} c = f with no blob: c = c_b + (-D L_0)^{-1} f (the sine-transform solve)."""
    from paper_1306_3159_amd import FP64
    rng = np.random.default_rng(1306_503)
    f = 1.0 + 0.5 * rng.standard_normal(SHAPE)
    S = box(dev, SHAPE, np.zeros((0, 3)), precision=FP64, rtol=1e-11)
    _say("box poisson", SHAPE)
    c, st = S.solve_reactive(T(f, dev))
    assert st["rc"] == 0, st
    ref = CB + dr.solve_A0(f, 0.0)
    assert rel(H(c), ref) < 1e-9
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_box_reactive_parity(dev, precision, alpha):
    from paper_1306_3159_amd import FP64, MIXED
    rng = np.random.default_rng(1306_504)
    N = 12
    q = inner_blobs(rng, SHAPE, N)
    kappa = 10 ** rng.uniform(-1, 2, N)
    f = 1.0 + 0.5 * rng.standard_normal(SHAPE)
    S = box(dev, SHAPE, q, kappa, precision=FP64 if precision == "fp64" else MIXED, rtol=1e-10)
    _say("box reactive", precision, alpha)
    c, st = S.solve_reactive(T(f, dev), alpha=alpha)
    assert st["rc"] == 0 and st["rel_resid"] <= 1e-10, st
    cr, _ = dr.solve_reactive_box(f, q, kappa, alpha, CB)
    assert rel(H(c), cr) < 1e-8
    assert dr.reactive_residual_box(H(c), f, q, kappa, alpha, CB) < 2e-10
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_box_ragged_rows(dev, precision):
    """Rows whose half-length is not a multiple of the vector width (nx = 20: 10 split cells)
    take the one-cell-per-thread kernels; the answer is the same."""
    from paper_1306_3159_amd import FP64, MIXED, SOLVER_BLOCK
    rng = np.random.default_rng(1306_509)
    shape = (16, 16, 20)  # (nz, ny, nx): levels 20x16x16 -> 10x8x8 -> 5x4x4 (coarsest)
    N = 6
    q = inner_blobs(rng, shape, N)
    kappa = 10 ** rng.uniform(-1, 2, N)
    f = 1.0 + 0.5 * rng.standard_normal(shape)
    prec = FP64 if precision == "fp64" else MIXED
    _say("box ragged", precision)
    S = box(dev, shape, q, kappa, precision=prec, rtol=1e-10, saddle_solver=SOLVER_BLOCK)
    c, st = S.solve_reactive(T(f, dev), alpha=0.2)
    assert st["rc"] == 0, st
    cr, _ = dr.solve_reactive_box(f, q, kappa, 0.2, CB)
    assert rel(H(c), cr) < 1e-8
    c, lam, st = S.solve_absorbing(T(f, dev))
    assert st["rc"] == 0, st
    cr, lr = dr.solve_absorbing_box(f, q, 0.0, CB)
    assert rel(H(c), cr) < 1e-8 and rel(H(lam), lr) < 1e-8
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("alpha", [0.0, 0.4])
def test_box_absorbing_parity(dev, precision, alpha):
    from paper_1306_3159_amd import FP64, MIXED, SOLVER_BLOCK
    rng = np.random.default_rng(1306_505)
    N = 12
    q = inner_blobs(rng, SHAPE, N)
    f = 1.0 + 0.5 * rng.standard_normal(SHAPE)
    S = box(dev, SHAPE, q, precision=FP64 if precision == "fp64" else MIXED, rtol=1e-10,
            saddle_solver=SOLVER_BLOCK)
    _say("box absorbing", precision, alpha)
    c, lam, st = S.solve_absorbing(T(f, dev), alpha=alpha)
    assert st["rc"] == 0 and st["rel_resid"] <= 1e-10, st
    cr, lr = dr.solve_absorbing_box(f, q, alpha, CB)
    assert rel(H(c), cr) < 1e-8
    assert rel(H(lam), lr) < 1e-8
    assert dr.absorbing_residual_box(H(c), H(lam), f, q, alpha, CB) < 2e-10
    # the explicit-options entry point solves the same lifted system
    c2, lam2, st2 = S.solve_absorbing_fgmres(T(f, dev), alpha=alpha, precond="diagonal", restart=60, rtol=1e-10)
    assert st2["rc"] == 0, st2
    assert rel(H(c2), cr) < 1e-8 and rel(H(lam2), lr) < 1e-8
    S.close()


def test_box_steps(dev):
    """Two backward-Euler steps, reactive and absorbing (warm-started), against the oracle."""
    from paper_1306_3159_amd import MIXED, SOLVER_BLOCK
    rng = np.random.default_rng(1306_506)
    N = 8
    q = inner_blobs(rng, SHAPE, N)
    kappa = 10 ** rng.uniform(-1, 2, N)
    s = 1.0 + 0.5 * rng.standard_normal(SHAPE)
    c0 = CB + 0.1 * rng.standard_normal(SHAPE)
    dt = 0.7
    Sr = box(dev, SHAPE, q, kappa, precision=MIXED, rtol=1e-10)
    Sa = box(dev, SHAPE, q, precision=MIXED, rtol=1e-10, saddle_solver=SOLVER_BLOCK)
    cr, ca = T(c0, dev), T(c0, dev)
    lam = torch.zeros(N, dtype=torch.float64, device=dev)
    xr, xa = c0.copy(), c0.copy()
    for k in range(2):
        _say("box steps", k)
        st = Sr.step(T(s, dev), cr, dt)
        assert st["rc"] == 0, st
        xr, _ = dr.solve_reactive_box(s + xr / dt, q, kappa, 1.0 / dt, CB)
        assert rel(H(cr), xr) < 1e-8
        st = Sa.step_absorbing(T(s, dev), ca, lam, dt)
        assert st["rc"] == 0, st
        xa, la = dr.solve_absorbing_box(s + xa / dt, q, 1.0 / dt, CB)
        assert rel(H(ca), xa) < 1e-8
        assert rel(H(lam), la) < 1e-8
    Sr.close()
    Sa.close()


def test_box_far_field_e9(dev):
    """E9: one absorbing blob at the centre node of a 96^3 box held at c_inf = 1, no source.
    The solution matches the oracle, and c(r) follows eq. c_r_approx,
    c(r)/c_inf ~ L/(L - 2a) (1 - a/r) with a = 1.255 h, within 1 % along an axis."""
    from paper_1306_3159_amd import MIXED, SOLVER_BLOCK
    n = 96
    q = np.array([[48.0, 48.0, 48.0]])
    S = box(dev, n, q, cb=1.0, precision=MIXED, rtol=1e-10, saddle_solver=SOLVER_BLOCK)
    _say("box far field", n)
    c, lam, st = S.solve_absorbing(torch.zeros((n, n, n), dtype=torch.float64, device=dev))
    assert st["rc"] == 0, st
    cr, lr = dr.solve_absorbing_box(np.zeros((n, n, n)), q, 0.0, 1.0)
    assert rel(H(c), cr) < 1e-8
    assert abs(float(lam[0]) - lr[0]) < 1e-8 * abs(lr[0])
    ch = H(c)
    a = 1.255
    for k in (54, 58, 64, 72, 84):
        r = k + 0.5 - 48.0
        assert ch[47, 47, k] == pytest.approx(n / (n - 2 * a) * (1 - a / r), rel=0.01)
    S.close()


def test_box_e2_negative_inside_kernel(dev):
    """E2: with J c = 0 imposed at an absorbing blob the concentration dips below zero inside
    the kernel support (the averaged value is zero while the far field is positive)."""
    from paper_1306_3159_amd import FP64, SOLVER_BLOCK
    n = 32
    q = np.array([[16.3, 15.8, 16.1]])
    S = box(dev, n, q, cb=1.0, precision=FP64, rtol=1e-10, saddle_solver=SOLVER_BLOCK)
    _say("box E2", n)
    c, lam, st = S.solve_absorbing(torch.zeros((n, n, n), dtype=torch.float64, device=dev))
    assert st["rc"] == 0, st
    ch = H(c)
    assert abs(ex.interp(ch, q, 1.0, 4)[0]) < 1e-9
    k = np.unravel_index(np.argmin(ch), ch.shape)
    assert ch[k] < 0.0
    assert np.linalg.norm(np.array([k[2], k[1], k[0]]) + 0.5 - q[0]) < 2.0
    S.close()


def test_box_errors(dev):
    from paper_1306_3159_amd import BlobRD, BlobRDError, BOUNDARY_DIRICHLET, SOLVER_SCHUR
    rng = np.random.default_rng(1306_507)
    _say("box errors")
    with pytest.raises(BlobRDError, match="3h inside"):
        box(dev, 16, np.array([[2.5, 8.0, 8.0]]))
    with pytest.raises(BlobRDError):
        BlobRD(16, T(np.array([[8.0, 8.0, 8.0]]), dev), boundary=7)
    S = box(dev, 16, inner_blobs(rng, (16, 16, 16), 3), saddle_solver=SOLVER_SCHUR)
    with pytest.raises(BlobRDError, match="saddle_solver BLOCK"):
        S.solve_absorbing(torch.ones((16, 16, 16), dtype=torch.float64, device=dev))
    with pytest.raises(BlobRDError, match="periodic"):
        S.autotune(reps=2)
    S.close()


def test_box_kernel_timing(dev):
    """A box handle times the box forms of its kernels (positive times, the periodic byte counts)."""
    from paper_1306_3159_amd import MIXED
    rng = np.random.default_rng(1306_508)
    S = box(dev, SHAPE, inner_blobs(rng, SHAPE, 3), precision=MIXED)
    _say("box kernel timing")
    n = SHAPE[0] * SHAPE[1] * SHAPE[2]
    for k in ("gs", "stencil", "restrict", "prolong", "vcycle"):
        ms, by = S.time_kernel(k, reps=3)
        assert ms > 0.0 and by > 0.0
    ms, by = S.time_kernel("gs", reps=3, cold=True)
    assert ms > 0.0 and by == pytest.approx(n * 0.5 * 4 * 3)
    S.close()


def test_box_in_batches(dev):
    """Box handles in a lock-step batch run on their own streams (the batched kernels are the
    periodic ones) and return what they return alone; the periodic member is unaffected."""
    from paper_1306_3159_amd import BlobRD, MIXED, SOLVER_BLOCK, solve_batched
    rng = np.random.default_rng(1306_510)
    shape = (32, 32, 32)
    qb = inner_blobs(rng, shape, 10)
    kb = 10 ** rng.uniform(-1, 2, 10)
    qp = rng.uniform(0, 32, (10, 3))
    kp = 10 ** rng.uniform(-1, 2, 10)
    f = 1.0 + 0.5 * rng.standard_normal(shape)
    st = [torch.cuda.Stream(dev) for _ in range(3)]
    mk = [lambda s: box(dev, 32, qb, kb, precision=MIXED, rtol=1e-10, stream=s),
          lambda s: box(dev, 32, qb, precision=MIXED, rtol=1e-10, saddle_solver=SOLVER_BLOCK, stream=s),
          lambda s: BlobRD(32, T(qp, dev), T(kp, dev), precision=MIXED, rtol=1e-10, stream=s)]
    kinds = [0, 1, 0]
    _say("box in batches")
    solo = []
    for i in range(3):
        S = mk[i](None)  # alone, on the current stream
        if kinds[i] == 0:
            c, _ = S.solve_reactive(T(f, dev))
            solo.append((H(c), None))
        else:
            c, lam, _ = S.solve_absorbing(T(f, dev))
            solo.append((H(c), H(lam)))
        S.close()
    Ss = [mk[i](st[i]) for i in range(3)]
    cs = [torch.zeros(shape, dtype=torch.float64, device=dev) for _ in range(3)]
    lams = [None, torch.zeros(10, dtype=torch.float64, device=dev), None]
    rc, stats = solve_batched(Ss, kinds, [T(f, dev)] * 3, cs, lams, lockstep_max_cells=64 ** 3)
    assert rc == 0, stats
    for i in range(3):
        assert np.array_equal(H(cs[i]), solo[i][0]), i
    assert np.array_equal(H(lams[1]), solo[1][1])
    cr, _ = dr.solve_reactive_box(f, qb, kb, 0.0, CB)
    assert rel(H(cs[0]), cr) < 1e-8
    for S in Ss:
        S.close()


@pytest.mark.parametrize("w", [3, 4])
def test_box_scaled_units_and_kernels(dev, w):
    """h, D != 1 and both kernels: the lifted solves scale like the oracle's (positions in
    physical units, at least 3h inside each face); the learned handle option falls back to the
    plain inner iteration in a box."""
    from paper_1306_3159_amd import FP64, SOLVER_BLOCK_LEARNED
    rng = np.random.default_rng(1306_511 + w)
    h, D = 0.5, 2.5
    N = 7
    q = h * inner_blobs(rng, SHAPE, N)
    kappa = 10 ** rng.uniform(-1, 2, N)
    f = 1.0 + 0.5 * rng.standard_normal(SHAPE)
    _say("box units", w)
    S = box(dev, SHAPE, q, kappa, h=h, D=D, kernel_w=w, precision=FP64, rtol=1e-10,
            saddle_solver=SOLVER_BLOCK_LEARNED)
    c, st = S.solve_reactive(T(f, dev), alpha=0.3)
    assert st["rc"] == 0, st
    cr, _ = dr.solve_reactive_box(f, q, kappa, 0.3, CB, D=D, h=h, w=w)
    assert rel(H(c), cr) < 1e-8
    c, lam, st = S.solve_absorbing(T(f, dev))
    assert st["rc"] == 0, st
    cr, lr = dr.solve_absorbing_box(f, q, 0.0, CB, D=D, h=h, w=w)
    assert rel(H(c), cr) < 1e-8 and rel(H(lam), lr) < 1e-8
    S.close()
