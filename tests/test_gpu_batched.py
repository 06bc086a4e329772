"""Lock-step batched launches: the CG iterations of uneven instances run in shared batched
kernels (one captured graph replayed in rounds) and give bitwise the solo results."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _instances(specs, seed0):
    out = []
    for k, (n, N, kind) in enumerate(specs):
        rng = np.random.default_rng(seed0 + k)
        q = W.rsa_positions(rng, n, N, 3.0)
        kap = W.log_uniform(rng, 1e-2, 1e2, N)
        f = 1.0 + 0.5 * rng.standard_normal((n, n, n))
        out.append((n, q, kap, kind, f))
    return out


def _handles(dev, inst, prec):
    from paper_1306_3159_amd import BlobRD
    return [BlobRD(n, torch.tensor(q, device=dev), torch.tensor(kap, device=dev), precision=prec,
                   stream=torch.cuda.Stream(dev)) for n, q, kap, kind, f in inst]


def _solo(dev, inst, prec):
    res = []
    for S, (n, q, kap, kind, f) in zip(_handles(dev, inst, prec), inst):
        ft = torch.tensor(f, device=dev)
        torch.cuda.synchronize()
        if kind == 0:
            c, st = S.solve_reactive(ft)
            res.append((c.cpu().numpy(), None, st))
        else:
            c, lam, st = S.solve_absorbing(ft)
            res.append((c.cpu().numpy(), lam.cpu().numpy(), st))
        assert st["rc"] == 0
        S.close()
    return res


def _oracle_check(inst, cs, ls, rtol=1e-8):
    """Every batched answer meets the tolerance by the oracle's own FP64 residual (so a fault
    shared by the batched and the solo path, e.g. in the spread lists, cannot pass)."""
    from oracle import exact as ex
    for (n, q, kap, kind, f), c, l in zip(inst, cs, ls):
        if kind == 0:
            r = ex.reactive_residual(c.cpu().numpy(), f, q, kap, 0.0)
        else:
            r = ex.absorbing_residual(c.cpu().numpy(), l.cpu().numpy(), f, q, 0.0)
        assert r <= rtol, (n, q.shape[0], kind, r)


@pytest.mark.parametrize("prec,max_cells", [(1, 0), (0, 0), (1, 300000)])
def test_batched_matches_solo(dev, prec, max_cells):
    """All instances in the lock-step launches (max_cells 0), or only grids up to 64^3 with the
    larger ones on their own streams meanwhile: bitwise the solo results either way."""
    _say("batched vs solo, prec", prec, "max_cells", max_cells)
    from paper_1306_3159_amd import solve_batched
    specs = [(32, 60, 0), (48, 200, 1), (64, 300, 0), (32, 20, 1), (96, 400, 1), (64, 150, 1), (48, 90, 0),
             (128, 500, 0)]
    inst = _instances(specs, 4100)
    solo = _solo(dev, inst, prec)
    Hs = _handles(dev, inst, prec)
    for rep in range(2):  # a second batched call on the same handles (fresh tables and graph)
        fs = [torch.tensor(f, device=dev) for *_, f in inst]
        cs = [torch.zeros_like(f) for f in fs]
        ls = [torch.zeros(q.shape[0], dtype=torch.float64, device=dev) if kind else None
              for _, q, _, kind, _ in inst]
        rc, stats = solve_batched(Hs, [kind for _, _, _, kind, _ in inst], fs, cs, ls, lockstep_max_cells=max_cells,
                                  threads=3 if rep else 0)
        assert rc == 0, stats
        for (c0, l0, st0), c, l, st in zip(solo, cs, ls, stats):
            assert np.array_equal(c.cpu().numpy(), c0)
            if l0 is not None:
                assert np.array_equal(l.cpu().numpy(), l0)
            assert st["outer_iters"] == st0["outer_iters"]
        if rep == 0:
            _oracle_check(inst, cs, ls)
    # the handles still solve alone afterwards
    n, q, kap, kind, f = inst[0]
    c, st = Hs[0].solve_reactive(torch.tensor(f, device=dev))
    assert np.array_equal(c.cpu().numpy(), solo[0][0])
    for S in Hs:
        S.close()


def test_batched_serves_unfit_instances_on_streams(dev):
    """A grid whose split rows are not 4-wide (x = 20) cannot join the batched kernels; it is solved
    on its own stream while the others use the lock-step launches, with the same results."""
    _say("batched with an unfit instance")
    from paper_1306_3159_amd import BlobRD, solve_batched
    rng = np.random.default_rng(4200)
    shapes = [(32, 32, 20), (32, 32, 32), (48, 48, 48)]  # [z, y, x]
    Hs, fs, ref = [], [], []
    for sh in shapes:
        q = np.column_stack([rng.uniform(0, sh[2], 12), rng.uniform(0, sh[1], 12), rng.uniform(0, sh[0], 12)])
        kap = rng.uniform(0.5, 2.0, 12)
        f = 1.0 + 0.5 * rng.standard_normal(sh)
        S = BlobRD(sh, torch.tensor(q, device=dev), torch.tensor(kap, device=dev), precision=1,
                   stream=torch.cuda.Stream(dev))
        c, st = S.solve_reactive(torch.tensor(f, device=dev))
        assert st["rc"] == 0
        ref.append(c.cpu().numpy())
        Hs.append(S)
        fs.append(torch.tensor(f, device=dev))
    cs = [torch.zeros_like(f) for f in fs]
    rc, stats = solve_batched(Hs, [0, 0, 0], fs, cs, [None, None, None])
    assert rc == 0
    for c, r in zip(cs, ref):
        assert np.array_equal(c.cpu().numpy(), r)
    for S in Hs:
        S.close()


def test_batched_with_block_solver_instances(dev):
    """Absorbing instances whose handles solve by the block FGMRES run on their own streams while
    the reactive ones share the lock-step launches; every result is bitwise the solo solve, and
    the block handles' absorbing solves are those of blob_rd_solve_absorbing_fgmres."""
    _say("batched with block-solver instances")
    from paper_1306_3159_amd import BlobRD, solve_batched, solve_streams, SOLVER_BLOCK
    specs = [(32, 60, 0), (48, 200, 1), (64, 300, 0), (32, 20, 1), (64, 150, 1), (48, 90, 0)]
    inst = _instances(specs, 4300)

    def handles():
        return [BlobRD(n, torch.tensor(q, device=dev), torch.tensor(kap, device=dev), precision=1,
                       stream=torch.cuda.Stream(dev), saddle_solver=SOLVER_BLOCK if kind else 0)
                for n, q, kap, kind, f in inst]

    Hs = handles()
    solo = []
    for S, (n, q, kap, kind, f) in zip(Hs, inst):
        ft = torch.tensor(f, device=dev)
        if kind:
            c, lam, st = S.solve_absorbing(ft)
            c2, lam2, st2 = S.solve_absorbing_fgmres(ft, precond="schur")
            assert np.array_equal(c.cpu().numpy(), c2.cpu().numpy())
            assert st["outer_iters"] == st2["outer_iters"]
            solo.append((c.cpu().numpy(), lam.cpu().numpy()))
        else:
            c, st = S.solve_reactive(ft)
            solo.append((c.cpu().numpy(), None))
        assert st["rc"] == 0 and st["rel_resid"] <= 1e-8
    for runner in ("batched", "streams"):
        fs = [torch.tensor(f, device=dev) for *_, f in inst]
        cs = [torch.zeros_like(f) for f in fs]
        ls = [torch.zeros(q.shape[0], dtype=torch.float64, device=dev) if kind else None for _, q, _, kind, _ in inst]
        kinds = [kind for _, _, _, kind, _ in inst]
        if runner == "batched":
            rc, stats = solve_batched(Hs, kinds, fs, cs, ls)
        else:
            rc, stats = solve_streams(Hs, kinds, fs, cs, ls, threads=3)
        assert rc == 0, stats
        for (c0, l0), c, l in zip(solo, cs, ls):
            assert np.array_equal(c.cpu().numpy(), c0)
            if l0 is not None:
                assert np.array_equal(l.cpu().numpy(), l0)
        if runner == "batched":
            _oracle_check(inst, cs, ls)
    for S in Hs:
        S.close()
