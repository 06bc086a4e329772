"""Launch-shape tuning: any work-group table gives bitwise the same solves, the
autotuner picks valid sizes and its JSON cache is reused across handles."""
import json
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W
from paper_1306_3159_amd.native import BlobRDError

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


def _handle(dev, n, q, prec):
    from paper_1306_3159_amd import BlobRD
    return BlobRD(n, torch.tensor(q, device=dev), precision=prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_any_table_is_bitwise_identical(dev, prec):
    # 96^3: per-level launches on 96/48/24 (FP32) and a non-power-of-two LDS tail below
    _say("tuning tables, prec", prec)
    rng = np.random.default_rng(3301)
    n = 96
    q = W.rsa_positions(rng, n, 300, 3.0)
    f = torch.tensor(1.0 + 0.5 * rng.standard_normal((n, n, n)), device=dev)
    S = _handle(dev, n, q, prec)
    base = S.get_tuning()
    assert base.shape[1] == 4 and base.shape[0] >= 1
    assert np.all(base == 256)
    c0, l0, st0 = S.solve_absorbing(f)
    assert st0["rc"] == 0
    c0, l0 = c0.cpu().numpy(), l0.cpu().numpy()
    tables = [np.full_like(base, 64), np.full_like(base, 512),
              rng.choice([64, 128, 256, 512], size=base.shape).astype(np.int32)]
    for t in tables:
        S.set_tuning(t)
        assert np.array_equal(S.get_tuning(), t)
        c, lam, st = S.solve_absorbing(f)
        assert st["rc"] == 0
        assert np.array_equal(c.cpu().numpy(), c0)
        assert np.array_equal(lam.cpu().numpy(), l0)
    S.close()


def test_autotune_and_cache(dev, tmp_path):
    _say("autotune + cache")
    rng = np.random.default_rng(3302)
    n = 128
    q = W.rsa_positions(rng, n, 500, 3.0)
    f = torch.ones((n, n, n), dtype=torch.float64, device=dev)
    cache = str(tmp_path / "tune.json")
    S = _handle(dev, n, q, 1)
    ref, lref, _ = S.solve_absorbing(f)
    ref, lref = ref.cpu().numpy(), lref.cpu().numpy()
    nl = S.get_tuning().shape[0]
    assert S.autotune(reps=3, cache=cache) == nl
    t1 = S.get_tuning()
    assert np.isin(t1, [64, 128, 256, 512]).all()
    entries = json.load(open(cache))
    assert len(entries) == 4 * nl
    assert all(k.split("|")[1] == "f32" for k in entries)
    c, lam, st = S.solve_absorbing(f)
    assert st["rc"] == 0 and np.array_equal(c.cpu().numpy(), ref) and np.array_equal(lam.cpu().numpy(), lref)
    S.close()
    # a second handle of the same size reads every level from the cache
    S2 = _handle(dev, n, q, 1)
    assert S2.autotune(reps=3, cache=cache) == 0
    assert np.array_equal(S2.get_tuning(), t1)
    S2.close()
    # a 64^3 handle shares the 64^3 and 32^3 level entries
    S3 = _handle(dev, 64, q[:50] * 0.5, 1)
    assert S3.autotune(reps=3, cache=cache) == 0
    S3.close()


def test_tuning_rejects_bad_tables(dev):
    _say("tuning validation")
    rng = np.random.default_rng(3303)
    S = _handle(dev, 64, W.rsa_positions(rng, 64, 30, 3.0), 1)
    t = S.get_tuning()
    bad = t.copy()
    bad[0, 0] = 100
    with pytest.raises(BlobRDError):
        S.set_tuning(bad)
    assert np.array_equal(S.get_tuning(), t)
    with pytest.raises(BlobRDError):
        S.set_tuning(t.ravel()[:-1])
    S.close()
