"""The Sec. IV validation sweeps on the GPU: each reduced quantity against the oracle's exact
solve of the same cell, and against the values the paper prints (tests/golden)."""
import json
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact as ex

pytestmark = pytest.mark.gpu
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def g(key):
    return GOLDEN[key]["value"]


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


@pytest.mark.parametrize("w,key", [(4, "radius_phi4_node"), (3, "radius_phi3_node")])
def test_radius_at_node(dev, w, key):
    _say("sweep radius", w)
    from paper_1306_3159_amd import sweeps as SW
    rows = SW.sweep_radius_node(dev, (32, 64), w)
    V = 32.0 ** 3
    c, _ = ex.solve_absorbing(np.full((32, 32, 32), 1.0 / V), np.array([[16.0] * 3]), 0.0, w=w)
    assert rows[0]["cbar"] == pytest.approx(float(c.mean()), rel=1e-9)
    assert rows[0]["a"] == pytest.approx(ex.radius_extrapolated(ex.radius_from_mean(c.mean(), 1 / V, V), 32),
                                         rel=1e-9)
    for r in rows:
        assert r["a"] == pytest.approx(g(key), rel=0.01)


def test_translation_and_beta(dev):
    _say("sweep translation, beta0, finite P")
    from paper_1306_3159_amd import sweeps as SW
    t4 = SW.sweep_translation(dev, 48, 4, fractions=(0.0, 0.5, 1.0))
    t3 = SW.sweep_translation(dev, 48, 3, fractions=(0.0, 0.5, 1.0))
    assert 0.5 * g("radius_variation_phi4") < t4["spread"] < 1.5 * g("radius_variation_phi4")
    assert 0.5 * g("radius_variation_phi3") < t3["spread"] < 1.5 * g("radius_variation_phi3")
    assert t4["mean"] == pytest.approx(g("radius_phi4_average"), rel=0.01)
    for r in SW.sweep_beta0_cubic(dev, (8, 16)):
        assert r["beta0"] == pytest.approx(r["fit"], rel=0.05)
    rows = SW.sweep_finite_P(dev, 16, (0.0, 1.0))
    # eq. Omega for one blob in the discrete model: Omega(P) = Omega(0) + P / (1 - phi) exactly
    phi = rows[0]["phi"]
    assert rows[1]["Omega"] - rows[0]["Omega"] == pytest.approx(1.0 / (1 - phi), rel=1e-6)


def test_reactive_convergence_small(dev):
    _say("sweep reactive convergence")
    from paper_1306_3159_amd import sweeps as SW
    rows = SW.sweep_reactive_convergence(dev, (32,))
    assert all(r["rc"] == 0 and r["rel_resid"] <= 1e-8 for r in rows)
    by = {r["Ptilde"]: r["cg_iters"] for r in rows}
    # the diffusion-limited end is the hard one (Sec. III.E, Fig. NonSaddleGMRES)
    assert by[4 * math.pi * 1e-4] > by[1.0]
