"""Host-side pins of the seeded input generators and of the formulas the validation sweeps use
to reduce GPU solutions (no GPU)."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import workloads as W


def test_box_suspension_margin_and_separation():
    """The box workload keeps every blob at least 3h inside each face and 3h from every other
    blob (plain distance), and is reproducible from its seed."""
    a = W.box_suspension(64, 400)
    b = W.box_suspension(64, 400)
    assert np.array_equal(a.q, b.q)
    assert a.q.min() >= 3.0 and a.q.max() <= 64 - 3.0
    d, _ = cKDTree(a.q).query(a.q, k=2)
    assert d[:, 1].min() >= 3.0


def test_rsa_minimum_image_separation():
    rng = np.random.default_rng(5)
    q = W.rsa_positions(rng, 32, 300, 3.0)
    d = q[:, None, :] - q[None, :, :]
    d -= 32.0 * np.round(d / 32.0)
    r = np.sqrt((d * d).sum(-1)) + np.eye(len(q)) * 1e9
    assert r.min() >= 3.0


def test_far_field_law_limits():
    """eq. c_r_approx: zero at r = a, c_inf at r = L/2."""
    torch = pytest.importorskip("torch")  # the sweep module imports the binding's module
    try:
        from paper_1306_3159_amd import sweeps as SW
    except ImportError:
        pytest.skip("library not built")
    L, a = 100.0, 1.255
    assert SW.far_field_law(a, L, a) == pytest.approx(0.0, abs=1e-15)
    assert SW.far_field_law(L / 2, L, a) == pytest.approx(1.0, rel=1e-14)


def test_radius_extrapolation_inverts_series():
    """eq. a_phi: a_L = a (1 + x + x^2), x = 2.84 a / L; the bisection recovers a."""
    try:
        from paper_1306_3159_amd import sweeps as SW
    except ImportError:
        pytest.skip("library not built")
    for a, L in ((1.27, 16), (1.255, 64), (0.885, 256)):
        x = 2.84 * a / L
        assert SW.radius_extrapolated(a * (1 + x + x * x), L) == pytest.approx(a, rel=1e-12)
