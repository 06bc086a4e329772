"""CPU-side checks of the C ABI: the library builds, loads and exports every
entry point that include/blob_rd.h declares. No compute call needs a GPU here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blob_rd.h")
LIB = os.path.join(ROOT, "paper_1306_3159_amd", "libblob_rd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blob_rd_[a-z_]+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared_functions()
    for must in ("blob_rd_create", "blob_rd_destroy", "blob_rd_solve_reactive", "blob_rd_solve_absorbing",
                 "blob_rd_step", "blob_rd_last_error", "blob_rd_workspace_bytes", "blob_rd_create_batch",
                 "blob_rd_solve_batch", "blob_rd_precond_set_weights", "blob_rd_precond_train_step"):
        assert must in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1306_3159_amd import build as b
        b.build()
    import torch  # noqa: F401  (shares its HIP runtime with the library)
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_sizing_and_validation(lib):
    from paper_1306_3159_amd.native import Params, load_library
    L = load_library()

    def params(nx=32, ny=32, nz=32, w=4, h=1.0, D=1.0, prec=0, N=0):
        return Params(nx, ny, nz, h, D, w, N, None, None, prec, 0, 1e-8, 0, 0, 0, None, 0, None)

    ok = L.blob_rd_workspace_bytes(ctypes.byref(params()))
    assert ok > 7 * 32 ** 3 * 8
    mixed = L.blob_rd_workspace_bytes(ctypes.byref(params(prec=1)))
    assert mixed < ok                         # FP32 multigrid levels are half the size
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(nx=6))) == 0     # too small
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(w=5))) == 0      # kernel width
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(h=0.0))) == 0
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(nx=36, ny=36, nz=36))) == 0  # coarsest 9^3 > 512
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(nx=48, ny=48, nz=48))) > 0   # 48 -> ... -> 3
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(N=5))) == 0      # blobs without positions
    assert b"coarsest" in L.blob_rd_last_error(None) or b"q is null" in L.blob_rd_last_error(None)


def test_learned_handles_reserve_their_network(lib):
    """A handle created for the learned preconditioner reserves its network and room for W
    (BLOB_RD_LEARNED_ROW_CAP pairs per blob) in the workspace; other handles do not. The
    positions are not read when sizing, so a placeholder pointer suffices here."""
    from paper_1306_3159_amd.native import Params, load_library
    L = load_library()
    fake = ctypes.c_void_p(4096)

    def params(precond=0, solver=0, boundary=0, N=100):
        p = Params(32, 32, 32, 1.0, 1.0, 4, N, fake, None, 0, precond, 1e-8, 0, 0, 0, None, 0, None)
        p.saddle_solver, p.boundary = solver, boundary
        return p

    plain = L.blob_rd_workspace_bytes(ctypes.byref(params()))
    net = L.blob_rd_net_workspace_bytes()
    for kw in (dict(precond=2), dict(solver=2)):
        extra = L.blob_rd_workspace_bytes(ctypes.byref(params(**kw))) - plain
        if kw.get("solver"):
            extra -= L.blob_rd_workspace_bytes(ctypes.byref(params(solver=1))) - plain  # the FGMRES basis
        assert extra >= net + 100 * 256 * 20
    assert L.blob_rd_workspace_bytes(ctypes.byref(params(precond=2, N=0))) == \
        L.blob_rd_workspace_bytes(ctypes.byref(params(N=0)))


def test_weight_blob_round_trip():
    """The weight blob holds the weights as bfloat16 (nearest even) and the biases as float32."""
    import numpy as np
    from oracle import learned as LN
    from paper_1306_3159_amd.native import weights_blob, blob_params, PRECOND_BLOB_BYTES
    rng = np.random.default_rng(3)
    v = rng.standard_normal(LN.n_params()).astype(np.float32)
    b = weights_blob(v)
    assert len(b) == PRECOND_BLOB_BYTES == 2 * (768 + 4096 + 64) + 4 * (64 + 64 + 1)
    back = LN.unflatten(blob_params(b))
    ref = LN.rounded(LN.unflatten(v))
    for k in LN.PARAM_ORDER:
        assert np.array_equal(back[k].astype(np.float64), ref[k]), k
    assert weights_blob(blob_params(b)) == b
