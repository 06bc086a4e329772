"""ctypes binding of libblob_rd.so, argument marshalling only.

Names follow the C ABI (include/blob_rd.h): create/destroy, solve_reactive,
solve_absorbing, step, interp, spread, apply, vcycle.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple, Union

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblob_rd.so")

FP64 = 0
MIXED = 1
PRECOND_NONE = 0
PRECOND_DIAGONAL = 1
PRECOND_LEARNED = 2
SOLVER_SCHUR = 0
SOLVER_BLOCK = 1
SOLVER_BLOCK_LEARNED = 2
BOUNDARY_PERIODIC = 0
BOUNDARY_DIRICHLET = 1

OK = 0
ENOTCONV = 1
_ERRNAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESINGULAR", -5: "ENUMERIC"}


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("h", ctypes.c_double), ("D", ctypes.c_double), ("kernel_w", ctypes.c_int32),
        ("n_blobs", ctypes.c_int64), ("q", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
        ("precision", ctypes.c_int32), ("schur_precond", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
        ("inner_max_iter", ctypes.c_int32), ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p), ("saddle_solver", ctypes.c_int32),
        ("boundary", ctypes.c_int32), ("boundary_value", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int32), ("inner_iters_total", ctypes.c_int32),
        ("vcycles", ctypes.c_int32), ("fallback", ctypes.c_int32), ("refinements", ctypes.c_int32),
        ("rel_resid", ctypes.c_double), ("seconds", ctypes.c_double), ("alg_bytes", ctypes.c_double),
    ]

    def as_dict(self, rc: int = 0) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["rc"] = rc
        return d


class SaddleOpts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int32), ("m", ctypes.c_int32), ("n", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("diag", ctypes.c_double)]


class TrainBatch(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


SADDLE_PRECONDS = {"diagonal": 0, "schur": 1, "learned": 2}


def _saddle_opts(precond="schur", m=0, n=0, restart=0, maxit=0, rtol=0.0, diag=0.0) -> SaddleOpts:
    if precond not in SADDLE_PRECONDS:
        raise ValueError(f"precond must be one of {sorted(SADDLE_PRECONDS)}")
    return SaddleOpts(SADDLE_PRECONDS[precond], int(m), int(n), int(restart), int(maxit), float(rtol), float(diag))


class BlobRDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"blob_rd error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class NotConverged(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(path)
    vp, d, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER(Params)
    S = ctypes.POINTER(Stats)
    L.blob_rd_workspace_bytes.argtypes = [P]
    L.blob_rd_workspace_bytes.restype = ctypes.c_size_t
    L.blob_rd_create.argtypes = [P, ctypes.POINTER(vp)]
    L.blob_rd_create.restype = i32
    L.blob_rd_destroy.argtypes = [vp]
    L.blob_rd_destroy.restype = i32
    L.blob_rd_last_error.argtypes = [vp]
    L.blob_rd_last_error.restype = ctypes.c_char_p
    L.blob_rd_solve_reactive.argtypes = [vp, d, vp, vp, S]
    L.blob_rd_solve_reactive.restype = i32
    L.blob_rd_solve_absorbing.argtypes = [vp, d, vp, vp, vp, S]
    L.blob_rd_solve_absorbing.restype = i32
    L.blob_rd_step.argtypes = [vp, d, vp, vp, S]
    L.blob_rd_step.restype = i32
    L.blob_rd_step_absorbing.argtypes = [vp, d, vp, vp, vp, i32, S]
    L.blob_rd_step_absorbing.restype = i32
    L.blob_rd_fgmres_workspace_bytes.argtypes = [vp, i32]
    L.blob_rd_fgmres_workspace_bytes.restype = ctypes.c_size_t
    L.blob_rd_solve_absorbing_fgmres.argtypes = [vp, d, ctypes.POINTER(SaddleOpts), vp, vp, vp, vp, ctypes.c_size_t, S]
    L.blob_rd_solve_absorbing_fgmres.restype = i32
    L.blob_rd_solve_absorbing_fgmres_noalloc.argtypes = [vp, d, ctypes.POINTER(SaddleOpts), vp, vp, vp, S]
    L.blob_rd_solve_absorbing_fgmres_noalloc.restype = i32
    L.blob_rd_saddle_precond.argtypes = [vp, d, ctypes.POINTER(SaddleOpts), vp, vp, vp, vp]
    L.blob_rd_saddle_precond.restype = i32
    L.blob_rd_interp.argtypes = [vp, vp, vp]
    L.blob_rd_interp.restype = i32
    L.blob_rd_spread.argtypes = [vp, vp, vp]
    L.blob_rd_spread.restype = i32
    L.blob_rd_apply.argtypes = [vp, d, i32, vp, vp]
    L.blob_rd_apply.restype = i32
    L.blob_rd_vcycle.argtypes = [vp, d, vp, vp]
    L.blob_rd_vcycle.restype = i32
    L.blob_rd_time_kernel.argtypes = [vp, i32, i32, ctypes.POINTER(d), ctypes.POINTER(d)]
    L.blob_rd_time_kernel.restype = i32
    L.blob_rd_tune_levels.argtypes = [vp]
    L.blob_rd_tune_levels.restype = i32
    L.blob_rd_get_tuning.argtypes = [vp, vp, i32]
    L.blob_rd_get_tuning.restype = i32
    L.blob_rd_set_tuning.argtypes = [vp, vp, i32]
    L.blob_rd_set_tuning.restype = i32
    L.blob_rd_autotune.argtypes = [vp, i32, ctypes.c_char_p, ctypes.POINTER(i32)]
    L.blob_rd_autotune.restype = i32
    L.blob_rd_net_workspace_bytes.argtypes = []
    L.blob_rd_net_workspace_bytes.restype = ctypes.c_size_t
    L.blob_rd_net_create.argtypes = [vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.blob_rd_net_destroy.argtypes = [vp]
    L.blob_rd_net_set_params.argtypes = [vp, vp]
    L.blob_rd_net_get_params.argtypes = [vp, vp]
    L.blob_rd_net_zero_grad.argtypes = [vp]
    L.blob_rd_net_get_grad.argtypes = [vp, vp]
    L.blob_rd_net_adam_step.argtypes = [vp, ctypes.c_float]
    L.blob_rd_precond_build.argtypes = [vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.blob_rd_precond_apply.argtypes = [vp, vp, vp]
    L.blob_rd_precond_csr.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp, vp, vp]
    L.blob_rd_precond_loss_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.POINTER(d)]
    L.blob_rd_schur_apply.argtypes = [vp, d, vp, vp, d]
    L.blob_rd_schur_apply_cycles.argtypes = [vp, d, vp, vp, i32]
    L.blob_rd_schur_apply_cycles.restype = i32
    L.blob_rd_solve_streams.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), d,
                                        ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32, S]
    L.blob_rd_solve_streams.restype = i32
    L.blob_rd_create_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vp)]
    L.blob_rd_create_batch.restype = i32
    L.blob_rd_destroy_batch.argtypes = [vp]
    L.blob_rd_destroy_batch.restype = i32
    L.blob_rd_batch_member.argtypes = [vp, ctypes.c_int32]
    L.blob_rd_batch_member.restype = vp
    L.blob_rd_batch_set_executor.argtypes = [vp, ctypes.c_int64, ctypes.c_int32]
    L.blob_rd_batch_set_executor.restype = i32
    L.blob_rd_solve_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), S]
    L.blob_rd_solve_batch.restype = i32
    L.blob_rd_precond_set_weights.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.blob_rd_precond_set_weights.restype = i32
    L.blob_rd_precond_get_weights.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.blob_rd_precond_get_weights.restype = i32
    L.blob_rd_precond_train_step.argtypes = [vp, ctypes.POINTER(TrainBatch), ctypes.c_float,
                                             ctypes.POINTER(ctypes.c_float)]
    L.blob_rd_precond_train_step.restype = i32
    L.blob_rd_batch_workspace_bytes.argtypes = [ctypes.c_int32]
    L.blob_rd_batch_workspace_bytes.restype = ctypes.c_size_t
    L.blob_rd_solve_batched.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), d,
                                        ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int64,
                                        ctypes.c_int32, vp, ctypes.c_size_t, vp, S]
    L.blob_rd_solve_batched.restype = i32
    L.blob_rd_coarse_bytes.argtypes = [vp, ctypes.c_int32]
    L.blob_rd_coarse_bytes.restype = ctypes.c_size_t
    L.blob_rd_coarse_build.argtypes = [vp, d, ctypes.c_int32, d, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32)]
    L.blob_rd_coarse_build.restype = i32
    L.blob_rd_coarse_clear.argtypes = [vp]
    L.blob_rd_coarse_clear.restype = i32
    L.blob_rd_coarse_apply.argtypes = [vp, vp, vp]
    L.blob_rd_coarse_apply.restype = i32
    for name in ("blob_rd_net_create", "blob_rd_net_destroy", "blob_rd_net_set_params", "blob_rd_net_get_params",
                 "blob_rd_net_zero_grad", "blob_rd_net_get_grad", "blob_rd_net_adam_step", "blob_rd_precond_build",
                 "blob_rd_precond_apply", "blob_rd_precond_csr", "blob_rd_precond_loss_grad", "blob_rd_schur_apply"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _dev_f64(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


NET_PARAMS = 5057
PRECOND_BLOB_BYTES = 10372
# the weight blob: (parameter offset, count, stored as bfloat16) in the order of the float32 vector
_BLOB_PARTS = ((0, 768, True), (768, 64, False), (832, 4096, True), (4928, 64, False), (4992, 64, True),
               (5056, 1, False))


def weights_blob(params) -> bytes:
    """The weight blob of blob_rd_precond_set_weights from a float32 parameter vector (weights
    stored as bfloat16, the form the network uses them in; biases as float32)."""
    v = torch.as_tensor(np.asarray(params, dtype=np.float32).ravel())
    assert v.numel() == NET_PARAMS
    out = b""
    for off, n, bf in _BLOB_PARTS:
        part = v[off:off + n]
        out += (part.to(torch.bfloat16).view(torch.int16).numpy().tobytes() if bf else part.numpy().tobytes())
    assert len(out) == PRECOND_BLOB_BYTES
    return out


def blob_params(blob: bytes) -> np.ndarray:
    """The float32 parameter vector held in a weight blob."""
    assert len(blob) == PRECOND_BLOB_BYTES
    out, o = np.zeros(NET_PARAMS, np.float32), 0
    for off, n, bf in _BLOB_PARTS:
        if bf:
            out[off:off + n] = torch.frombuffer(bytearray(blob[o:o + 2 * n]), dtype=torch.bfloat16).float().numpy()
            o += 2 * n
        else:
            out[off:off + n] = np.frombuffer(blob[o:o + 4 * n], dtype=np.float32)
            o += 4 * n
    return out


class Net:
    """The learned preconditioner's network (weights, Adam state, gradient) on the GPU."""

    def __init__(self, device=None, stream: Optional[torch.cuda.Stream] = None):
        L = load_library()
        self._lib = L
        self.device = torch.device("cuda:0") if device is None else device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.blob_rd_net_workspace_bytes()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = L.blob_rd_net_create(ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise BlobRDError(rc, L.blob_rd_last_error(None).decode())
        self._h = h

    def _chk(self, rc):
        if rc != OK:
            raise BlobRDError(rc, self._lib.blob_rd_last_error(None).decode())

    def set_params(self, p: torch.Tensor):
        p = p.to(device=self.device, dtype=torch.float32).contiguous()
        assert p.numel() == NET_PARAMS
        self._chk(self._lib.blob_rd_net_set_params(self._h, _ptr(p)))

    def get_params(self) -> torch.Tensor:
        out = torch.empty(NET_PARAMS, dtype=torch.float32, device=self.device)
        self._chk(self._lib.blob_rd_net_get_params(self._h, _ptr(out)))
        return out

    def zero_grad(self):
        self._chk(self._lib.blob_rd_net_zero_grad(self._h))

    def get_grad(self) -> torch.Tensor:
        out = torch.empty(NET_PARAMS, dtype=torch.float32, device=self.device)
        self._chk(self._lib.blob_rd_net_get_grad(self._h, _ptr(out)))
        return out

    def adam_step(self, lr: float):
        self._chk(self._lib.blob_rd_net_adam_step(self._h, ctypes.c_float(lr)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.blob_rd_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BlobRD:
    """A blob configuration on a periodic grid, or in a box whose faces hold c = boundary_value
    (boundary=BOUNDARY_DIRICHLET), wrapping a blob_rd handle.

    Grid tensors are float64 CUDA tensors of shape (nz, ny, nx); q is (N, 3)
    float64 (x, y, z) and kappa (N,) float64 on the same device.
    """

    def __init__(self, shape: Union[int, Sequence[int]], q: torch.Tensor, kappa: Optional[torch.Tensor] = None,
                 h: float = 1.0, D: float = 1.0, kernel_w: int = 4, precision: int = FP64,
                 schur_precond: int = PRECOND_NONE, rtol: float = 1e-8, max_iter: int = 0,
                 gmres_restart: int = 0, inner_max_iter: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 saddle_solver: int = 0, boundary: int = 0, boundary_value: float = 0.0):
        L = load_library()
        if isinstance(shape, int):
            shape = (shape, shape, shape)
        self.shape = tuple(int(s) for s in shape)          # (nz, ny, nx)
        nz, ny, nx = self.shape
        self.device = q.device
        N = int(q.shape[0])
        self.N = N
        if N > 0:
            _dev_f64(q, (N, 3), "q")
        if kappa is not None:
            _dev_f64(kappa, (N,), "kappa")
        self.stream = stream if stream is not None else torch.cuda.current_stream(q.device)
        self._q, self._kappa = q, kappa
        p = Params(nx, ny, nz, float(h), float(D), int(kernel_w), N, q.data_ptr() if N > 0 else None,
                   None if kappa is None else kappa.data_ptr(), int(precision), int(schur_precond),
                   float(rtol), int(max_iter), int(gmres_restart), int(inner_max_iter), None, 0,
                   ctypes.c_void_p(self.stream.cuda_stream), int(saddle_solver), int(boundary),
                   float(boundary_value))
        nbytes = L.blob_rd_workspace_bytes(ctypes.byref(p))
        if nbytes == 0:
            raise BlobRDError(-1, L.blob_rd_last_error(None).decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=q.device)
        p.workspace = self.workspace.data_ptr()
        p.workspace_bytes = nbytes
        self.params = p
        h_ = ctypes.c_void_p()
        with torch.cuda.device(q.device):
            rc = L.blob_rd_create(ctypes.byref(p), ctypes.byref(h_))
        if rc != OK:
            raise BlobRDError(rc, L.blob_rd_last_error(None).decode())
        self._h = h_
        self._lib = L

    # -- helpers -------------------------------------------------------------
    def _check(self, rc: int, st: Optional[Stats] = None, allow_notconv: bool = True) -> dict:
        if rc < 0:
            raise BlobRDError(rc, self._lib.blob_rd_last_error(self._h).decode())
        out = st.as_dict(rc) if st is not None else {"rc": rc}
        if rc == ENOTCONV and not allow_notconv:
            raise NotConverged(str(out))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.blob_rd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _grid(self, t, name):
        return _dev_f64(t, self.shape, name)

    def _nvec(self, t, name):
        return _dev_f64(t, (self.N,), name)

    def _new_grid(self):
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    # -- solves ------------------------------------------------------------------
    def solve_reactive(self, f: torch.Tensor, c: Optional[torch.Tensor] = None, alpha: float = 0.0
                       ) -> Tuple[torch.Tensor, dict]:
        """(alpha I - D L + S kappa J) c = f; c is the initial guess (zeros if None)."""
        self._grid(f, "f")
        c = self._new_grid() if c is None else self._grid(c, "c")
        st = Stats()
        rc = self._lib.blob_rd_solve_reactive(self._h, float(alpha), _ptr(f), _ptr(c), ctypes.byref(st))
        return c, self._check(rc, st)

    def solve_absorbing(self, f: torch.Tensor, alpha: float = 0.0, c: Optional[torch.Tensor] = None,
                        lam: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor, dict]:
        """[alpha I - D L, S; J, 0][c; lam] = [f; 0]."""
        self._grid(f, "f")
        c = self._new_grid() if c is None else self._grid(c, "c")
        lam = torch.zeros(self.N, dtype=torch.float64, device=self.device) if lam is None else self._nvec(lam, "lam")
        st = Stats()
        rc = self._lib.blob_rd_solve_absorbing(self._h, float(alpha), _ptr(f), _ptr(c), _ptr(lam), ctypes.byref(st))
        return c, lam, self._check(rc, st)

    def step(self, f: torch.Tensor, c: torch.Tensor, dt: float) -> dict:
        """One backward-Euler step; c holds c^n on entry and c^{n+1} on exit."""
        self._grid(f, "f")
        self._grid(c, "c")
        st = Stats()
        rc = self._lib.blob_rd_step(self._h, float(dt), _ptr(f), _ptr(c), ctypes.byref(st))
        return self._check(rc, st)

    def step_absorbing(self, f: torch.Tensor, c: torch.Tensor, lam: torch.Tensor, dt: float, warm: bool = True
                       ) -> dict:
        """One backward-Euler step of an absorbing suspension; c holds c^n on entry and c^{n+1}
        on exit, lam the sink strengths (with warm, its entry values start GMRES)."""
        self._grid(f, "f")
        self._grid(c, "c")
        self._nvec(lam, "lam")
        st = Stats()
        rc = self._lib.blob_rd_step_absorbing(self._h, float(dt), _ptr(f), _ptr(c), _ptr(lam), int(bool(warm)),
                                              ctypes.byref(st))
        return self._check(rc, st)

    def solve_absorbing_fgmres(self, f: torch.Tensor, alpha: float = 0.0, precond: str = "schur", m: int = 0,
                               n: int = 0, restart: int = 0, maxit: int = 0, rtol: float = 0.0, diag: float = 0.0
                               ) -> Tuple[torch.Tensor, torch.Tensor, dict]:
        """The paper's own saddle solver: flexible GMRES on [alpha I - D L, S; J, 0][c; lam] = [f; 0]
        with the diagonal or approximate-Schur preconditioner (m inner iterations, n cycles)."""
        self._grid(f, "f")
        o = _saddle_opts(precond, m, n, restart, maxit, rtol, diag)
        nbytes = int(self._lib.blob_rd_fgmres_workspace_bytes(self._h, o.restart))
        if nbytes == 0:
            raise ValueError("FGMRES restart length out of range")
        if getattr(self, "_fg_ws", None) is None or self._fg_ws.numel() < nbytes:
            self._fg_ws = None
            self._fg_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        c = self._new_grid()
        lam = torch.zeros(self.N, dtype=torch.float64, device=self.device)
        st = Stats()
        rc = self._lib.blob_rd_solve_absorbing_fgmres(self._h, float(alpha), ctypes.byref(o), _ptr(f), _ptr(c),
                                                      _ptr(lam), _ptr(self._fg_ws), nbytes, ctypes.byref(st))
        return c, lam, self._check(rc, st)

    def saddle_precond(self, vg: torch.Tensor, vf: torch.Tensor, alpha: float = 0.0, precond: str = "schur",
                       m: int = 0, n: int = 0, diag: float = 0.0) -> Tuple[torch.Tensor, torch.Tensor]:
        """One application of the paper's saddle-point preconditioner to [vg; vf]."""
        self._grid(vg, "vg")
        self._nvec(vf, "vf")
        o = _saddle_opts(precond, m, n, 0, 0, 0.0, diag)
        zg = self._new_grid()
        zl = torch.zeros(self.N, dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_saddle_precond(self._h, float(alpha), ctypes.byref(o), _ptr(vg), _ptr(vf),
                                                     _ptr(zg), _ptr(zl)))
        return zg, zl

    # -- operators --------------------------------------------------------------
    def interp(self, c: torch.Tensor) -> torch.Tensor:
        self._grid(c, "c")
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_interp(self._h, _ptr(c), _ptr(out)))
        return out

    def spread(self, lam: torch.Tensor) -> torch.Tensor:
        out = self._new_grid()
        self._check(self._lib.blob_rd_spread(self._h, _ptr(lam), _ptr(out)))
        return out

    def apply(self, x: torch.Tensor, alpha: float = 0.0, with_blobs: bool = True) -> torch.Tensor:
        self._grid(x, "x")
        y = self._new_grid()
        self._check(self._lib.blob_rd_apply(self._h, float(alpha), int(bool(with_blobs)), _ptr(x), _ptr(y)))
        return y

    def vcycle(self, r: torch.Tensor, alpha: float = 0.0) -> torch.Tensor:
        self._grid(r, "r")
        z = self._new_grid()
        self._check(self._lib.blob_rd_vcycle(self._h, float(alpha), _ptr(r), _ptr(z)))
        return z

    # -- measurement ------------------------------------------------------------
    KERNELS = {"gs": 0, "stencil": 1, "restrict": 2, "prolong": 3, "vcycle": 4, "stream": 5, "stencil_plain": 6}

    def time_kernel(self, kernel: str, reps: int = 50, cold: bool = False) -> Tuple[float, float]:
        """Mean ms per launch (HIP events on this handle's stream) and algorithmic bytes per launch.
        cold=True evicts the last-level cache before each launch."""
        ms, by = ctypes.c_double(), ctypes.c_double()
        kid = self.KERNELS[kernel] | (256 if cold else 0)
        self._check(self._lib.blob_rd_time_kernel(self._h, kid, int(reps), ctypes.byref(ms), ctypes.byref(by)))
        return ms.value, by.value

    # -- launch-shape tuning -----------------------------------------------------
    TUNE_KINDS = ("gs", "resid", "restrict", "prolong")

    def get_tuning(self) -> np.ndarray:
        """Work-group size per (level, kernel) as a (levels, 4) int32 array."""
        nl = self._lib.blob_rd_tune_levels(self._h)
        self._check(min(nl, 0))
        t = np.zeros(max(nl, 1) * 4, dtype=np.int32)
        self._check(self._lib.blob_rd_get_tuning(self._h, t.ctypes.data_as(ctypes.c_void_p), t.size))
        return t[:nl * 4].reshape(nl, 4)

    def set_tuning(self, table) -> None:
        t = np.ascontiguousarray(table, dtype=np.int32).ravel()
        self._check(self._lib.blob_rd_set_tuning(self._h, t.ctypes.data_as(ctypes.c_void_p), t.size))

    def autotune(self, reps: int = 20, cache: Optional[str] = None) -> int:
        """Time candidate work-group sizes and keep the fastest; returns the number of levels timed
        (levels found in the JSON cache file are not timed)."""
        n = ctypes.c_int32()
        self._check(self._lib.blob_rd_autotune(self._h, int(reps), None if cache is None else cache.encode(),
                                               ctypes.byref(n)))
        return n.value

    # -- learned preconditioner -------------------------------------------------
    def precond_build(self, net: "Net") -> int:
        """Pair list + W from the network; returns nnz. The buffer is kept by this object."""
        need = ctypes.c_size_t()
        self._check(self._lib.blob_rd_precond_build(self._h, net._h, None, 0, ctypes.byref(need)))
        self._pbuf = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=self.device)
        self._check(self._lib.blob_rd_precond_build(self._h, net._h, ctypes.c_void_p(self._pbuf.data_ptr()),
                                                    self._pbuf.numel(), ctypes.byref(need)))
        nnz = ctypes.c_int64()
        self._check(self._lib.blob_rd_precond_csr(self._h, ctypes.byref(nnz), None, None, None))
        return int(nnz.value)

    def precond_set_weights(self, blob: bytes) -> None:
        """Set this handle's own network from a weight blob and build W (handles created with
        schur_precond=PRECOND_LEARNED or saddle_solver=SOLVER_BLOCK_LEARNED)."""
        self._check(self._lib.blob_rd_precond_set_weights(self._h, bytes(blob), len(blob)))

    def precond_get_weights(self) -> bytes:
        buf = ctypes.create_string_buffer(PRECOND_BLOB_BYTES)
        self._check(self._lib.blob_rd_precond_get_weights(self._h, buf, PRECOND_BLOB_BYTES))
        return buf.raw

    def precond_train_step(self, X: torch.Tensor, Y: torch.Tensor, lr: float) -> float:
        """One loss/gradient/Adam step of this handle's own network on sample pairs (rows of X,
        Y); W follows the new weights. Returns the loss before the step."""
        X = _dev_f64(X.contiguous(), (X.shape[0], self.N), "X")
        Y = _dev_f64(Y.contiguous(), (X.shape[0], self.N), "Y")
        b = TrainBatch(int(X.shape[0]), X.data_ptr(), Y.data_ptr())
        loss = ctypes.c_float()
        self._check(self._lib.blob_rd_precond_train_step(self._h, ctypes.byref(b), ctypes.c_float(lr),
                                                         ctypes.byref(loss)))
        return float(loss.value)

    def precond_csr(self):
        nnz = ctypes.c_int64()
        self._check(self._lib.blob_rd_precond_csr(self._h, ctypes.byref(nnz), None, None, None))
        ptr = torch.empty(self.N + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(int(nnz.value), dtype=torch.int32, device=self.device)
        val = torch.empty(int(nnz.value), dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_precond_csr(self._h, ctypes.byref(nnz), _ptr(ptr), _ptr(col), _ptr(val)))
        return ptr, col, val

    def precond_apply(self, r: torch.Tensor) -> torch.Tensor:
        z = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_precond_apply(self._h, _ptr(r), _ptr(z)))
        return z

    def precond_loss_grad(self, net: "Net", X: torch.Tensor, Y: torch.Tensor) -> float:
        X = X.contiguous()
        Y = Y.contiguous()
        S = int(X.shape[0])
        loss = ctypes.c_double()
        self._check(self._lib.blob_rd_precond_loss_grad(self._h, net._h, _ptr(X), _ptr(Y), S, ctypes.byref(loss)))
        return loss.value

    def schur_apply(self, x: torch.Tensor, alpha: float = 0.0, inner_rtol: float = 1e-10) -> torch.Tensor:
        y = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_schur_apply(self._h, float(alpha), _ptr(x.contiguous()), _ptr(y),
                                                  float(inner_rtol)))
        return y

    def coarse_build(self, alpha: float = 0.0, m2max: int = 3, inner_rtol: float = 1e-6) -> int:
        """Build the Fourier coarse level of the Schur preconditioner for alpha (wave vectors
        0 < |m|^2 <= m2max) in a buffer this object keeps; returns the number of columns K."""
        nbytes = int(self._lib.blob_rd_coarse_bytes(self._h, int(m2max)))
        if nbytes == 0:
            raise BlobRDError(-1, self._lib.blob_rd_last_error(self._h).decode())
        buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        k = ctypes.c_int32()
        self._check(self._lib.blob_rd_coarse_build(self._h, float(alpha), int(m2max), float(inner_rtol), _ptr(buf),
                                                   nbytes, ctypes.byref(k)))
        self._coarse_buf = buf
        return int(k.value)

    def coarse_clear(self) -> None:
        self._check(self._lib.blob_rd_coarse_clear(self._h))
        self._coarse_buf = None

    def coarse_apply(self, r: torch.Tensor) -> torch.Tensor:
        """z = B r, the two-level Schur preconditioner of the built coarse level."""
        self._nvec(r, "r")
        z = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_coarse_apply(self._h, _ptr(r), _ptr(z)))
        return z

    def schur_apply_cycles(self, x: torch.Tensor, alpha: float = 0.0, cycles: int = 1) -> torch.Tensor:
        """y = P J A_n^{-1} S P x with n multigrid cycles (the approximate-Schur operator)."""
        self._nvec(x, "x")
        y = torch.empty(self.N, dtype=torch.float64, device=self.device)
        self._check(self._lib.blob_rd_schur_apply_cycles(self._h, float(alpha), _ptr(x), _ptr(y), int(cycles)))
        return y


def solve_streams(solvers: Sequence["BlobRD"], kinds: Sequence[int], fs, cs, lams, alpha: float = 0.0,
                  threads: int = 8):
    """Solve independent instances concurrently (each solver should own its own stream).
    kinds: 0 reactive, 1 absorbing. Returns (rc, list of stats dicts)."""
    L = load_library()
    n = len(solvers)
    H = (ctypes.c_void_p * n)(*[s._h for s in solvers])
    K = (ctypes.c_int32 * n)(*[int(k) for k in kinds])
    F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    C = (ctypes.c_void_p * n)(*[c.data_ptr() for c in cs])
    Lm = (ctypes.c_void_p * n)(*[(l.data_ptr() if l is not None else None) for l in lams])
    st = (Stats * n)()
    rc = L.blob_rd_solve_streams(H, n, K, float(alpha), F, C, Lm, int(threads), st)
    if rc < 0:
        raise BlobRDError(rc, L.blob_rd_last_error(None).decode())
    return rc, [st[i].as_dict(rc) for i in range(n)]


def solve_batched(solvers: Sequence["BlobRD"], kinds: Sequence[int], fs, cs, lams, alpha: float = 0.0,
                  stream: Optional[torch.cuda.Stream] = None, lockstep_max_cells: int = 0, threads: int = 0):
    """Lock-step batched solve: the CG iterations of the member instances (grids of at most
    lockstep_max_cells cells, 0 = all that fit) run in shared batched launches (one captured graph
    replayed in rounds); the others run on their own streams meanwhile, at most `threads` at a time
    (0 = all). kinds: 0 reactive, 1 absorbing. Returns (rc, stats)."""
    L = load_library()
    n = len(solvers)
    dev = solvers[0].device
    H = (ctypes.c_void_p * n)(*[s._h for s in solvers])
    K = (ctypes.c_int32 * n)(*[int(k) for k in kinds])
    F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    C = (ctypes.c_void_p * n)(*[c.data_ptr() for c in cs])
    Lm = (ctypes.c_void_p * n)(*[(l.data_ptr() if l is not None else None) for l in lams])
    st = (Stats * n)()
    nbytes = int(L.blob_rd_batch_workspace_bytes(n))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    strm = stream if stream is not None else torch.cuda.current_stream(dev)
    torch.cuda.synchronize(dev)
    rc = L.blob_rd_solve_batched(H, n, K, float(alpha), F, C, Lm, int(lockstep_max_cells), int(threads),
                                 ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.c_void_p(strm.cuda_stream), st)
    if rc < 0:
        raise BlobRDError(rc, L.blob_rd_last_error(None).decode())
    return rc, [st[i].as_dict(rc) for i in range(n)]


class _Member(BlobRD):
    """A member handle of a Batch (owned by the batch: closing it does nothing)."""

    def __init__(self, lib, h, shape, N, device, stream):
        self._lib, self._h, self.shape, self.N, self.device, self.stream = lib, h, shape, N, device, stream

    def close(self):
        self._h = None


class Batch:
    """A blob_rd batch handle (blob_rd_create_batch): instances with their own grids, blobs,
    precisions, solvers and streams, solved together by blob_rd_solve_batch.

    specs: one dict per instance with the BlobRD keyword arguments (shape, q, kappa, precision,
    saddle_solver, ...) and `kind` (0 reactive, 1 absorbing); each instance gets its own stream."""

    def __init__(self, specs: Sequence[dict], lockstep_max_cells: Optional[int] = None, threads: Optional[int] = None):
        L = load_library()
        self._lib = L
        n = len(specs)
        params = (Params * n)()
        self._keep, self.members, self.kinds = [], [], []
        for i, sp in enumerate(specs):
            sp = dict(sp)
            kind = int(sp.pop("kind"))
            shape = sp.pop("shape")
            shape = (shape,) * 3 if isinstance(shape, int) else tuple(int(v) for v in shape)
            q = sp.pop("q")
            kappa = sp.pop("kappa", None)
            N = int(q.shape[0])
            if N > 0:
                _dev_f64(q, (N, 3), "q")
            if kappa is not None:
                _dev_f64(kappa, (N,), "kappa")
            stream = sp.pop("stream", None) or torch.cuda.Stream(q.device)
            a = dict(h=1.0, D=1.0, kernel_w=4, precision=FP64, schur_precond=PRECOND_NONE, rtol=1e-8, max_iter=0,
                     gmres_restart=0, inner_max_iter=0, saddle_solver=0, boundary=0, boundary_value=0.0)
            unknown = set(sp) - set(a)
            if unknown:
                raise ValueError(f"unknown instance options {sorted(unknown)}")
            a.update(sp)
            nz, ny, nx = shape
            p = Params(nx, ny, nz, float(a["h"]), float(a["D"]), int(a["kernel_w"]), N,
                       q.data_ptr() if N > 0 else None, None if kappa is None else kappa.data_ptr(),
                       int(a["precision"]), int(a["schur_precond"]), float(a["rtol"]), int(a["max_iter"]),
                       int(a["gmres_restart"]), int(a["inner_max_iter"]), None, 0,
                       ctypes.c_void_p(stream.cuda_stream), int(a["saddle_solver"]), int(a["boundary"]),
                       float(a["boundary_value"]))
            nbytes = int(L.blob_rd_workspace_bytes(ctypes.byref(p)))
            if nbytes == 0:
                raise BlobRDError(-1, L.blob_rd_last_error(None).decode())
            if i == 0:
                nbytes += int(L.blob_rd_batch_workspace_bytes(n))
            ws = torch.empty(nbytes, dtype=torch.uint8, device=q.device)
            p.workspace, p.workspace_bytes = ws.data_ptr(), nbytes
            params[i] = p
            self._keep += [ws, q, kappa, stream]
            self.members.append((shape, N, q.device, stream))
            self.kinds.append(kind)
        K = (ctypes.c_int32 * n)(*self.kinds)
        h = ctypes.c_void_p()
        rc = L.blob_rd_create_batch(params, n, K, ctypes.byref(h))
        if rc != OK:
            raise BlobRDError(rc, L.blob_rd_last_error(None).decode())
        self._h = h
        self.members = [_Member(L, L.blob_rd_batch_member(h, i), shape, N, dev, st)
                        for i, (shape, N, dev, st) in enumerate(self.members)]
        if lockstep_max_cells is not None or threads is not None:
            rc = L.blob_rd_batch_set_executor(h, int(64 ** 3 if lockstep_max_cells is None else lockstep_max_cells),
                                              int(8 if threads is None else threads))
            if rc != OK:
                raise BlobRDError(rc, L.blob_rd_last_error(None).decode())

    def solve(self, fs, cs, lams):
        """blob_rd_solve_batch: fs, cs grid tensors per member (cs: initial guess of reactive members,
        solution out), lams multiplier tensors of absorbing members (None for reactive ones)."""
        n = len(self.members)
        F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        C = (ctypes.c_void_p * n)(*[c.data_ptr() for c in cs])
        Lm = (ctypes.c_void_p * n)(*[(l.data_ptr() if l is not None else None) for l in lams])
        st = (Stats * n)()
        torch.cuda.synchronize()
        rc = self._lib.blob_rd_solve_batch(self._h, F, C, Lm, st)
        if rc < 0:
            raise BlobRDError(rc, self._lib.blob_rd_last_error(None).decode())
        return rc, [st[i].as_dict(rc) for i in range(n)]

    def close(self):
        if getattr(self, "_h", None):
            for m in self.members:
                m.close()
            self._lib.blob_rd_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
