"""Thin Python binding of the lbsep C ABI (include/lbsep.h).

Argument marshalling only: every step of the solver runs in the HIP library
``liblbsep.so`` built next to this file. torch provides the device workspace
(one uint8 tensor) and the stream; nothing here computes any part of the
method, and there is no fallback: if the library is missing, importing a
channel raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

import numpy as np
import torch  # noqa: F401  (load torch's HIP runtime first; the library binds to it)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbsep.so")

OK, EINVAL, ESIZE, EDEVICE, ENONFINITE, ERANGE = 0, -1, -2, -3, -4, -5
PERIODIC_X, PERIODIC_Y, MFP_OFF, BGK_TEST = 0x1, 0x2, 0x4, 0x8
TILE_AUTO, TILE_SPLIT, TILE_NODE = 0, 1, 2
F64, F32, F16 = 0, 1, 2
_DTYPES = {"f64": F64, "f32": F32, "f16": F16}
_TORCH = {F64: torch.float64, F32: torch.float32, F16: torch.float16}


class LbsepError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbsep error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    """Mirror of ``lbsep_params``."""
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32),
        ("m_a", c_double), ("m_b", c_double),
        ("cl_in", c_double), ("cl_out", c_double),
        ("theta", c_double), ("kn_out", c_double),
        ("dbb_r", c_double), ("accom", c_double), ("tau_bgk", c_double),
        ("flags", c_uint32), ("dtype", c_int32), ("hist_cap", c_int32), ("tile_mode", c_int32),
        ("tile_rows", c_int32), ("fused_steps", c_int32),
    ]


_lib = None


def load():
    """Load liblbsep.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = POINTER(Params)
    sig = {
        "lbsep_workspace_bytes": (c_size_t, [P]),
        "lbsep_state_bytes": (c_size_t, [P]),
        "lbsep_init": (c_int, [P, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
        "lbsep_step": (c_int, [c_void_p, c_int64]),
        "lbsep_time": (c_int64, [c_void_p]),
        "lbsep_read_cl": (c_int, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int32),
                                  POINTER(c_double)]),
        "lbsep_read_column_sums": (c_int, [c_void_p, POINTER(c_double)]),
        "lbsep_read_history": (c_int, [c_void_p, c_int64, c_int64, POINTER(c_double)]),
        "lbsep_read_moments": (c_int, [c_void_p, POINTER(c_double)]),
        "lbsep_read_volume_flow": (c_int, [c_void_p, POINTER(c_double)]),
        "lbsep_get_state": (c_int, [c_void_p, c_void_p]),
        "lbsep_set_state": (c_int, [c_void_p, c_void_p, c_int64]),
        "lbsep_get_populations": (c_int, [c_void_p, c_void_p]),
        "lbsep_get_post_collision": (c_int, [c_void_p, c_void_p]),
        "lbsep_step_record": (c_int, [c_void_p, c_void_p, c_void_p]),
        "lbsep_set_populations": (c_int, [c_void_p, c_void_p, c_int64]),
        "lbsep_dbb_r_from_cm": (c_double, [c_double, c_double, c_double, c_double]),
        "lbsep_wall_function": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p]),
        "lbsep_destroy": (None, [c_void_p]),
        "lbsep_last_error": (c_char_p, []),
        "lbsep_batch_workspace_bytes": (c_size_t, [POINTER(c_void_p), c_int32]),
        "lbsep_batch_create": (c_int, [POINTER(c_void_p), c_int32, c_void_p, c_size_t, POINTER(c_void_p)]),
        "lbsep_batch_step": (c_int, [c_void_p, c_int64]),
        "lbsep_batch_capture": (c_int, [c_void_p, c_int64]),
        "lbsep_batch_size": (c_int32, [c_void_p]),
        "lbsep_batch_destroy": (None, [c_void_p]),
        "lbsep_adjoint_workspace_bytes": (c_size_t, [P]),
        "lbsep_adjoint_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_size_t]),
        "lbsep_adjoint_step_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "lbsep_adjoint_seed_cl": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
        "lbsep_adjoint_initial": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return load().lbsep_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise LbsepError(rc, last_error())


def make_params(nx, ny, m_a, m_b, cl_in, cl_out, theta, kn_out, dbb_r, accom=1.0, tau_bgk=0.0,
                flags=0, dtype="f64", hist_cap=4096, tile_mode=TILE_AUTO, tile_rows=0, fused_steps=0) -> Params:
    return Params(int(nx), int(ny), float(m_a), float(m_b), float(cl_in), float(cl_out), float(theta),
                  float(kn_out), float(dbb_r), float(accom), float(tau_bgk), int(flags),
                  _DTYPES[dtype] if isinstance(dtype, str) else int(dtype), int(hist_cap), int(tile_mode),
                  int(tile_rows), int(fused_steps))


def workspace_bytes(params: Params) -> int:
    n = load().lbsep_workspace_bytes(byref(params))
    if n == 0:
        raise LbsepError(EINVAL, last_error())
    return n


def dbb_r_from_cm(c_m: float, m_a: float, m_b: float, cl: float) -> float:
    return load().lbsep_dbb_r_from_cm(c_m, m_a, m_b, cl)


def wall_function(alpha: torch.Tensor, dtype="f64", table=True):
    """(psi, psi'/2) of the device wall function for a float64 cuda tensor
    (FP64: as channels above 2^17 nodes evaluate it if `table`, else as smaller
    ones do)."""
    if alpha.dtype != torch.float64 or alpha.device.type != "cuda":
        raise ValueError("alpha must be a float64 cuda tensor")
    a = alpha.contiguous()
    psi = torch.empty_like(a)
    h = torch.empty_like(a)
    code = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    _check(load().lbsep_wall_function(c_void_p(a.data_ptr()), c_void_p(psi.data_ptr()), c_void_p(h.data_ptr()),
                                      a.numel(), code, 1 if table else 0,
                                      c_void_p(torch.cuda.current_stream().cuda_stream)))
    return psi, h


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


class Channel:
    """One channel on one GPU: owns its workspace tensor and the library handle."""

    def __init__(self, params: Params, device="cuda", stream=None):
        L = load()
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        self.dtype = _TORCH[params.dtype]
        self.device = torch.device(device)
        nbytes = workspace_bytes(params)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if self.stream != torch.cuda.current_stream(self.device):
            raw.record_stream(self.stream)  # the allocator must not recycle it under the channel's work
        h = c_void_p()
        _check(L.lbsep_init(byref(params), c_void_p(self.ws.data_ptr()), c_size_t(nbytes),
                            c_void_p(self.stream.cuda_stream), byref(h)))
        self._h = h

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lbsep_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    # -- stepping ------------------------------------------------------------
    def step(self, nsteps: int = 1):
        _check(load().lbsep_step(self._h, int(nsteps)))

    def step_record(self, pre: torch.Tensor | None = None, post: torch.Tensor | None = None):
        """One step that also returns the new level's pre- and post-collision
        populations (float64 [2, 9, ny, nx]; FP64 channels with one level per
        launch)."""
        if pre is None:
            pre = torch.empty((2, 9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        if post is None:
            post = torch.empty_like(pre)
        for a in (pre, post):
            if a.dtype != torch.float64 or a.shape != (2, 9, self.ny, self.nx) or not a.is_contiguous():
                raise LbsepError("step_record outputs must be contiguous float64 [2, 9, ny, nx]")
        _check(load().lbsep_step_record(self._h, c_void_p(pre.data_ptr()), c_void_p(post.data_ptr())))
        self._hand_over(pre)
        self._hand_over(post)
        return pre, post

    @property
    def t(self) -> int:
        return int(load().lbsep_time(self._h))

    # -- readouts ------------------------------------------------------------
    def read_cl(self, profile: bool = False):
        cl, clt, xm = c_double(), c_double(), c_int32()
        prof = np.empty(self.nx) if profile else None
        _check(load().lbsep_read_cl(self._h, byref(cl), byref(clt), byref(xm),
                                    _dptr(prof) if profile else None))
        out = {"cl": cl.value, "cl_tilde": clt.value, "x_min": xm.value}
        if profile:
            out["profile"] = prof
        return out

    def read_column_sums(self) -> np.ndarray:
        out = np.empty((4, self.nx))
        _check(load().lbsep_read_column_sums(self._h, _dptr(out)))
        return out

    def read_history(self, t0: int, count: int) -> np.ndarray:
        out = np.empty((count, 4))
        _check(load().lbsep_read_history(self._h, int(t0), int(count), _dptr(out)))
        return out

    def read_moments(self) -> np.ndarray:
        out = np.empty((6, self.ny, self.nx))
        _check(load().lbsep_read_moments(self._h, _dptr(out)))
        return out

    def read_volume_flow(self) -> np.ndarray:
        out = np.empty(self.nx)
        _check(load().lbsep_read_volume_flow(self._h, _dptr(out)))
        return out

    def get_state(self) -> torch.Tensor:
        """Raw state in the storage type (f for f64, deviations for f32/f16)."""
        out = torch.empty((2, 9, self.ny, self.nx), dtype=self.dtype, device=self.device)
        _check(load().lbsep_get_state(self._h, c_void_p(out.data_ptr())))
        self._hand_over(out)
        return out

    def set_state(self, f: torch.Tensor, t: int = 0):
        if f.shape != (2, 9, self.ny, self.nx) or f.dtype != self.dtype or f.device.type != "cuda":
            raise ValueError(f"state must be a {self.dtype} cuda tensor of shape (2, 9, {self.ny}, {self.nx})")
        f = f.contiguous()
        self._take_over()
        _check(load().lbsep_set_state(self._h, c_void_p(f.data_ptr()), int(t)))
        self._keep = f  # keep the source alive until the stream has consumed it

    def get_populations(self) -> torch.Tensor:
        """Pre-collision populations f in float64, whatever the storage type."""
        out = torch.empty((2, 9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        _check(load().lbsep_get_populations(self._h, c_void_p(out.data_ptr())))
        self._hand_over(out)
        return out

    def get_post_collision(self) -> torch.Tensor:
        """Post-collision populations f'(t) = C(f(t)) of the current level in
        float64 (the state the next step streams)."""
        out = torch.empty((2, 9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        _check(load().lbsep_get_post_collision(self._h, c_void_p(out.data_ptr())))
        self._hand_over(out)
        return out

    def set_populations(self, f: torch.Tensor, t: int = 0):
        if f.shape != (2, 9, self.ny, self.nx) or f.dtype != torch.float64 or f.device.type != "cuda":
            raise ValueError(f"populations must be a float64 cuda tensor of shape (2, 9, {self.ny}, {self.nx})")
        f = f.contiguous()
        self._take_over()
        _check(load().lbsep_set_populations(self._h, c_void_p(f.data_ptr()), int(t)))
        self._keep = f

    def synchronize(self):
        self.stream.synchronize()

    # -- stream hand-over (the channel may run on a stream other than torch's) --
    def _take_over(self):
        """The channel's stream waits for torch's current stream (inputs ready)."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _hand_over(self, out: torch.Tensor):
        """torch's current stream waits for the channel's stream (output ready)."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
            out.record_stream(self.stream)


class Batch:
    """Several channels advanced by one sweep launch per step (lbsep_batch_*).

    The channels must share one dtype and one stream; they stay usable through
    their own readouts between batch steps. For a captured step graph
    (``capture``) that stream must not be the default stream."""

    def __init__(self, channels):
        L = load()
        self.channels = list(channels)
        arr = (c_void_p * len(self.channels))(*[c._h.value for c in self.channels])
        self._arr = arr
        nbytes = L.lbsep_batch_workspace_bytes(arr, len(self.channels))
        if nbytes == 0:
            raise LbsepError(EINVAL, last_error())
        dev = self.channels[0].device
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + nbytes]
        self.stream = self.channels[0].stream
        if self.stream != torch.cuda.current_stream(dev):
            raw.record_stream(self.stream)
        h = c_void_p()
        _check(L.lbsep_batch_create(arr, len(self.channels), c_void_p(self.ws.data_ptr()), c_size_t(nbytes),
                                    byref(h)))
        self._h = h

    def step(self, nsteps: int = 1):
        _check(load().lbsep_batch_step(self._h, int(nsteps)))

    def capture(self, steps: int):
        _check(load().lbsep_batch_capture(self._h, int(steps)))

    def __len__(self):
        return int(load().lbsep_batch_size(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lbsep_batch_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
