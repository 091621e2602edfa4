"""Thin Python binding of libdemag.so (ctypes): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory and
the current stream.  Importing this module does not load the library; the
first call of ``library()`` does and raises if it is missing, so a GPU run
can never fall back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdemag.so")
_lib = None

DEMAG_FP64, DEMAG_FP32, DEMAG_BF16X2, DEMAG_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": DEMAG_FP64, "fp32": DEMAG_FP32, "bf16x2": DEMAG_BF16X2, "bf16x3": DEMAG_BF16X3}
STATUS = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_HIP", 4: "E_UNSUPPORTED"}


class DemagError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {message}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3)]


class Quad(C.Structure):
    _fields_ = [("M", C.c_int32), ("c0", C.c_double), ("step_rule", C.c_int32),
                ("t", C.POINTER(C.c_double)), ("alpha", C.POINTER(C.c_double))]


_P = C.c_void_p
_SIGS = {
    "demag_last_error": (C.c_char_p, []),
    "demag_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "demag_destroy": (C.c_int, [_P]),
    "demag_set_stream": (C.c_int, [_P, _P]),
    "demag_set_workspace_limit": (C.c_int, [_P, C.c_size_t]),
    "demag_assemble_factors": (C.c_int, [_P, C.POINTER(Grid), C.POINTER(Quad), C.POINTER(_P)]),
    "demag_factors_free": (C.c_int, [_P]),
    "demag_factors_count": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "demag_factors_nodes": (C.c_int, [_P, _P, _P, _P]),
    "demag_factors_download": (C.c_int, [_P, _P, C.c_int32, _P]),
    "demag_apply_full": (C.c_int, [_P, _P, C.c_int, _P, _P, _P]),
    "demag_bf16_split": (C.c_int, [_P, _P, _P, C.c_size_t, C.c_int32]),
    "demag_profile_enable": (C.c_int, [_P, C.c_int32]),
    "demag_profile_read": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, C.POINTER(C.c_int32)]),
}


def library():
    """Load libdemag.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_1212_3509_amd/build.py")
        lib = C.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int, where: str):
    if status != 0:
        msg = library().demag_last_error().decode(errors="replace")
        raise DemagError(status, where, msg)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _current_stream(device: int):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Factors:
    """Assembled 1D factors of one grid and quadrature rule (library handle)."""

    def __init__(self, ctx: "Context", handle, n, h):
        self.ctx, self.handle, self.n, self.h = ctx, handle, tuple(n), tuple(h)

    @property
    def M(self) -> int:
        m = C.c_int32()
        _check(library().demag_factors_count(self.handle, C.byref(m)), "demag_factors_count")
        return m.value

    def nodes(self):
        M = self.M
        t, tau, alpha = (np.empty(M) for _ in range(3))
        _check(library().demag_factors_nodes(self.handle, t.ctypes.data, tau.ctypes.data, alpha.ctypes.data),
               "demag_factors_nodes")
        return t, tau, alpha

    def download(self, d: int) -> np.ndarray:
        """FP64 factor table of axis d as [4][M][2 n_d - 1]."""
        out = np.empty((4, self.M, 2 * self.n[d] - 1))
        _check(library().demag_factors_download(self.ctx.handle, self.handle, d, out.ctypes.data),
               "demag_factors_download")
        return out

    def free(self):
        if self.handle:
            library().demag_factors_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """Library context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        h = C.c_void_p()
        s = _current_stream(device) if stream is None else C.c_void_p(stream)
        torch.cuda.init()
        _check(library().demag_create(device, s, C.byref(h)), "demag_create")
        self.handle = h

    def use_current_stream(self):
        _check(library().demag_set_stream(self.handle, _current_stream(self.device)), "demag_set_stream")

    def set_workspace_limit(self, nbytes: int):
        _check(library().demag_set_workspace_limit(self.handle, nbytes), "demag_set_workspace_limit")

    def assemble(self, n, h, M: int = 40, c0: float = 2.15, step_rule: int = 0, t=None, alpha=None) -> Factors:
        g = Grid((C.c_int32 * 3)(*n), (C.c_double * 3)(*h))
        keep = []
        if t is not None:
            ta = np.ascontiguousarray(t, dtype=np.float64)
            aa = np.ascontiguousarray(alpha, dtype=np.float64)
            keep += [ta, aa]
            q = Quad(len(ta), c0, step_rule, ta.ctypes.data_as(C.POINTER(C.c_double)),
                     aa.ctypes.data_as(C.POINTER(C.c_double)))
        else:
            q = Quad(M, c0, step_rule, None, None)
        out = C.c_void_p()
        self.use_current_stream()
        _check(library().demag_assemble_factors(self.handle, C.byref(g), C.byref(q), C.byref(out)),
               "demag_assemble_factors")
        return Factors(self, out, n, h)

    def apply_full(self, f: Factors, m, phi=None, h=None, prec: str = "fp64"):
        """m: [3][nz][ny][nx] contiguous device tensor (float64 for fp64, else
        float32); phi/h outputs are allocated if not given.  Returns (phi, h)."""
        import torch
        nx, ny, nz = f.n
        dt = torch.float64 if prec == "fp64" else torch.float32
        if m.dtype != dt or not m.is_cuda or not m.is_contiguous() or tuple(m.shape) != (3, nz, ny, nx):
            raise ValueError(f"m must be a contiguous {dt} CUDA tensor of shape {(3, nz, ny, nx)}")
        if phi is None:
            phi = torch.empty((nz, ny, nx), dtype=dt, device=m.device)
        if h is None:
            h = torch.empty((3, nz, ny, nx), dtype=dt, device=m.device)
        self.use_current_stream()
        _check(library().demag_apply_full(self.handle, f.handle, PRECISIONS[prec], _ptr(m), _ptr(phi), _ptr(h)),
               "demag_apply_full")
        return phi, h

    def bf16_split(self, x, nparts: int = 3):
        """Device split of a contiguous float32 CUDA tensor into bfloat16 bit
        patterns, returned as an int16 tensor [nparts][numel]."""
        import torch
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 CUDA tensor")
        parts = torch.empty((nparts, x.numel()), dtype=torch.int16, device=x.device)
        self.use_current_stream()
        _check(library().demag_bf16_split(self.handle, _ptr(x), _ptr(parts), x.numel(), nparts), "demag_bf16_split")
        return parts

    def profile_enable(self, on: bool = True):
        _check(library().demag_profile_enable(self.handle, 1 if on else 0), "demag_profile_enable")

    def profile_read(self, max_labels: int = 64):
        """{label: dict(ms, launches, flops, bytes)} of the kernels timed since
        profiling was enabled."""
        labels = C.create_string_buffer(48 * max_labels)
        ms, fl, by = (np.zeros(max_labels) for _ in range(3))
        la = np.zeros(max_labels, dtype=np.int64)
        cnt = C.c_int32()
        _check(library().demag_profile_read(self.handle, max_labels, labels, ms.ctypes.data, la.ctypes.data,
                                            fl.ctypes.data, by.ctypes.data, C.byref(cnt)), "demag_profile_read")
        out = {}
        raw = labels.raw
        for i in range(cnt.value):
            name = raw[48 * i:48 * (i + 1)].split(b"\0", 1)[0].decode()
            out[name] = {"ms": float(ms[i]), "launches": int(la[i]), "flops": float(fl[i]), "bytes": float(by[i])}
        return out

    def close(self):
        if self.handle:
            library().demag_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
