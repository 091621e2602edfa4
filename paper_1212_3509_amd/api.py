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
STATUS = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_HIP", 4: "E_UNSUPPORTED", 5: "E_ACCURACY"}


class DemagError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {message}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3)]


class Quad(C.Structure):
    _fields_ = [("M", C.c_int32), ("c0", C.c_double), ("step_rule", C.c_int32),
                ("t", C.POINTER(C.c_double)), ("alpha", C.POINTER(C.c_double))]


class QuadResult(C.Structure):
    _fields_ = [("R", C.c_int32), ("fell_back", C.c_int32), ("fits", C.c_int32), ("mode", C.c_int32),
                ("err_phi", C.c_double), ("err_h", C.c_double), ("predicted", C.c_double), ("seconds", C.c_double),
                ("t", C.c_double * 64), ("alpha", C.c_double * 64)]


PREDICT_MODES = {"network": 0, "network_proposal": 1, "search": 2}


class TuckerIn(C.Structure):
    _fields_ = [("r", C.c_int32 * 3), ("core", C.c_void_p), ("rows", C.c_void_p * 3)]

_P = C.c_void_p
_SIGS = {
    "demag_last_error": (C.c_char_p, []),
    "demag_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "demag_destroy": (C.c_int, [_P]),
    "demag_set_stream": (C.c_int, [_P, _P]),
    "demag_set_workspace_limit": (C.c_int, [_P, C.c_size_t]),
    "demag_set_input_check": (C.c_int, [_P, C.c_int32]),
    "demag_set_tiles": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "demag_assemble_factors": (C.c_int, [_P, C.POINTER(Grid), C.POINTER(Quad), C.POINTER(_P)]),
    "demag_factors_free": (C.c_int, [_P]),
    "demag_assemble_factors_grid": (C.c_int, [_P, _P, _P, C.POINTER(Quad), C.POINTER(_P)]),
    "demag_factors_count": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "demag_factors_length_scale": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "demag_factors_nodes": (C.c_int, [_P, _P, _P, _P]),
    "demag_factors_download": (C.c_int, [_P, _P, C.c_int32, _P]),
    "demag_apply_full": (C.c_int, [_P, _P, C.c_int, _P, _P, _P]),
    "demag_apply_full_workspace_size": (C.c_int, [_P, C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "demag_apply_full_ws": (C.c_int, [_P, _P, C.c_int, _P, _P, _P, _P, C.c_size_t]),
    "demag_apply_fft": (C.c_int, [_P, _P, _P, _P, _P]),
    "demag_batch_create": (C.c_int, [_P, C.c_int32, _P, C.POINTER(Quad), C.c_int, C.POINTER(_P)]),
    "demag_batch_free": (C.c_int, [_P]),
    "demag_batch_offsets": (C.c_int, [_P, _P]),
    "demag_batch_info": (C.c_int, [_P, _P, _P, _P]),
    "demag_batch_apply": (C.c_int, [_P, _P, _P, _P, _P, C.c_int32]),
    "demag_batch_tune": (C.c_int, [_P, _P, C.c_char_p, C.c_int32]),
    "demag_mlp_param_count": (C.c_int32, []),
    "demag_mlp_forward": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P]),
    "demag_mlp_backward": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int32, _P, _P]),
    "demag_adam_step": (C.c_int, [_P, _P, _P, _P, _P, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                                  C.c_float]),
    "demag_quad_judge": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, C.c_int32, _P, _P, _P, C.c_int32, _P, _P, _P,
                                   _P]),
    "demag_quad_certify": (C.c_int, [_P, C.POINTER(Grid), C.c_int32, _P, _P, _P]),
    "demag_quad_offsets": (C.c_int, [_P, C.c_int32, _P, _P]),
    "demag_quad_features": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, _P]),
    "demag_quad_rules": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P]),
    "demag_quad_fit": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, C.c_int32, _P, _P, C.c_int32, C.c_double, _P, _P,
                                 _P, _P, _P, _P]),
    "demag_quad_loss_grad": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int32, C.c_float, _P, _P]),
    "demag_quad_train": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_float, C.c_float, _P]),
    "demag_quad_predict": (C.c_int, [_P, _P, C.POINTER(Grid), C.c_double, C.c_int32, C.c_int32,
                                     C.POINTER(QuadResult)]),
    "demag_prepare_structured": (C.c_int, [_P, _P]),
    "demag_apply_columns": (C.c_int, [_P, _P, C.c_int, _P, _P, _P]),
    "demag_apply_columns_noalloc": (C.c_int, [_P, _P, _P, _P, _P]),
    "demag_apply_cp": (C.c_int, [_P, _P, C.c_int, C.c_int32, _P, _P, _P]),
    "demag_apply_tucker": (C.c_int, [_P, _P, C.c_int, _P, _P, _P, _P]),
    "demag_apply_tt": (C.c_int, [_P, _P, C.c_int, C.c_int32, C.c_int32, _P, _P, _P, _P, _P]),
    "demag_recompress_cp": (C.c_int, [_P, _P, C.c_int32, _P, _P, _P, _P, C.c_double, C.c_int32, C.c_int32, _P,
                                      _P, _P, _P, _P, _P, _P]),
    "demag_ktucker_create": (C.c_int, [_P, _P, C.c_double, C.POINTER(_P)]),
    "demag_ktucker_ranks": (C.c_int, [_P, C.c_int32, _P]),
    "demag_ktucker_copy": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "demag_ktucker_free": (C.c_int, [_P]),
    "demag_potential_tucker": (C.c_int, [_P, _P, _P, C.c_double, C.c_int32, _P, _P, _P]),
    "demag_tucker_sum": (C.c_int, [_P, _P, C.c_int32, _P, C.c_double, C.c_int32, _P, _P, _P]),
    "demag_tt_round": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, _P, _P, C.c_double, C.c_int32, _P, _P, _P,
                                 _P]),
    "demag_cp_to_tt": (C.c_int, [_P, _P, C.c_int32, _P, _P, _P, _P, _P]),
    "demag_tucker_to_tt": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "demag_tt_to_tucker": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, _P, _P, C.c_double, C.c_int32, _P, _P, _P]),
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


def quad_offsets(n, count: int = 256):
    """Offsets [count][3] (int32) and weights [count] (float64) of the judge
    on grid n, computed by the library (host only, no device needed)."""
    J = np.zeros((count, 3), dtype=np.int32)
    w = np.zeros(count, dtype=np.float64)
    _check(library().demag_quad_offsets((C.c_int32 * 3)(*n), count, J.ctypes.data, w.ctypes.data),
           "demag_quad_offsets")
    return J, w


def quad_features(n, h, log10_tol, R):
    """Network input (float32 [6]) of one case, computed by the library."""
    x = np.zeros(6, dtype=np.float32)
    _check(library().demag_quad_features((C.c_int32 * 3)(*n), h, log10_tol, R, x.ctypes.data),
           "demag_quad_features")
    return x


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

    dense = False

    def __init__(self, ctx: "Context", handle, n, h):
        self.ctx, self.handle, self.n, self.h = ctx, handle, tuple(n), tuple(h)

    @property
    def M(self) -> int:
        m = C.c_int32()
        _check(library().demag_factors_count(self.handle, C.byref(m)), "demag_factors_count")
        return m.value

    @property
    def length_scale(self) -> float:
        """L: structured potentials are L times their sum of terms."""
        L = C.c_double()
        _check(library().demag_factors_length_scale(self.handle, C.byref(L)), "demag_factors_length_scale")
        return L.value

    def workspace_size(self, prec: str = "fp64"):
        """(one_chunk, minimum) workspace bytes of apply_full(_ws)."""
        a, b = C.c_size_t(), C.c_size_t()
        _check(library().demag_apply_full_workspace_size(self.handle, PRECISIONS[prec], C.byref(a), C.byref(b)),
               "demag_apply_full_workspace_size")
        return a.value, b.value

    def nodes(self):
        M = self.M
        t, tau, alpha = (np.empty(M) for _ in range(3))
        _check(library().demag_factors_nodes(self.handle, t.ctypes.data, tau.ctypes.data, alpha.ctypes.data),
               "demag_factors_nodes")
        return t, tau, alpha

    def download(self, d: int) -> np.ndarray:
        """FP64 factor table of axis d as [4][M][2 n_d - 1] (non-uniform
        grids: dense [4][M][n_d][n_d])."""
        n = self.n[d]
        out = np.empty((4, self.M, n, n) if self.dense else (4, self.M, 2 * n - 1))
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


class Batch:
    """Many states on uneven grids (library handle); fields are packed."""

    def __init__(self, ctx: "Context", handle, count):
        self.ctx, self.handle, self.count = ctx, handle, count

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.count + 1, dtype=np.int64)
        _check(library().demag_batch_offsets(self.handle, off.ctypes.data), "demag_batch_offsets")
        return off

    def info(self):
        kc, grid, fl = C.c_int32(), C.c_int32(), C.c_double()
        _check(library().demag_batch_info(self.handle, C.byref(kc), C.byref(grid), C.byref(fl)), "demag_batch_info")
        return {"node_chunk": kc.value, "persistent_groups": grid.value, "flops": fl.value}

    def tune(self, path=None, reps: int = 3):
        self.ctx.use_current_stream()
        _check(library().demag_batch_tune(self.ctx.handle, self.handle, None if path is None else path.encode(), reps),
               "demag_batch_tune")

    def apply(self, m, phi, h, use_graph: bool = False):
        self.ctx.use_current_stream()
        _check(library().demag_batch_apply(self.ctx.handle, self.handle, _ptr(m), _ptr(phi), _ptr(h),
                                           1 if use_graph else 0), "demag_batch_apply")

    def free(self):
        if self.handle:
            library().demag_batch_free(self.handle)
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

    def set_input_check(self, on: bool = True):
        """Reject NaN / infinite inputs (one device scan and a stream sync per call)."""
        _check(library().demag_set_input_check(self.handle, 1 if on else 0), "demag_set_input_check")

    def set_tiles(self, rows: int = 0, cols: int = 0):
        """Tile shape of the full-format products (0 = automatic)."""
        _check(library().demag_set_tiles(self.handle, rows, cols), "demag_set_tiles")

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

    def assemble_grid(self, edges, M: int = 40, c0: float = 2.15, step_rule: int = 0) -> Factors:
        """Factors of a non-uniform tensor-product grid: edges[d] = the n_d + 1
        cell boundaries of axis d (x, y, z)."""
        ed = [np.ascontiguousarray(e, dtype=np.float64) for e in edges]
        n = tuple(len(e) - 1 for e in ed)
        ptrs = (C.c_void_p * 3)(*[e.ctypes.data for e in ed])
        q = Quad(M, c0, step_rule, None, None)
        out = C.c_void_p()
        self.use_current_stream()
        _check(library().demag_assemble_factors_grid(self.handle, (C.c_int32 * 3)(*n), ptrs, C.byref(q),
                                                     C.byref(out)), "demag_assemble_factors_grid")
        f = Factors(self, out, n, tuple(float(np.min(np.diff(e))) for e in ed))
        f.dense = True
        return f

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

    def apply_full_ws(self, f: Factors, m, workspace, phi=None, h=None, prec: str = "fp64"):
        """apply_full on a caller-owned workspace (a contiguous CUDA tensor; its
        byte size bounds the node chunks)."""
        import torch
        nx, ny, nz = f.n
        dt = torch.float64 if prec == "fp64" else torch.float32
        if m.dtype != dt or not m.is_cuda or not m.is_contiguous() or tuple(m.shape) != (3, nz, ny, nx):
            raise ValueError(f"m must be a contiguous {dt} CUDA tensor of shape {(3, nz, ny, nx)}")
        if phi is None:
            phi = torch.empty((nz, ny, nx), dtype=dt, device=m.device)
        if h is None:
            h = torch.empty((3, nz, ny, nx), dtype=dt, device=m.device)
        nbytes = workspace.numel() * workspace.element_size()
        self.use_current_stream()
        _check(library().demag_apply_full_ws(self.handle, f.handle, PRECISIONS[prec], _ptr(m), _ptr(phi), _ptr(h),
                                             _ptr(workspace), nbytes), "demag_apply_full_ws")
        return phi, h

    def apply_fft(self, f: Factors, m, phi=None, h=None):
        """Same operator as apply_full, by 3D FFT convolution (FP64 only)."""
        import torch
        nx, ny, nz = f.n
        if m.dtype != torch.float64 or not m.is_cuda or not m.is_contiguous() or tuple(m.shape) != (3, nz, ny, nx):
            raise ValueError(f"m must be a contiguous float64 CUDA tensor of shape {(3, nz, ny, nx)}")
        if phi is None:
            phi = torch.empty((nz, ny, nx), dtype=torch.float64, device=m.device)
        if h is None:
            h = torch.empty((3, nz, ny, nx), dtype=torch.float64, device=m.device)
        self.use_current_stream()
        _check(library().demag_apply_fft(self.handle, f.handle, _ptr(m), _ptr(phi), _ptr(h)), "demag_apply_fft")
        return phi, h

    def batch(self, grids, M: int = 40, c0: float = 2.15, step_rule: int = 0, prec: str = "fp32") -> Batch:
        """grids: list of ((nx, ny, nz), (hx, hy, hz))."""
        arr = (Grid * len(grids))()
        for i, (n, h) in enumerate(grids):
            arr[i] = Grid((C.c_int32 * 3)(*n), (C.c_double * 3)(*h))
        q = Quad(M, c0, step_rule, None, None)
        out = C.c_void_p()
        self.use_current_stream()
        _check(library().demag_batch_create(self.handle, len(grids), arr, C.byref(q), PRECISIONS[prec],
                                            C.byref(out)), "demag_batch_create")
        return Batch(self, out, len(grids))

    # ------------------------------------------------------------ structured
    def _cols_out(self, f: Factors, R, device):
        import torch
        M = f.M
        return [torch.empty((3, 2, M, R[d], f.n[d]), dtype=torch.float32, device=device) for d in range(3)]

    @staticmethod
    def _ptr3(ts):
        return (C.c_void_p * 3)(*[t.data_ptr() for t in ts])

    def prepare_structured(self, f: Factors):
        self.use_current_stream()
        _check(library().demag_prepare_structured(self.handle, f.handle), "demag_prepare_structured")

    def apply_columns(self, f: Factors, cols_in, prec: str = "fp64"):
        """cols_in[d]: float32 CUDA tensor [3][R_d][n_d].  Returns out[d]
        [3][2][M][R_d][n_d].  prec: "fp64" or "fp32" transforms."""
        R = [int(c.shape[1]) for c in cols_in]
        out = self._cols_out(f, R, cols_in[0].device)
        self.use_current_stream()
        Ra = (C.c_int32 * 3)(*R)
        _check(library().demag_apply_columns(self.handle, f.handle, PRECISIONS[prec], Ra, self._ptr3(cols_in),
                                             self._ptr3(out)), "demag_apply_columns")
        return out

    def apply_cp(self, f: Factors, U, prec: str = "fp64"):
        """U[d]: float32 CUDA tensor [3][r][n_d].  Returns (out[3], table)."""
        r = int(U[0].shape[1])
        out = self._cols_out(f, [r, r, r], U[0].device)
        table = np.empty((4, 3 * f.M * r, 3), dtype=np.int32)
        self.use_current_stream()
        _check(library().demag_apply_cp(self.handle, f.handle, PRECISIONS[prec], r, self._ptr3(U), self._ptr3(out),
                                        table.ctypes.data), "demag_apply_cp")
        return out, table

    def apply_tucker(self, f: Factors, U, prec: str = "fp64"):
        r = [int(u.shape[1]) for u in U]
        out = self._cols_out(f, r, U[0].device)
        table = np.empty((4, 3 * f.M, 3), dtype=np.int32)
        self.use_current_stream()
        _check(library().demag_apply_tucker(self.handle, f.handle, PRECISIONS[prec], (C.c_int32 * 3)(*r),
                                            self._ptr3(U), self._ptr3(out), table.ctypes.data), "demag_apply_tucker")
        return out, table

    def apply_tt(self, f: Factors, G1, G2, G3, prec: str = "fp64"):
        """G1 [3][r1][n_x], G2 [3][r1][r2][n_y], G3 [3][r2][n_z] (float32 CUDA)."""
        r1, r2 = int(G1.shape[1]), int(G3.shape[1])
        out = self._cols_out(f, [r1, r1 * r2, r2], G1.device)
        table = np.empty((4, 3 * f.M, 3), dtype=np.int32)
        self.use_current_stream()
        _check(library().demag_apply_tt(self.handle, f.handle, PRECISIONS[prec], r1, r2, _ptr(G1), _ptr(G2),
                                        _ptr(G3), self._ptr3(out), table.ctypes.data), "demag_apply_tt")
        return out, table

    def recompress_cp(self, n, cols, table, lam, eps, rmax=32, max_sweeps=10, seed=7):
        """HOOI recompression of the CP tensor sum_t lam[t] cols[0][table[t,0]] o
        cols[1][table[t,1]] o cols[2][table[t,2]] (cols: contiguous float32 CUDA
        column sets, ncols x n_p values, e.g. the outputs of apply_cp;
        table int32 [T][3], lam float64 [T], CUDA) to Tucker form.  The
        Gaussian test matrices come from inputs.recompress_test_matrices(seed).
        Returns dict(U [3] (r_p x n_p), core (r0, r1, r2), ranks, rel_err, sweeps)."""
        import torch
        from . import inputs
        T = int(lam.shape[0])
        dev = lam.device
        omega, gmat = inputs.recompress_test_matrices(tuple(n), rmax, seed)
        om = torch.from_numpy(omega).to(dev)
        gm = torch.from_numpy(gmat).to(dev)
        U = [torch.empty((rmax, n[p]), dtype=torch.float64, device=dev) for p in range(3)]
        core = torch.empty(rmax ** 3, dtype=torch.float64, device=dev)
        ranks = (C.c_int32 * 3)()
        err, sweeps = C.c_double(), C.c_int32()
        n3 = (C.c_int32 * 3)(*n)
        nc = (C.c_int32 * 3)(*[int(cols[p].numel() // n[p]) for p in range(3)])   # columns of n_p values
        self.use_current_stream()
        _check(library().demag_recompress_cp(self.handle, n3, T, self._ptr3(cols), nc, _ptr(table), _ptr(lam), eps,
                                             rmax, max_sweeps, _ptr(om), _ptr(gm), self._ptr3(U), _ptr(core),
                                             ranks, C.byref(err), C.byref(sweeps)), "demag_recompress_cp")
        r = [ranks[p] for p in range(3)]
        return {"U": [U[p][:r[p]] for p in range(3)], "core": core[:r[0] * r[1] * r[2]].reshape(r),
                "ranks": tuple(r), "rel_err": err.value, "sweeps": sweeps.value}

    # ------------------------------------------------------------ learned rule
    def mlp_forward(self, params, x):
        """params: float32 CUDA [12993]; x: float32 CUDA [B][6].  Returns (y, z, a)."""
        import torch
        B = int(x.shape[0])
        y = torch.empty((B, 65), dtype=torch.float32, device=x.device)
        z = torch.empty((B, 3, 64), dtype=torch.float32, device=x.device)
        a = torch.empty((B, 3, 64), dtype=torch.float32, device=x.device)
        self.use_current_stream()
        _check(library().demag_mlp_forward(self.handle, _ptr(params), _ptr(x), B, _ptr(y), _ptr(z), _ptr(a)),
               "demag_mlp_forward")
        return y, z, a

    def mlp_backward(self, params, x, z, a, dy):
        import torch
        B = int(x.shape[0])
        delta = torch.empty((B, 3, 64), dtype=torch.float32, device=x.device)
        grad = torch.empty(params.numel(), dtype=torch.float32, device=x.device)
        self.use_current_stream()
        _check(library().demag_mlp_backward(self.handle, _ptr(params), _ptr(x), _ptr(z), _ptr(a), _ptr(dy), B,
                                            _ptr(delta), _ptr(grad)), "demag_mlp_backward")
        return grad

    def adam_step(self, params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.use_current_stream()
        _check(library().demag_adam_step(self.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(),
                                         step, lr, b1, b2, eps), "demag_adam_step")

    def quad_rules(self, y, R):
        """Rules from network outputs y (CUDA float32 [B][65], or None for the
        base rule) and node counts R (CUDA int32 [B]): (t, alpha) [B][32]."""
        import torch
        B = int(R.shape[0])
        t = torch.zeros((B, 32), dtype=torch.float64, device=R.device)
        a = torch.zeros((B, 32), dtype=torch.float64, device=R.device)
        self.use_current_stream()
        _check(library().demag_quad_rules(self.handle, _ptr(y), _ptr(R), B, _ptr(t), _ptr(a)), "demag_quad_rules")
        return t, a

    def quad_judge(self, grids, hmin, sent, weights, t, alpha, R, grad=False, parts=False):
        """grids int32 [B][3], hmin float64 [B], sent int32 [B][S][3], weights
        float64 [B][S], t/alpha float64 [B][KM], R int32 [B] (all CUDA).
        Returns err [B] (plus (e_phi, e_h) [B][2] with parts, and the
        gradients [B][KM] with respect to t and alpha with grad)."""
        import torch
        B, S = int(sent.shape[0]), int(sent.shape[1])
        KM = int(t.shape[1])
        err = torch.empty(B, dtype=torch.float64, device=t.device)
        pp = torch.empty((B, 2), dtype=torch.float64, device=t.device) if parts else None
        dt = torch.empty((B, KM), dtype=torch.float64, device=t.device) if grad else None
        da = torch.empty((B, KM), dtype=torch.float64, device=t.device) if grad else None
        self.use_current_stream()
        _check(library().demag_quad_judge(self.handle, B, _ptr(grids), _ptr(hmin), _ptr(sent), _ptr(weights), S,
                                          _ptr(t), _ptr(alpha), _ptr(R), KM, _ptr(err), _ptr(pp), _ptr(dt),
                                          _ptr(da)), "demag_quad_judge")
        out = (err,)
        if parts:
            out += (pp,)
        if grad:
            out += (dt, da)
        return out if len(out) > 1 else err

    def quad_certify(self, n, h, t, alpha):
        """Certificate (e_phi, e_h) of the rule (host t, alpha, scaled domain)
        on the grid n with cell sizes h (physical; scaled internally)."""
        ta = np.ascontiguousarray(t, dtype=np.float64)
        aa = np.ascontiguousarray(alpha, dtype=np.float64)
        g = Grid((C.c_int32 * 3)(*n), (C.c_double * 3)(*h))
        err = np.zeros(2)
        self.use_current_stream()
        _check(library().demag_quad_certify(self.handle, C.byref(g), len(ta), ta.ctypes.data, aa.ctypes.data,
                                            err.ctypes.data), "demag_quad_certify")
        return float(err[0]), float(err[1])

    def quad_fit(self, grids, hmin, sent, weights, R, y0=None, iters=30, mu0=1e-3, want_h=False):
        """Levenberg-Marquardt fit of the outputs per case (all CUDA: grids int32
        [B][3], hmin float64 [B], sent int32 [B][S][3], weights float64 [B][S],
        R int32 [B], y0 float32 [B][65] or None).  Returns (y [B][65], t [B][32],
        alpha [B][32], err [B]), plus (x [B][64], H [B][64][64]) with want_h."""
        import torch
        B, S = int(sent.shape[0]), int(sent.shape[1])
        dev = sent.device
        y = torch.empty((B, 65), dtype=torch.float32, device=dev)
        t = torch.empty((B, 32), dtype=torch.float64, device=dev)
        a = torch.empty((B, 32), dtype=torch.float64, device=dev)
        err = torch.empty(B, dtype=torch.float64, device=dev)
        x = torch.empty((B, 64), dtype=torch.float64, device=dev) if want_h else None
        H = torch.empty((B, 64, 64), dtype=torch.float32, device=dev) if want_h else None
        self.use_current_stream()
        _check(library().demag_quad_fit(self.handle, B, _ptr(grids), _ptr(hmin), _ptr(sent), _ptr(weights), S,
                                        _ptr(R), _ptr(y0), iters, mu0, _ptr(y), _ptr(x), _ptr(H), _ptr(t), _ptr(a),
                                        _ptr(err)), "demag_quad_fit")
        return (y, t, a, err, x, H) if want_h else (y, t, a, err)

    def quad_loss_grad(self, y, targets, xfit, H, R, lam=0.1):
        """Training loss per case and d loss / d y (see demag_quad_loss_grad)."""
        import torch
        B = int(y.shape[0])
        dy = torch.empty_like(y)
        loss = torch.empty(B, dtype=torch.float32, device=y.device)
        self.use_current_stream()
        _check(library().demag_quad_loss_grad(self.handle, _ptr(y), _ptr(targets), _ptr(xfit), _ptr(H), _ptr(R), B,
                                              lam, _ptr(dy), _ptr(loss)), "demag_quad_loss_grad")
        return loss, dy

    def quad_train(self, params, m, v, x, targets, R, steps, batch, step0=0, lr=1e-3, lam=0.1, xfit=None, H=None):
        """Adam on the distillation loss against fitted targets [count][65]
        (with xfit, H; else squared output errors)."""
        loss = np.zeros(max(steps, 1), dtype=np.float32)
        self.use_current_stream()
        _check(library().demag_quad_train(self.handle, _ptr(params), _ptr(m), _ptr(v), _ptr(x), _ptr(targets),
                                          _ptr(xfit), _ptr(H), _ptr(R), int(x.shape[0]), steps, batch, step0, lr, lam,
                                          loss.ctypes.data), "demag_quad_train")
        return loss[:steps]

    def quad_predict(self, params, n, h, tol, fit_iters=200, mode="network"):
        """Shortened rule for grid n with cubic cells h at tolerance tol (both
        certificates).  params: CUDA float32 network parameters (None in the
        "search" mode).  Returns a dict: t, alpha, R, fell_back, fits,
        err_phi, err_h, predicted, seconds, accuracy_met (False when even the
        fallback rule misses tol: DEMAG_E_ACCURACY)."""
        g = Grid((C.c_int32 * 3)(*n), (C.c_double * 3)(*((h,) * 3 if np.isscalar(h) else h)))
        res = QuadResult()
        self.use_current_stream()
        st = library().demag_quad_predict(self.handle, _ptr(params), C.byref(g), tol, fit_iters, PREDICT_MODES[mode],
                                          C.byref(res))
        if st not in (0, 5):
            _check(st, "demag_quad_predict")
        R = res.R
        return {"t": np.array(res.t[:R]), "alpha": np.array(res.alpha[:R]), "R": R,
                "fell_back": bool(res.fell_back), "fits": res.fits, "err_phi": res.err_phi, "err_h": res.err_h,
                "judged": max(res.err_phi, res.err_h), "predicted": res.predicted, "seconds": res.seconds,
                "accuracy_met": st == 0, "mode": mode}

    # ------------------------------------------------------------ Tucker route

    def ktucker(self, f: "Factors", tol: float):
        """Set-up of Alg. scpot_fft_tucker: the factors' three kernels
        compressed to Tucker with tol, with their factor-row DFTs."""
        h = C.c_void_p()
        _check(library().demag_ktucker_create(self.handle, f.handle, tol, C.byref(h)), "demag_ktucker_create")
        return KTucker(self, h, f.n)

    @staticmethod
    def _tucker_in(t):
        core, rows = t
        for x in (core, *rows):
            if not (x.is_cuda and x.is_contiguous()) or str(x.dtype) != "torch.float64":
                raise ValueError("Tucker cores and factor rows must be contiguous float64 CUDA tensors")
        r = [int(rows[p].shape[0]) for p in range(3)]
        if tuple(core.shape) != tuple(r):
            raise ValueError(f"core shape {tuple(core.shape)} does not match the factor rows {r}")
        return TuckerIn((C.c_int32 * 3)(*r), core.data_ptr(), (C.c_void_p * 3)(*[rows[p].data_ptr() for p in range(3)]))

    def _tucker_out(self, call, n, rmax, where):
        import torch
        core = torch.empty(rmax ** 3, dtype=torch.float64, device="cuda")
        rows = [torch.empty((rmax, n[p]), dtype=torch.float64, device="cuda") for p in range(3)]
        rout = (C.c_int32 * 3)()
        self.use_current_stream()
        _check(call(rout, _ptr(core), self._ptr3(rows)), where)
        r = [rout[p] for p in range(3)]
        return core[:r[0] * r[1] * r[2]].reshape(r), [rows[p][:r[p]] for p in range(3)]

    def potential_tucker(self, kt: "KTucker", mag, tol: float, rmax: int = 128):
        """Alg. scpot_fft_tucker for the three magnetization components
        mag[q] = (core [r0][r1][r2], [rows_p [r_p][n_p]]) (float64 CUDA).
        Returns the potential (core, rows) in the factors' scaled units."""
        ins = (TuckerIn * 3)(*[self._tucker_in(mag[q]) for q in range(3)])
        return self._tucker_out(lambda ro, co, ro3: library().demag_potential_tucker(
            self.handle, kt.handle, ins, tol, rmax, ro, co, ro3), kt.n, rmax, "demag_potential_tucker")

    def tucker_sum(self, n, terms, tol: float, rmax: int = 128):
        """Approximate summation of the Tucker tensors terms[t] = (core, rows)."""
        ins = (TuckerIn * len(terms))(*[self._tucker_in(t) for t in terms])
        n3 = (C.c_int32 * 3)(*n)
        return self._tucker_out(lambda ro, co, ro3: library().demag_tucker_sum(
            self.handle, n3, len(terms), ins, tol, rmax, ro, co, ro3), n, rmax, "demag_tucker_sum")

    def tt_round(self, G1, G2, G3, tol: float, rmax: int = 128):
        """TT rounding of G1 [r1][n0], G2 [r1][r2][n1], G3 [r2][n2] (float64
        CUDA).  Returns the rounded cores in the same layout."""
        import torch
        r1, r2 = int(G1.shape[0]), int(G3.shape[0])
        n = (int(G1.shape[1]), int(G2.shape[2]), int(G3.shape[1]))
        if tuple(G2.shape) != (r1, r2, n[1]):
            raise ValueError("G2 must be [r1][r2][n1]")
        for x in (G1, G2, G3):
            if not (x.is_cuda and x.is_contiguous()) or x.dtype != torch.float64:
                raise ValueError("TT cores must be contiguous float64 CUDA tensors")
        H1 = torch.empty((rmax, n[0]), dtype=torch.float64, device="cuda")
        H2 = torch.empty(rmax * rmax * n[1], dtype=torch.float64, device="cuda")
        H3 = torch.empty((rmax, n[2]), dtype=torch.float64, device="cuda")
        rout = (C.c_int32 * 2)()
        self.use_current_stream()
        _check(library().demag_tt_round(self.handle, (C.c_int32 * 3)(*n), r1, r2, _ptr(G1), _ptr(G2), _ptr(G3), tol,
                                        rmax, rout, _ptr(H1), _ptr(H2), _ptr(H3)), "demag_tt_round")
        s1, s2 = rout[0], rout[1]
        return H1[:s1], H2[:s1 * s2 * n[1]].reshape(s1, s2, n[1]), H3[:s2]

    def cp_to_tt(self, lam, U):
        """CP (lam [R], U[p] [R][n_p], float64 CUDA) -> TT cores G1 [R][n0],
        G2 [R][R][n1], G3 [R][n2] (the library's TT layout)."""
        import torch
        R = int(lam.shape[0])
        n = [int(U[p].shape[1]) for p in range(3)]
        for x in (lam, *U):
            if not (x.is_cuda and x.is_contiguous()) or x.dtype != torch.float64:
                raise ValueError("CP weights and factor rows must be contiguous float64 CUDA tensors")
        G1 = torch.empty((R, n[0]), dtype=torch.float64, device="cuda")
        G2 = torch.empty((R, R, n[1]), dtype=torch.float64, device="cuda")
        G3 = torch.empty((R, n[2]), dtype=torch.float64, device="cuda")
        self.use_current_stream()
        _check(library().demag_cp_to_tt(self.handle, (C.c_int32 * 3)(*n), R, _ptr(lam), self._ptr3(U), _ptr(G1),
                                        _ptr(G2), _ptr(G3)), "demag_cp_to_tt")
        return G1, G2, G3

    def tucker_to_tt(self, core, rows):
        """Tucker (core, rows) -> TT cores in the library's TT layout."""
        import torch
        t = self._tucker_in((core, rows))
        n = [int(rows[p].shape[1]) for p in range(3)]
        r = [int(rows[p].shape[0]) for p in range(3)]
        G1 = torch.empty((r[0], n[0]), dtype=torch.float64, device="cuda")
        G2 = torch.empty((r[0], r[2], n[1]), dtype=torch.float64, device="cuda")
        G3 = torch.empty((r[2], n[2]), dtype=torch.float64, device="cuda")
        self.use_current_stream()
        _check(library().demag_tucker_to_tt(self.handle, (C.c_int32 * 3)(*n), C.byref(t), _ptr(G1), _ptr(G2),
                                            _ptr(G3)), "demag_tucker_to_tt")
        return G1, G2, G3

    def tt_to_tucker(self, G1, G2, G3, tol: float, rmax: int = 128):
        """TT cores (library layout) -> Tucker (core, rows), recompressed with tol."""
        import torch
        r1, r2 = int(G1.shape[0]), int(G3.shape[0])
        n = (int(G1.shape[1]), int(G2.shape[2]), int(G3.shape[1]))
        for x in (G1, G2, G3):
            if not (x.is_cuda and x.is_contiguous()) or x.dtype != torch.float64:
                raise ValueError("TT cores must be contiguous float64 CUDA tensors")
        n3 = (C.c_int32 * 3)(*n)
        return self._tucker_out(lambda ro, co, ro3: library().demag_tt_to_tucker(
            self.handle, n3, r1, r2, _ptr(G1), _ptr(G2), _ptr(G3), tol, rmax, ro, co, ro3), n, rmax,
            "demag_tt_to_tucker")

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


class KTucker:
    """Compressed kernels of Alg. scpot_fft_tucker (library handle)."""

    def __init__(self, ctx: "Context", handle, n):
        self.ctx, self.handle, self.n = ctx, handle, tuple(n)

    def ranks(self, q: int):
        r = (C.c_int32 * 3)()
        _check(library().demag_ktucker_ranks(self.handle, q, r), "demag_ktucker_ranks")
        return tuple(r)

    def kernel(self, q: int):
        """(core, rows) of the compressed kernel q: rows[p] [r_p][2 n_p - 1]."""
        import torch
        r = self.ranks(q)
        core = torch.empty(r, dtype=torch.float64, device="cuda")
        rows = [torch.empty((r[p], 2 * self.n[p] - 1), dtype=torch.float64, device="cuda") for p in range(3)]
        self.ctx.use_current_stream()
        _check(library().demag_ktucker_copy(self.ctx.handle, self.handle, q, _ptr(core), Context._ptr3(rows)),
               "demag_ktucker_copy")
        return core, rows

    def close(self):
        if self.handle:
            library().demag_ktucker_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
