"""Python binding of libbatched_omp.so (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; this module only
checks tensor shapes, allocates outputs and workspace with torch (device
memory) and passes raw pointers and the current torch stream through the C ABI
declared in include/batched_omp.h. If the library is missing it raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from collections import namedtuple
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbatched_omp.so")

OMP_OK, OMP_EINVAL, OMP_EWORKSPACE, OMP_EDEVICE, OMP_ENOTSUPP = 0, -1, -2, -3, -4
OMP_MAX_S = 256
PREC = {"fp32": 0, "bf16": 1}
NPHASE = 6
PHASES = ("dict", "init", "corr", "update", "output", "residual")
SIG_EPS, SIG_SMAX, SIG_DEPENDENT, SIG_NONFINITE, SIG_EXHAUSTED, SIG_WIDENED = 1, 2, 4, 8, 32, 64

EXPORTED = ("omp_dict_size", "omp_dict_init", "omp_opts_default", "omp_workspace_size", "omp_solve",
            "omp_status_string", "omp_last_hip_error", "omp_version")


class OmpError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        lib = load()
        msg = lib.omp_status_string(code).decode()
        if code == OMP_EDEVICE:
            msg += f" (hipError_t {lib.omp_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")


class OmpDictStruct(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("precision", ctypes.c_int32), ("M", ctypes.c_int64),
                ("N", ctypes.c_int64), ("Mp", ctypes.c_int64), ("Np", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("mem", ctypes.c_void_p), ("bytes", ctypes.c_size_t)]


class OmpOptsStruct(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tile_config", ctypes.c_int32),
                ("S_per_signal", ctypes.c_void_p), ("eps_per_signal", ctypes.c_void_p),
                ("status_out", ctypes.c_void_p), ("rnorm_out", ctypes.c_void_p),
                ("coef_out", ctypes.c_void_p), ("dict", ctypes.POINTER(OmpDictStruct)),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("phase_ms", ctypes.POINTER(ctypes.c_float)),
                ("phase_launches", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2407_06434_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.omp_dict_size.restype = SZ
    lib.omp_dict_size.argtypes = [I64, I64, I32]
    lib.omp_dict_init.restype = ctypes.c_int
    lib.omp_dict_init.argtypes = [ctypes.POINTER(OmpDictStruct), P, I64, I64, I64, I32, P, SZ, P]
    lib.omp_opts_default.restype = None
    lib.omp_opts_default.argtypes = [ctypes.POINTER(OmpOptsStruct)]
    lib.omp_workspace_size.restype = SZ
    lib.omp_workspace_size.argtypes = [I64, I64, I64, I32, ctypes.POINTER(OmpOptsStruct)]
    lib.omp_solve.restype = ctypes.c_int
    lib.omp_solve.argtypes = [P, I64, I64, I64, P, I64, I64, I32, ctypes.c_float, P, P,
                              ctypes.POINTER(OmpOptsStruct), P]
    lib.omp_status_string.restype = ctypes.c_char_p
    lib.omp_status_string.argtypes = [ctypes.c_int]
    lib.omp_last_hip_error.restype = ctypes.c_int
    lib.omp_last_hip_error.argtypes = []
    lib.omp_version.restype = ctypes.c_char_p
    lib.omp_version.argtypes = []
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream: Optional[torch.cuda.Stream], device) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _check_matrix(t: torch.Tensor, name: str, cols: int = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float32 CUDA tensor")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} rows must be contiguous (stride(1) == 1)")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name} must have {cols} columns")


class Dictionary:
    """A dictionary prepared once (norms, Gram matrix A^T A, padded and BF16 copies)
    and shared between solves. A is atom-major: shape (N, M), row n = atom a_n."""

    def __init__(self, A: torch.Tensor, precision: str = "fp32", stream=None):
        _check_matrix(A, "A")
        lib = load()
        self.A = A
        self.N, self.M = A.shape
        self.precision = precision
        p = PREC[precision]
        nbytes = lib.omp_dict_size(self.M, self.N, p)
        if nbytes == 0:
            raise ValueError("invalid dictionary shape")
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        self.struct = OmpDictStruct()
        with torch.cuda.device(A.device):
            rc = lib.omp_dict_init(ctypes.byref(self.struct), _ptr(A), self.M, self.N, A.stride(0), p,
                                   _ptr(self.mem), nbytes, _stream_handle(stream, A.device))
        if rc != OMP_OK:
            raise OmpError(rc, "omp_dict_init")


Result = namedtuple("Result", "X support coef status rnorm")


def workspace_bytes(M: int, N: int, B: int, S: int, precision: str = "fp32", with_dict: bool = False,
                    tile_config: int = 0) -> int:
    lib = load()
    o = OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(o))
    o.precision = PREC[precision]
    o.tile_config = int(tile_config)
    d = OmpDictStruct()
    if with_dict:
        o.dict = ctypes.pointer(d)
    return int(lib.omp_workspace_size(M, N, B, S, ctypes.byref(o)))


def solve(A: torch.Tensor, Y: torch.Tensor, S: int, eps: float = 0.0, *, precision: str = "fp32",
          dictionary: Optional[Dictionary] = None, S_per_signal: Optional[torch.Tensor] = None,
          eps_per_signal: Optional[torch.Tensor] = None, dense: bool = True,
          workspace: Optional[torch.Tensor] = None, out: Optional[Result] = None, stream=None,
          timing: Optional[dict] = None, tile_config: int = 0) -> Result:
    """Batched OMP (Algorithm 1) on the GPU.

    A: (N, M) float32 atom-major dictionary; Y: (B, M) float32 signals.
    Returns Result(X (B,N) dense or None, support (B,S) int32 -1 padded,
    coef (B,S) float32, status (B,) int32 = (k << 8) | bits, rnorm (B,) float32).
    Work is enqueued on `stream` (default: torch's current stream); the call does
    not synchronise, unless `timing` is a dict: then each kernel launch is timed
    with HIP events inside the library, the call waits for the stream, and
    timing[phase] accumulates (milliseconds, launches) per phase.
    """
    _check_matrix(A, "A")
    N, M = A.shape
    _check_matrix(Y, "Y", M)
    B = Y.shape[0]
    dev = A.device
    lib = load()
    o = OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(o))
    o.precision = PREC[precision]
    o.tile_config = int(tile_config)
    if dictionary is not None:
        if dictionary.A is not A or dictionary.precision != precision:
            raise ValueError("dictionary was prepared for another A or precision")
        o.dict = ctypes.pointer(dictionary.struct)
    if S_per_signal is not None:
        if S_per_signal.dtype != torch.int32 or S_per_signal.shape != (B,) or not S_per_signal.is_contiguous():
            raise TypeError("S_per_signal must be a contiguous int32 tensor of shape (B,)")
        o.S_per_signal = _ptr(S_per_signal)
    if eps_per_signal is not None:
        if eps_per_signal.dtype != torch.float32 or eps_per_signal.shape != (B,) or not eps_per_signal.is_contiguous():
            raise TypeError("eps_per_signal must be a contiguous float32 tensor of shape (B,)")
        o.eps_per_signal = _ptr(eps_per_signal)
    if out is None:
        X = torch.empty((B, N), dtype=torch.float32, device=dev) if dense else None
        sup = torch.empty((B, S), dtype=torch.int32, device=dev)
        coef = torch.empty((B, S), dtype=torch.float32, device=dev)
        status = torch.empty(B, dtype=torch.int32, device=dev)
        rnorm = torch.empty(B, dtype=torch.float32, device=dev)
        out = Result(X, sup, coef, status, rnorm)
    o.status_out = _ptr(out.status)
    o.rnorm_out = _ptr(out.rnorm)
    o.coef_out = _ptr(out.coef)
    need = lib.omp_workspace_size(M, N, B, S, ctypes.byref(o))
    if need == 0:
        raise OmpError(OMP_EINVAL, "omp_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    o.workspace = _ptr(workspace)
    o.workspace_bytes = workspace.numel()
    if timing is not None:
        ms = (ctypes.c_float * NPHASE)()
        nl = (ctypes.c_int32 * NPHASE)()
        o.phase_ms = ms
        o.phase_launches = nl
    with torch.cuda.device(dev):
        rc = lib.omp_solve(_ptr(A), M, N, A.stride(0), _ptr(Y), B, Y.stride(0), int(S), float(eps),
                           _ptr(out.X), _ptr(out.support), ctypes.byref(o), _stream_handle(stream, dev))
    if rc != OMP_OK:
        raise OmpError(rc, "omp_solve")
    if timing is not None:
        for p, name in enumerate(PHASES):
            t0, n0 = timing.get(name, (0.0, 0))
            timing[name] = (t0 + float(ms[p]), n0 + int(nl[p]))
    return out
