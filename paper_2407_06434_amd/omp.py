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
PREC = {"fp32": 0, "bf16": 1, "fp64": 2, "fp16": 3}
NPHASE = 6
PHASES = ("dict", "init", "corr", "update", "output", "residual")
SIG_EPS, SIG_SMAX, SIG_DEPENDENT, SIG_NONFINITE, SIG_EXHAUSTED, SIG_WIDENED = 1, 2, 4, 8, 32, 64
SIG_NEARTIE = 16

EXPORTED = ("omp_dict_size", "omp_dict_init", "omp_opts_default", "omp_workspace_size", "omp_solve",
            "omp_status_string", "omp_last_hip_error", "omp_version", "omp_multi_workspace_size",
            "omp_solve_multi", "omp_tune", "omp_mlp_size", "omp_mlp_init", "omp_mlp_export",
            "omp_mlp_workspace_size", "omp_mlp_features", "omp_mlp_forward", "omp_mlp_grad", "omp_mlp_train_step",
            "omp_learned_workspace_size", "omp_learned_solve", "omp_solve_noalloc", "omp_noalloc_max_bytes")
SIG_LEARNED = 128
OMP_MAX_PROBLEMS = 8


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
                ("phase_launches", ctypes.POINTER(ctypes.c_int32)), ("use_graph", ctypes.c_int32),
                ("gram_on_the_fly", ctypes.c_int32), ("refactor", ctypes.c_int32),
                ("gram_domain", ctypes.c_int32), ("flag_near_ties", ctypes.c_int32), ("v0", ctypes.c_int32)]


class OmpProblemStruct(ctypes.Structure):
    _fields_ = [("dict", ctypes.POINTER(OmpDictStruct)), ("Y", ctypes.c_void_p), ("B", ctypes.c_int64),
                ("ldy", ctypes.c_int64), ("S", ctypes.c_int32), ("eps", ctypes.c_float),
                ("S_per_signal", ctypes.c_void_p), ("eps_per_signal", ctypes.c_void_p),
                ("support_out", ctypes.c_void_p), ("coef_out", ctypes.c_void_p), ("X_out", ctypes.c_void_p),
                ("status_out", ctypes.c_void_p), ("rnorm_out", ctypes.c_void_p),
                ("tile_config", ctypes.c_int32), ("slots", ctypes.c_int32), ("residual_lanes", ctypes.c_int32)]


class OmpMultiOptsStruct(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("iters_per_graph", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("elapsed_ms", ctypes.POINTER(ctypes.c_float)), ("iterations", ctypes.POINTER(ctypes.c_int32))]


class OmpMlpStruct(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("step", ctypes.c_int64), ("mem", ctypes.c_void_p),
                ("bytes", ctypes.c_size_t)]


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
    PP = ctypes.POINTER(OmpProblemStruct)
    PO = ctypes.POINTER(OmpMultiOptsStruct)
    lib.omp_multi_workspace_size.restype = SZ
    lib.omp_multi_workspace_size.argtypes = [PP, I32, PO]
    lib.omp_solve_multi.restype = ctypes.c_int
    lib.omp_solve_multi.argtypes = [PP, I32, PO, P]
    lib.omp_tune.restype = ctypes.c_int
    lib.omp_tune.argtypes = [PP, I32, PO, I64, P]
    PM = ctypes.POINTER(OmpMlpStruct)
    PD = ctypes.POINTER(OmpDictStruct)
    P6 = ctypes.POINTER(ctypes.c_void_p)
    lib.omp_mlp_size.restype = SZ
    lib.omp_mlp_size.argtypes = [I32, I32, I32]
    lib.omp_mlp_init.restype = ctypes.c_int
    lib.omp_mlp_init.argtypes = [PM, I32, I32, I32, P6, P, SZ, P]
    lib.omp_mlp_export.restype = ctypes.c_int
    lib.omp_mlp_export.argtypes = [PM, P6, P]
    lib.omp_mlp_workspace_size.restype = SZ
    lib.omp_mlp_workspace_size.argtypes = [PM, I64, I64]
    lib.omp_mlp_features.restype = ctypes.c_int
    lib.omp_mlp_features.argtypes = [PD, P, I64, I64, P, PM, P, SZ, P]
    lib.omp_mlp_forward.restype = ctypes.c_int
    lib.omp_mlp_forward.argtypes = [PM, P, I64, P, P, SZ, P]
    lib.omp_mlp_grad.restype = ctypes.c_int
    lib.omp_mlp_grad.argtypes = [PM, P, P, P, I64, I32, P, P6, P, SZ, P]
    lib.omp_mlp_train_step.restype = ctypes.c_int
    lib.omp_mlp_train_step.argtypes = [PM, P, P, P, I64, I32, ctypes.c_float, P, P, SZ, P]
    lib.omp_learned_workspace_size.restype = SZ
    lib.omp_learned_workspace_size.argtypes = [PD, PM, I64, I32, ctypes.POINTER(OmpOptsStruct)]
    lib.omp_learned_solve.restype = ctypes.c_int
    lib.omp_learned_solve.argtypes = [PD, PM, P, I64, I64, I32, ctypes.c_float, P, P, P, P, P,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(OmpOptsStruct), P, SZ, P]
    lib.omp_solve_noalloc.restype = ctypes.c_int
    lib.omp_solve_noalloc.argtypes = lib.omp_solve.argtypes
    lib.omp_noalloc_max_bytes.restype = SZ
    lib.omp_noalloc_max_bytes.argtypes = []
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


def _used_on(stream: Optional[torch.cuda.Stream], *tensors) -> None:
    """Tells torch's caching allocator that `tensors` (allocated here, on torch's
    current stream) are used by work enqueued on `stream`: their memory is then
    not handed out again before that work is done, even if they are freed first."""
    if stream is None:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


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
        _used_on(stream, self.mem)


Result = namedtuple("Result", "X support coef status rnorm")


def workspace_bytes(M: int, N: int, B: int, S: int, precision: str = "fp32", with_dict: bool = False,
                    tile_config: int = 0, gram_domain=False, flag_near_ties: bool = False, v0: bool = False) -> int:
    lib = load()
    o = OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(o))
    o.precision = PREC[precision]
    o.tile_config = int(tile_config)
    o.gram_domain = 2 if gram_domain == "auto" else (1 if gram_domain else 0)
    o.flag_near_ties = 1 if flag_near_ties else 0
    o.v0 = 1 if v0 else 0
    d = OmpDictStruct()
    if with_dict:
        o.dict = ctypes.pointer(d)
    return int(lib.omp_workspace_size(M, N, B, S, ctypes.byref(o)))


def solve(A: torch.Tensor, Y: torch.Tensor, S: int, eps: float = 0.0, *, precision: str = "fp32",
          dictionary: Optional[Dictionary] = None, S_per_signal: Optional[torch.Tensor] = None,
          eps_per_signal: Optional[torch.Tensor] = None, dense: bool = True,
          workspace: Optional[torch.Tensor] = None, out: Optional[Result] = None, stream=None,
          timing: Optional[dict] = None, tile_config: int = 0, graph: bool = True,
          gram_on_the_fly: bool = False, refactor: bool = False, gram_domain=False,
          flag_near_ties: bool = False, v0: bool = False) -> Result:
    """Batched OMP (Algorithm 1) on the GPU.

    A: (N, M) float32 atom-major dictionary; Y: (B, M) float32 signals.
    Returns Result(X (B,N) dense or None, support (B,S) int32 -1 padded,
    coef (B,S) float32, status (B,) int32 = (k << 8) | bits, rnorm (B,) float32).
    Work is enqueued on `stream` (default: torch's current stream); the call does
    not synchronise, unless `timing` is a dict: then each kernel launch is timed
    with HIP events inside the library, the call waits for the stream, and
    timing[phase] accumulates (milliseconds, launches) per phase. With `graph` (default)
    the library replays the solve from a captured hipGraph cached per argument set.
    `gram_on_the_fly` (ablation only) computes each pick's Gram row from the atoms
    instead of reading the prepared Gram matrix; `refactor` (ablation only) rebuilds
    the Cholesky factor of the support's Gram block at every step instead of
    appending one row to it. `gram_domain` (FP32 only) takes each step's correlations
    from P = A^T y and the Gram matrix instead of from residual vectors;
    gram_domain="auto" picks that form for FP32 solves with 4M >= N, except
    dictionaries under 1 MiB in batches of more than 4096 signals.
    `flag_near_ties` sets status bit SIG_NEARTIE on signals where, at some step, the
    runner-up atom scored within 1e-5 (relative) of the picked one. `v0` (FP32 only)
    runs the paper's Algorithm v0 (inverse Cholesky factor and D = A^T Q).
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
    o.use_graph = 1 if graph else 0
    o.gram_on_the_fly = 1 if gram_on_the_fly else 0
    o.refactor = 1 if refactor else 0
    o.gram_domain = 2 if gram_domain == "auto" else (1 if gram_domain else 0)
    o.flag_near_ties = 1 if flag_near_ties else 0
    o.v0 = 1 if v0 else 0
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
    _used_on(stream, workspace, *out)
    if timing is not None:
        for p, name in enumerate(PHASES):
            t0, n0 = timing.get(name, (0.0, 0))
            timing[name] = (t0 + float(ms[p]), n0 + int(nl[p]))
    return out


def solve_noalloc(A: torch.Tensor, Y: torch.Tensor, S: int, eps: float = 0.0, *, precision: str = "fp32",
                  dictionary: Optional[Dictionary] = None, S_per_signal: Optional[torch.Tensor] = None,
                  eps_per_signal: Optional[torch.Tensor] = None, dense: bool = True,
                  out: Optional[Result] = None, stream=None, tile_config: int = 0, gram_domain=False,
                  v0: bool = False) -> Result:
    """omp_solve_noalloc: the solve of `solve` with the library's static device scratch as
    its workspace (no workspace tensor; the library allocates nothing). Outputs are
    allocated here unless `out` is given. Calls overlapping on one GPU race."""
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
    o.gram_domain = 2 if gram_domain == "auto" else (1 if gram_domain else 0)
    o.v0 = 1 if v0 else 0
    if dictionary is not None:
        if dictionary.A is not A or dictionary.precision != precision:
            raise ValueError("dictionary was prepared for another A or precision")
        o.dict = ctypes.pointer(dictionary.struct)
    for name, t, dt in (("S_per_signal", S_per_signal, torch.int32), ("eps_per_signal", eps_per_signal,
                                                                       torch.float32)):
        if t is not None and (t.dtype != dt or t.shape != (B,) or not t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous {dt} tensor of shape (B,)")
    o.S_per_signal = _ptr(S_per_signal)
    o.eps_per_signal = _ptr(eps_per_signal)
    if out is None:
        out = Result(torch.empty((B, N), dtype=torch.float32, device=dev) if dense else None,
                     torch.empty((B, S), dtype=torch.int32, device=dev),
                     torch.empty((B, S), dtype=torch.float32, device=dev),
                     torch.empty(B, dtype=torch.int32, device=dev), torch.empty(B, dtype=torch.float32, device=dev))
    o.status_out = _ptr(out.status)
    o.rnorm_out = _ptr(out.rnorm)
    o.coef_out = _ptr(out.coef)
    with torch.cuda.device(dev):
        rc = lib.omp_solve_noalloc(_ptr(A), M, N, A.stride(0), _ptr(Y), B, Y.stride(0), int(S), float(eps),
                                   _ptr(out.X), _ptr(out.support), ctypes.byref(o), _stream_handle(stream, dev))
    if rc != OMP_OK:
        raise OmpError(rc, "omp_solve_noalloc")
    _used_on(stream, *out)
    return out


class Problem:
    """One batch of an uneven multi-problem solve: signals Y (B, M) over a prepared
    dictionary, with optional per-signal S and eps. `tile_config`, `slots` and
    `residual_lanes` are the schedule (0 = by shape; tune() fills them)."""

    def __init__(self, dictionary: Dictionary, Y: torch.Tensor, S: int, eps: float = 0.0,
                 S_per_signal: Optional[torch.Tensor] = None, eps_per_signal: Optional[torch.Tensor] = None,
                 dense: bool = False, tile_config: int = 0, slots: int = 0, residual_lanes: int = 0):
        _check_matrix(Y, "Y", dictionary.M)
        B = Y.shape[0]
        dev = Y.device
        for name, t, dt in (("S_per_signal", S_per_signal, torch.int32), ("eps_per_signal", eps_per_signal,
                                                                           torch.float32)):
            if t is not None and (t.dtype != dt or t.shape != (B,) or not t.is_contiguous() or not t.is_cuda):
                raise TypeError(f"{name} must be a contiguous {dt} CUDA tensor of shape (B,)")
        self.dictionary, self.Y, self.S, self.eps = dictionary, Y, int(S), float(eps)
        self.S_per_signal, self.eps_per_signal = S_per_signal, eps_per_signal
        self.tile_config, self.slots, self.residual_lanes = int(tile_config), int(slots), int(residual_lanes)
        self.out = Result(torch.empty((B, dictionary.N), dtype=torch.float32, device=dev) if dense else None,
                          torch.empty((B, self.S), dtype=torch.int32, device=dev),
                          torch.empty((B, self.S), dtype=torch.float32, device=dev),
                          torch.empty(B, dtype=torch.int32, device=dev),
                          torch.empty(B, dtype=torch.float32, device=dev))

    def struct(self) -> OmpProblemStruct:
        p = OmpProblemStruct()
        p.dict = ctypes.pointer(self.dictionary.struct)
        p.Y = self.Y.data_ptr()
        p.B = self.Y.shape[0]
        p.ldy = self.Y.stride(0)
        p.S = self.S
        p.eps = self.eps
        p.S_per_signal = None if self.S_per_signal is None else self.S_per_signal.data_ptr()
        p.eps_per_signal = None if self.eps_per_signal is None else self.eps_per_signal.data_ptr()
        p.support_out = self.out.support.data_ptr()
        p.coef_out = self.out.coef.data_ptr()
        p.X_out = None if self.out.X is None else self.out.X.data_ptr()
        p.status_out = self.out.status.data_ptr()
        p.rnorm_out = self.out.rnorm.data_ptr()
        p.tile_config, p.slots, p.residual_lanes = self.tile_config, self.slots, self.residual_lanes
        return p


def _multi_call(problems, precision, iters_per_graph, workspace):
    if not 1 <= len(problems) <= OMP_MAX_PROBLEMS:
        raise ValueError(f"1..{OMP_MAX_PROBLEMS} problems")
    precs = {p.dictionary.precision for p in problems}
    if precs != {precision}:
        raise ValueError("every dictionary must be prepared for the solve's precision")
    lib = load()
    arr = (OmpProblemStruct * len(problems))(*[p.struct() for p in problems])
    o = OmpMultiOptsStruct()
    o.precision = PREC[precision]
    o.iters_per_graph = int(iters_per_graph)
    need = lib.omp_multi_workspace_size(arr, len(problems), ctypes.byref(o))
    if need == 0:
        raise OmpError(OMP_EINVAL, "omp_multi_workspace_size")
    dev = problems[0].Y.device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    o.workspace = workspace.data_ptr()
    o.workspace_bytes = workspace.numel()
    return lib, arr, o, dev, workspace


def solve_multi(problems, precision: str = "fp32", iters_per_graph: int = 0, workspace=None, stream=None,
                info: Optional[dict] = None):
    """Solve several OMP problems together with the slot scheduler (waits for the
    result). Returns each problem's Result; `info` receives elapsed_ms and iterations."""
    lib, arr, o, dev, workspace = _multi_call(problems, precision, iters_per_graph, workspace)
    ms = ctypes.c_float(0.0)
    it = ctypes.c_int32(0)
    o.elapsed_ms = ctypes.pointer(ms)
    o.iterations = ctypes.pointer(it)
    with torch.cuda.device(dev):
        rc = lib.omp_solve_multi(arr, len(problems), ctypes.byref(o), _stream_handle(stream, dev))
    if rc != OMP_OK:
        raise OmpError(rc, "omp_solve_multi")
    if info is not None:
        info["elapsed_ms"] = float(ms.value)
        info["iterations"] = int(it.value)
    return [p.out for p in problems]


def tune(problems, precision: str = "fp32", sample: int = 0, iters_per_graph: int = 0, workspace=None,
         stream=None):
    """Autotune each problem's schedule (tile configuration, slots, residual lanes) on
    its first `sample` signals; writes the choices into the Problem objects."""
    for p in problems:
        if p.slots == 0:
            p.slots = min(8192, ((p.Y.shape[0] + 255) // 256) * 256)
    lib, arr, o, dev, workspace = _multi_call(problems, precision, iters_per_graph, workspace)
    with torch.cuda.device(dev):
        rc = lib.omp_tune(arr, len(problems), ctypes.byref(o), int(sample), _stream_handle(stream, dev))
    if rc != OMP_OK:
        raise OmpError(rc, "omp_tune")
    for p, st in zip(problems, arr):
        p.tile_config, p.slots, p.residual_lanes = int(st.tile_config), int(st.slots), int(st.residual_lanes)
    return [(p.tile_config, p.slots, p.residual_lanes) for p in problems]


PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


class MLP:
    """The support-proposal network on the GPU (weights, BF16 copies and Adam state in
    one device allocation). `params` maps W1 (n_hidden, n_in), b1, W2 (n_hidden,
    n_hidden), b2, W3 (n_out, n_hidden), b3 to float32 arrays or tensors (the initial
    values, drawn by the caller)."""

    def __init__(self, params: dict, device="cuda:0", stream=None):
        lib = load()
        self.device = torch.device(device)
        t = {k: torch.as_tensor(params[k], dtype=torch.float32).to(self.device).contiguous() for k in PARAM_NAMES}
        n_hidden, n_in = t["W1"].shape
        n_out = t["W3"].shape[0]
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        nbytes = lib.omp_mlp_size(n_in, n_hidden, n_out)
        if nbytes == 0:
            raise ValueError("network sizes must be multiples of 256")
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.struct = OmpMlpStruct()
        ptrs = (ctypes.c_void_p * 6)(*[t[k].data_ptr() for k in PARAM_NAMES])
        with torch.cuda.device(self.device):
            rc = lib.omp_mlp_init(ctypes.byref(self.struct), n_in, n_hidden, n_out, ptrs, _ptr(self.mem), nbytes,
                                  _stream_handle(stream, self.device))
            torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()
        if rc != OMP_OK:
            raise OmpError(rc, "omp_mlp_init")
        self._ws = None

    def _workspace(self, M, B):
        need = load().omp_mlp_workspace_size(ctypes.byref(self.struct), M, B)
        if need == 0:
            raise OmpError(OMP_EINVAL, "omp_mlp_workspace_size")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def export(self, stream=None) -> dict:
        out = {"W1": torch.empty((self.n_hidden, self.n_in)), "b1": torch.empty(self.n_hidden),
               "W2": torch.empty((self.n_hidden, self.n_hidden)), "b2": torch.empty(self.n_hidden),
               "W3": torch.empty((self.n_out, self.n_hidden)), "b3": torch.empty(self.n_out)}
        out = {k: v.to(self.device) for k, v in out.items()}
        ptrs = (ctypes.c_void_p * 6)(*[out[k].data_ptr() for k in PARAM_NAMES])
        with torch.cuda.device(self.device):
            rc = load().omp_mlp_export(ctypes.byref(self.struct), ptrs, _stream_handle(stream, self.device))
        if rc != OMP_OK:
            raise OmpError(rc, "omp_mlp_export")
        _used_on(stream, *out.values())
        return out

    def features(self, dictionary: Dictionary, Y: torch.Tensor, stream=None) -> torch.Tensor:
        """f[b, n] = a_n^T y_b / (||a_n|| ||y_b||) as BF16 bits (int16 tensor, shape (B, N))."""
        _check_matrix(Y, "Y", dictionary.M)
        B = Y.shape[0]
        F = torch.empty((B, dictionary.N), dtype=torch.int16, device=self.device)
        ws = self._workspace(dictionary.M, B)
        with torch.cuda.device(self.device):
            rc = load().omp_mlp_features(ctypes.byref(dictionary.struct), _ptr(Y), B, Y.stride(0), _ptr(F),
                                         ctypes.byref(self.struct), _ptr(ws), ws.numel(),
                                         _stream_handle(stream, self.device))
        if rc != OMP_OK:
            raise OmpError(rc, "omp_mlp_features")
        _used_on(stream, ws, F)
        return F

    def forward(self, F: torch.Tensor, stream=None) -> torch.Tensor:
        B = F.shape[0]
        Z = torch.empty((B, self.n_out), dtype=torch.float32, device=self.device)
        ws = self._workspace(0, B)
        with torch.cuda.device(self.device):
            rc = load().omp_mlp_forward(ctypes.byref(self.struct), _ptr(F.contiguous()), B, _ptr(Z), _ptr(ws),
                                        ws.numel(), _stream_handle(stream, self.device))
        if rc != OMP_OK:
            raise OmpError(rc, "omp_mlp_forward")
        _used_on(stream, ws, Z)
        return Z

    def grad(self, F: torch.Tensor, support: torch.Tensor, rows: Optional[torch.Tensor] = None, stream=None):
        """(loss tensor [1], dict of FP32 gradients) on one batch (rows `rows` of F and
        support, default all); the network is unchanged."""
        S = support.shape[1]
        B = support.shape[0] if rows is None else rows.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        g = {k: torch.empty(v, dtype=torch.float32, device=self.device) for k, v in
             (("W1", (self.n_hidden, self.n_in)), ("b1", (self.n_hidden,)), ("W2", (self.n_hidden, self.n_hidden)),
              ("b2", (self.n_hidden,)), ("W3", (self.n_out, self.n_hidden)), ("b3", (self.n_out,)))}
        ptrs = (ctypes.c_void_p * 6)(*[g[k].data_ptr() for k in PARAM_NAMES])
        ws = self._workspace(0, B)
        with torch.cuda.device(self.device):
            rc = load().omp_mlp_grad(ctypes.byref(self.struct), _ptr(F.contiguous()), _ptr(support.contiguous()),
                                     _ptr(rows), B, S, _ptr(loss), ptrs, _ptr(ws), ws.numel(),
                                     _stream_handle(stream, self.device))
        if rc != OMP_OK:
            raise OmpError(rc, "omp_mlp_grad")
        _used_on(stream, ws, loss, *g.values())
        return loss, g

    def train_step(self, F: torch.Tensor, support: torch.Tensor, lr: float, loss: Optional[torch.Tensor] = None,
                   rows: Optional[torch.Tensor] = None, stream=None):
        """One Adam step on rows `rows` (int32 device tensor, default all) of F and support.
        `loss` (a one-element float32 device tensor or view) receives the batch loss."""
        S = support.shape[1]
        B = support.shape[0] if rows is None else rows.shape[0]
        ws = self._workspace(0, B)
        with torch.cuda.device(self.device):
            rc = load().omp_mlp_train_step(ctypes.byref(self.struct), _ptr(F), _ptr(support), _ptr(rows), B, S,
                                           float(lr), _ptr(loss), _ptr(ws), ws.numel(),
                                           _stream_handle(stream, self.device))
        if rc != OMP_OK:
            raise OmpError(rc, "omp_mlp_train_step")
        _used_on(stream, ws)
        return loss


def learned_solve(dictionary: Dictionary, mlp: MLP, Y: torch.Tensor, S: int, eps: float = 0.0,
                  eps_per_signal: Optional[torch.Tensor] = None, tile_config: int = 0, workspace=None, stream=None):
    """Proposal + least-squares check, plain OMP for the rejects. Returns (Result with
    X None, number accepted). Waits for the stream once."""
    _check_matrix(Y, "Y", dictionary.M)
    B = Y.shape[0]
    dev = Y.device
    lib = load()
    o = OmpOptsStruct()
    lib.omp_opts_default(ctypes.byref(o))
    o.precision = PREC[dictionary.precision]
    o.tile_config = int(tile_config)
    need = lib.omp_learned_workspace_size(ctypes.byref(dictionary.struct), ctypes.byref(mlp.struct), B, int(S),
                                          ctypes.byref(o))
    if need == 0:
        raise OmpError(OMP_EINVAL, "omp_learned_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    out = Result(None, torch.empty((B, S), dtype=torch.int32, device=dev),
                 torch.empty((B, S), dtype=torch.float32, device=dev), torch.empty(B, dtype=torch.int32, device=dev),
                 torch.empty(B, dtype=torch.float32, device=dev))
    acc = ctypes.c_int64(0)
    if eps_per_signal is not None and (eps_per_signal.dtype != torch.float32 or eps_per_signal.shape != (B,)):
        raise TypeError("eps_per_signal must be float32 of shape (B,)")
    with torch.cuda.device(dev):
        rc = lib.omp_learned_solve(ctypes.byref(dictionary.struct), ctypes.byref(mlp.struct), _ptr(Y), B,
                                   Y.stride(0), int(S), float(eps), _ptr(eps_per_signal), _ptr(out.support),
                                   _ptr(out.coef), _ptr(out.status), _ptr(out.rnorm), ctypes.byref(acc),
                                   ctypes.byref(o), _ptr(workspace), workspace.numel(),
                                   _stream_handle(stream, dev))
    if rc != OMP_OK:
        raise OmpError(rc, "omp_learned_solve")
    _used_on(stream, workspace, *out)
    return out, int(acc.value)
