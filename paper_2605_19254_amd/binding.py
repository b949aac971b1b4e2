"""ctypes binding of librns.so (the C ABI declared in include/rns.h).

Argument marshalling only: device tensors are passed by pointer and stride,
streams as torch's current HIP stream.  Every step of the computation runs in
the library's HIP kernels; there is no fallback.  Importing this module on a
tree without the built library raises ImportError.

Residue planes are torch.int32 tensors (values in [0, 2^26) fit) of shape
[L, rows, cols]; the C ABI sees them as uint32.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librns.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("librns.so is not built (run __graft_entry__.build() or "
                      "python paper_2605_19254_amd/build.py)")



def _preload_torch_hip_runtime():
    """Load the HIP runtime that torch carries (if any) with RTLD_GLOBAL before
    librns, so that librns binds to the same runtime as torch: one process must
    not drive the GPU through two HIP runtimes."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return None
    path = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    if os.path.exists(path):
        ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
        return path
    return None


HIP_RUNTIME = _preload_torch_hip_runtime()
_lib = ctypes.CDLL(LIB_PATH)


def loaded_hip_runtimes():
    """Paths of every libamdhip64 mapped into this process (should be one)."""
    out = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    out.add(line.split()[-1])
    except OSError:
        pass
    return sorted(out)

OK, EINVAL, ENOMEM, EDEVICE, EBOUND, EOVERFLOW, ESINGULAR, ERETRY, ENOTSUP, EPENDING, ESCRATCH = range(11)
PATH_AUTO, PATH_FP64, PATH_INT8 = 0, 1, 2
_PATHS = {"auto": PATH_AUTO, "fp64": PATH_FP64, "int8": PATH_INT8}
CTX_SEPARATE_CRT = 4          # rns_ctx_create flag
I8_HALF_CRT = 5               # plan info variant of a plan that fuses the CRT into the GEMM

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int


class RnsGemmDesc(ctypes.Structure):
    _fields_ = [("m", _I64), ("n", _I64), ("k", _I64),
                ("A", _P), ("lda", _I64), ("a_plane_stride", _I64),
                ("B", _P), ("ldb", _I64), ("b_plane_stride", _I64),
                ("C", _P), ("ldc", _I64), ("c_plane_stride", _I64),
                ("prime_begin", ctypes.c_int32), ("L", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RnsSmithStats(ctypes.Structure):
    _fields_ = [("t_lif", ctypes.c_double), ("t_im", ctypes.c_double),
                ("t_uc", ctypes.c_double), ("t_total", ctypes.c_double),
                ("restarts", _I32), ("lift_steps", _I32), ("products", _I64),
                ("residue_ops", ctypes.c_double), ("cert_primes", _I32),
                ("columns", _I32), ("path", _I32), ("cert_exact", _I32),
                ("lift_a_bytes", _I32), ("lift_kernels", _I32), ("t_host_cpu", ctypes.c_double),
                ("batches", _I32), ("cert_kind", _I32), ("uc_steps", _I32), ("uc_rejects", _I32),
                ("uc_dim", _I64), ("t_uc_cert", ctypes.c_double), ("uc_x_primes", _I32), ("uc_lambda", _I32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_lib_strerror = _sig("rns_strerror", ctypes.c_char_p, [_I32])
_lib_primes_below = _sig("rns_primes_below", _I32, [ctypes.c_uint64, _I32, _P])
_lib_ctx_create = _sig("rns_ctx_create", _I32, [ctypes.POINTER(_P), _I32, _P, _I32, ctypes.c_uint64])
_lib_ctx_destroy = _sig("rns_ctx_destroy", None, [_P])
_lib_ctx_num_primes = _sig("rns_ctx_num_primes", _I32, [_P])
_lib_ctx_primes = _sig("rns_ctx_primes", _I32, [_P, _P])
_lib_ctx_reserve = _sig("rns_ctx_reserve", _I32, [_P, ctypes.c_size_t])
_lib_workspace_bytes = _sig("rns_workspace_bytes", _I32,
                            [_P, ctypes.POINTER(RnsGemmDesc), _I32, _I32, ctypes.POINTER(ctypes.c_size_t)])
_lib_primes_for_bound = _sig("rns_primes_for_bound", _I32, [_P, _P, _I32, ctypes.POINTER(_I32)])
_lib_reduce = _sig("rns_reduce", _I32, [_P, _P, _I64, _I64, _I64, _I32, _I32, _P, _I64, _I64, _P])
_lib_reduce_mw = _sig("rns_reduce_mw", _I32, [_P, _P, _I32, _I64, _I64, _I64, _I32, _I32, _P, _I64, _I64, _P])
_lib_modmatmul = _sig("modmatmul_batched", _I32, [_P, ctypes.POINTER(RnsGemmDesc), _I32, _I32, _P])
_lib_modmatmul_noalloc = _sig("modmatmul_batched_noalloc", _I32, [_P, ctypes.POINTER(RnsGemmDesc), _I32, _I32, _P])
_lib_noalloc_bytes = _sig("rns_noalloc_scratch_bytes", _I32, [ctypes.POINTER(ctypes.c_size_t)])
_lib_crt = _sig("crt_reconstruct", _I32, [_P, _P, _I64, _I64, _I64, _I64, _I32, _I32, _P, _I32,
                                          _P, _I32, _I64, _P, _P])
_lib_status = _sig("rns_ctx_status", _I32, [_P, _P])
_lib_convert = _sig("rns_base_convert", _I32, [_P, _P, _I64, _I64, _I64, _I64, _I32, _I32, _P, _I32,
                                               _P, _I64, _I64, _I32, _I32, _P, _P])
_lib_force = _sig("rns_ctx_force_cert_failures", _I32, [_P, _I32])
_lib_smith_path = _sig("rns_ctx_set_smith_path", _I32, [_P, _I32])
_lib_smith = _sig("smith_form", _I32, [_P, _P, _I64, ctypes.c_uint64, ctypes.POINTER(_P)])
_lib_lif = _sig("rns_largest_invariant", _I32, [_P, _P, _I64, ctypes.c_uint64, ctypes.POINTER(_P)])
_lib_smith_get = _sig("rns_smith_get", _I32, [_P, _I64, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint64)),
                                              ctypes.POINTER(_I32)])
_lib_smith_size = _sig("rns_smith_size", _I64, [_P])
_lib_smith_stats = _sig("rns_smith_stats_get", _I32, [_P, ctypes.POINTER(RnsSmithStats)])
_lib_smith_free = _sig("rns_smith_free", None, [_P])
_lib_massager = _sig("rns_smith_massager", _I32, [_P, _P, _I64, ctypes.c_uint64, ctypes.POINTER(_P)])
_lib_massager_width = _sig("rns_smith_massager_width", _I32, [_P, _I32, _I64])
_lib_massager_vector = _sig("rns_smith_massager_vector", _I32, [_P, _I32, _I64, _P, _I32])


class RnsUnimodInfo(ctypes.Structure):
    _fields_ = [("verdict", _I32), ("reason", _I32), ("steps", _I32), ("steps_needed", _I32),
                ("x_primes", _I32), ("q_primes", _I32),
                ("x_prime", ctypes.c_uint32 * 4), ("q_prime", ctypes.c_uint32 * 4),
                ("log2_bound", ctypes.c_double), ("log2_x", ctypes.c_double), ("seconds", ctypes.c_double),
                ("residue_ops", ctypes.c_double), ("products", _I32), ("reserved", _I32)]


_lib_unimodular = _sig("rns_unimodular_certify", _I32,
                       [_P, _P, _I64, _I32, _P, ctypes.POINTER(RnsUnimodInfo)])
class RnsPlanInfo(ctypes.Structure):
    _fields_ = [("path", _I32), ("variant", _I32), ("tiles", _I64), ("workspace_bytes", ctypes.c_size_t),
                ("residue_ops", ctypes.c_double)]


class RnsMatmulDesc(ctypes.Structure):
    _fields_ = [("m", _I64), ("n", _I64), ("k", _I64), ("A", _P), ("lda", _I64), ("B", _P), ("ldb", _I64),
                ("C", _P), ("ldc", _I64), ("prime_begin", ctypes.c_int32), ("L", ctypes.c_int32),
                ("bound", ctypes.c_uint64)]


_lib_gplan_create = _sig("rns_gemm_plan_create", _I32, [_P, ctypes.POINTER(RnsGemmDesc), _I32, _I32,
                                                       ctypes.POINTER(_P)])
_lib_gplan_execute = _sig("rns_gemm_plan_execute", _I32, [_P, _P])
_lib_gplan_info = _sig("rns_gemm_plan_info", _I32, [_P, ctypes.POINTER(RnsPlanInfo)])
_lib_gplan_set_variant = _sig("rns_gemm_plan_set_variant", _I32, [_P, _I32])
_lib_gplan_destroy = _sig("rns_gemm_plan_destroy", None, [_P])
_lib_gplan_autotune = _sig("rns_gemm_plan_autotune", _I32, [_P, _P, ctypes.POINTER(_I32)])
_lib_set_tune_cache = _sig("rns_ctx_set_tune_cache", _I32, [_P, ctypes.c_char_p])
_lib_autotune = _sig("rns_autotune", _I32, [_P, ctypes.POINTER(RnsGemmDesc), _I32, _I32, _P,
                                            ctypes.POINTER(_I32)])
_lib_mplan_create = _sig("rns_matmul_plan_create", _I32, [_P, ctypes.POINTER(RnsMatmulDesc), _I32, _I32,
                                                         _I32, ctypes.POINTER(_P)])
_lib_mplan_execute = _sig("rns_matmul_plan_execute", _I32, [_P, _P])
_lib_mplan_info = _sig("rns_matmul_plan_info", _I32, [_P, ctypes.POINTER(RnsPlanInfo)])
_lib_mplan_gemm = _sig("rns_matmul_plan_gemm", _P, [_P])
_lib_mplan_destroy = _sig("rns_matmul_plan_destroy", None, [_P])
class RnsRequestInfo(ctypes.Structure):
    _fields_ = [("status", _I32), ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_end", ctypes.c_double), ("footprint", ctypes.c_size_t), ("worker", _I32)]


class RnsServerStats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_size_t), ("in_use", ctypes.c_size_t), ("high_water", ctypes.c_size_t),
                ("running", _I32), ("max_running", _I32), ("queued", _I32)]


_lib_srv_create = _sig("rns_server_create", _I32, [_I32, _I32, ctypes.c_size_t, ctypes.POINTER(_P)])
_lib_srv_aging = _sig("rns_server_set_aging", _I32, [_P, ctypes.c_double])
_lib_srv_submit = _sig("rns_server_submit", _I32, [_P, _P, _I64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)])
_lib_srv_wait = _sig("rns_server_wait", _I32, [_P, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_P),
                                               ctypes.POINTER(RnsRequestInfo)])
_lib_srv_stats = _sig("rns_server_stats", _I32, [_P, ctypes.POINTER(RnsServerStats)])
_lib_srv_footprint = _sig("rns_server_footprint", _I32, [_I64, ctypes.POINTER(ctypes.c_size_t)])
_lib_srv_destroy = _sig("rns_server_destroy", None, [_P])
_lib_profile = _sig("rns_ctx_profile", _I32, [_P, _I32])
_lib_calibrate = _sig("rns_calibrate", _I32, [_P, _I32, _I32, _I32, _P, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)])
_lib_lift_step = _sig("rns_lift_step", _I32, [_I32, _P, _P, _P, _I64, _I32, ctypes.c_uint32, _I32, _P, _P, _P,
                                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_I32), _P])
_lib_profile_read = _sig("rns_ctx_profile_read", _I32, [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                                        ctypes.POINTER(_I64)])

EXPORTS = ["rns_strerror", "rns_primes_below", "rns_ctx_create", "rns_ctx_destroy",
           "rns_ctx_num_primes", "rns_ctx_primes", "rns_ctx_reserve", "rns_workspace_bytes",
           "rns_primes_for_bound", "rns_reduce", "rns_reduce_mw", "modmatmul_batched", "crt_reconstruct",
           "rns_ctx_status", "smith_form", "rns_smith_get", "rns_smith_size",
           "rns_smith_stats_get", "rns_smith_free", "rns_ctx_force_cert_failures",
           "rns_ctx_profile", "rns_ctx_profile_read", "rns_gemm_plan_create", "rns_gemm_plan_execute",
           "rns_gemm_plan_info", "rns_gemm_plan_set_variant", "rns_gemm_plan_destroy",
           "rns_ctx_set_tune_cache", "rns_autotune", "rns_gemm_plan_autotune", "rns_matmul_plan_create", "rns_matmul_plan_execute",
           "rns_matmul_plan_info", "rns_matmul_plan_gemm", "rns_matmul_plan_destroy",
           "rns_server_create", "rns_server_set_aging", "rns_server_submit", "rns_server_wait",
           "rns_server_stats", "rns_server_footprint", "rns_server_destroy", "rns_calibrate",
           "rns_ctx_set_smith_path", "rns_largest_invariant", "rns_lift_step",
           "modmatmul_batched_noalloc", "rns_noalloc_scratch_bytes", "rns_base_convert",
           "rns_smith_massager", "rns_smith_massager_width", "rns_smith_massager_vector",
           "rns_unimodular_certify"]


class RnsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, rns_strerror(status), status))


def rns_strerror(status: int) -> str:
    return _lib_strerror(status).decode()


def _check(status: int, what: str):
    if status != OK:
        raise RnsError(status, what)


def rns_primes_below(bound: int, count: int) -> List[int]:
    out = (ctypes.c_uint32 * count)()
    _check(_lib_primes_below(bound, count, ctypes.cast(out, _P)), "rns_primes_below")
    return list(out)


def _words(x: int) -> List[int]:
    x = int(x)
    assert x >= 0
    w = []
    while True:
        w.append(x & 0xFFFFFFFFFFFFFFFF)
        x >>= 64
        if not x:
            return w


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t) -> int:
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda, "device tensor expected"
    return t.data_ptr()


class Context:
    """An RNS basis on one GPU (rns_ctx)."""

    def __init__(self, device: int = 0, primes: Optional[Sequence[int]] = None, L: int = 24,
                 path: Optional[str] = None, separate_crt: bool = False):
        """path: None (the library chooses), "fp64" or "int8": what the "auto"
        path resolves to in this context's products (RNS_CTX_PATH_*).
        separate_crt: whole-product plans keep the CRT as a launch of its own
        even where they could fuse it into the GEMM (RNS_CTX_SEPARATE_CRT)."""
        flags = {None: 0, "auto": 0, "fp64": 1, "int8": 2}[path] | (CTX_SEPARATE_CRT if separate_crt else 0)
        h = _P()
        if primes is not None:
            arr = (ctypes.c_uint32 * len(primes))(*[int(p) for p in primes])
            _check(_lib_ctx_create(ctypes.byref(h), device, ctypes.cast(arr, _P), len(primes), flags),
                   "rns_ctx_create")
        else:
            _check(_lib_ctx_create(ctypes.byref(h), device, None, L, flags), "rns_ctx_create")
        self.handle = h
        self.device = device
        n = _lib_ctx_num_primes(h)
        out = (ctypes.c_uint32 * n)()
        _check(_lib_ctx_primes(h, ctypes.cast(out, _P)), "rns_ctx_primes")
        self.primes = list(out)

    def close(self):
        if self.handle:
            _lib_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def L(self) -> int:
        return len(self.primes)

    def reserve(self, nbytes: int):
        _check(_lib_ctx_reserve(self.handle, nbytes), "rns_ctx_reserve")

    def primes_for_bound(self, bound: int) -> int:
        w = _words(bound)
        arr = (ctypes.c_uint64 * len(w))(*w)
        out = _I32()
        _check(_lib_primes_for_bound(self.handle, ctypes.cast(arr, _P), len(w), ctypes.byref(out)),
               "rns_primes_for_bound")
        return out.value

    def status(self, stream=None) -> int:
        return _lib_status(self.handle, _stream(stream))

    def profile(self, enable: bool = True):
        """Bracket every library kernel launch with HIP events."""
        _check(_lib_profile(self.handle, 1 if enable else 0), "rns_ctx_profile")

    def profile_read(self, name: str = ""):
        """(total ms, launches) of traced kernels whose name contains `name`;
        the matching records are consumed."""
        ms = ctypes.c_double()
        cnt = _I64()
        _check(_lib_profile_read(self.handle, name.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
               "rns_ctx_profile_read")
        return ms.value, cnt.value

    CALIBRATE_KINDS = {"i8_16x16x64": 0, "i8_32x32x32": 1, "f64_mfma": 2, "f64_fma": 3}

    def calibrate(self, kind: str, iters: int = 20000, random_operands: bool = True, stream=None):
        """(ops per second, ms) of one unit's sustained rate on this device."""
        rate = ctypes.c_double()
        ms = ctypes.c_double()
        _check(_lib_calibrate(self.handle, self.CALIBRATE_KINDS[kind], iters, 1 if random_operands else 0,
                              _stream(stream), ctypes.byref(rate), ctypes.byref(ms)), "rns_calibrate")
        return rate.value, ms.value

    def set_tune_cache(self, path: str):
        _check(_lib_set_tune_cache(self.handle, path.encode() if path else None), "rns_ctx_set_tune_cache")

    def force_cert_failures(self, count: int):
        _check(_lib_force(self.handle, count), "rns_ctx_force_cert_failures")

    SMITH_PATHS = {"auto": 0, "residue": 1, "lifting": 2}

    def set_smith_path(self, path: str):
        """Which Smith-form path smith_form takes: auto, residue or lifting."""
        _check(_lib_smith_path(self.handle, self.SMITH_PATHS[path]), "rns_ctx_set_smith_path")


def rns_reduce(ctx: Context, x, prime_begin: int = 0, L: Optional[int] = None, out=None, stream=None):
    """x: int64 device tensor (rows, cols), row stride >= cols, unit column
    stride.  Returns int32 residue planes [L, rows, cols]."""
    import torch
    L = ctx.L - prime_begin if L is None else L
    assert x.dtype == torch.int64 and x.dim() == 2 and x.stride(1) == 1
    rows, cols = x.shape
    if out is None:
        out = torch.empty((L, rows, cols), dtype=torch.int32, device=x.device)
    assert out.dtype == torch.int32 and out.stride(2) == 1
    _check(_lib_reduce(ctx.handle, _dev_ptr(x), rows, cols, x.stride(0), prime_begin, L,
                       _dev_ptr(out), out.stride(1), out.stride(0), _stream(stream)), "rns_reduce")
    return out


def rns_reduce_mw(ctx: Context, x, prime_begin: int = 0, L: Optional[int] = None, out=None, stream=None):
    """x: int64 device tensor (rows, cols, W) of two's-complement words, least
    significant first (the layout crt_reconstruct returns), unit stride over
    the last two dimensions.  Returns int32 residue planes [L, rows, cols]."""
    import torch
    L = ctx.L - prime_begin if L is None else L
    assert x.dtype == torch.int64 and x.dim() == 3 and x.stride(2) == 1 and x.stride(1) == x.shape[2]
    rows, cols, W = x.shape
    if out is None:
        out = torch.empty((L, rows, cols), dtype=torch.int32, device=x.device)
    assert out.dtype == torch.int32 and out.stride(2) == 1
    _check(_lib_reduce_mw(ctx.handle, _dev_ptr(x), W, rows, cols, x.stride(0) // W, prime_begin, L,
                          _dev_ptr(out), out.stride(1), out.stride(0), _stream(stream)), "rns_reduce_mw")
    return out


@dataclass
class GemmProblem:
    """C[j] = A[j] @ B[j] mod p_{prime_begin+j} (or, with subtract,
    C[j] = C[j] - A[j] @ B[j] mod p); A [L, m, k], B [L, k, n], C [L, m, n],
    int32 device tensors with unit column stride."""
    A: object
    B: object
    C: object
    prime_begin: int = 0
    subtract: bool = False

    def desc(self) -> RnsGemmDesc:
        L, m, k = self.A.shape
        L2, k2, n = self.B.shape
        assert L == L2 and k == k2 and tuple(self.C.shape) == (L, m, n)
        for t in (self.A, self.B, self.C):
            assert t.stride(2) == 1
        d = RnsGemmDesc()
        d.m, d.n, d.k = m, n, k
        d.A, d.lda, d.a_plane_stride = _dev_ptr(self.A), self.A.stride(1), self.A.stride(0)
        d.B, d.ldb, d.b_plane_stride = _dev_ptr(self.B), self.B.stride(1), self.B.stride(0)
        d.C, d.ldc, d.c_plane_stride = _dev_ptr(self.C), self.C.stride(1), self.C.stride(0)
        d.prime_begin, d.L = self.prime_begin, L
        d.flags = 1 if self.subtract else 0
        return d


def _descs(problems: Sequence[GemmProblem]):
    arr = (RnsGemmDesc * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = p.desc()
    return arr


def modmatmul_batched(ctx: Context, problems: Sequence[GemmProblem], path="auto", stream=None):
    path = _PATHS[path] if isinstance(path, str) else int(path)
    arr = _descs(problems)
    _check(_lib_modmatmul(ctx.handle, arr, len(problems), path, _stream(stream)), "modmatmul_batched")


def modmatmul_batched_noalloc(ctx: Context, problems: Sequence[GemmProblem], path="auto", stream=None):
    """modmatmul_batched with its scratch in the library's fixed per-device
    array (no device allocation); RnsError(ESCRATCH) when it does not fit."""
    path = _PATHS[path] if isinstance(path, str) else int(path)
    arr = _descs(problems)
    _check(_lib_modmatmul_noalloc(ctx.handle, arr, len(problems), path, _stream(stream)),
           "modmatmul_batched_noalloc")


def noalloc_scratch_bytes() -> int:
    out = ctypes.c_size_t()
    _check(_lib_noalloc_bytes(ctypes.byref(out)), "rns_noalloc_scratch_bytes")
    return out.value


def workspace_bytes(ctx: Context, problems: Sequence[GemmProblem], path="auto") -> int:
    path = _PATHS[path] if isinstance(path, str) else int(path)
    arr = _descs(problems)
    out = ctypes.c_size_t()
    _check(_lib_workspace_bytes(ctx.handle, arr, len(problems), path, ctypes.byref(out)),
           "rns_workspace_bytes")
    return out.value


def _path(path):
    return _PATHS[path] if isinstance(path, str) else int(path)


def _info(fn, h) -> dict:
    info = RnsPlanInfo()
    _check(fn(h, ctypes.byref(info)), "plan info")
    return {"path": {1: "fp64", 2: "int8"}.get(info.path, info.path), "variant": info.variant,
            "tiles": info.tiles, "workspace_bytes": info.workspace_bytes, "residue_ops": info.residue_ops}


class GemmPlan:
    """rns_gemm_plan: modmatmul_batched set up once; execute() only launches
    kernels and may be captured into a HIP graph.  Keeps the tensors alive."""

    def __init__(self, ctx: Context, problems: Sequence[GemmProblem], path="auto"):
        self.ctx = ctx
        self._keep = list(problems)
        arr = _descs(problems)
        h = _P()
        _check(_lib_gplan_create(ctx.handle, arr, len(problems), _path(path), ctypes.byref(h)),
               "rns_gemm_plan_create")
        self.handle = h

    def execute(self, stream=None):
        _check(_lib_gplan_execute(self.handle, _stream(stream)), "rns_gemm_plan_execute")

    def info(self) -> dict:
        return _info(_lib_gplan_info, self.handle)

    def set_variant(self, v: int):
        _check(_lib_gplan_set_variant(self.handle, v), "rns_gemm_plan_set_variant")

    def autotune(self, stream=None) -> int:
        v = _I32()
        _check(_lib_gplan_autotune(self.handle, _stream(stream), ctypes.byref(v)), "rns_gemm_plan_autotune")
        return v.value

    def close(self):
        if self.handle:
            _lib_gplan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ctx: Context, problems: Sequence[GemmProblem], path="auto", stream=None) -> int:
    arr = _descs(problems)
    v = _I32()
    _check(_lib_autotune(ctx.handle, arr, len(problems), _path(path), _stream(stream), ctypes.byref(v)),
           "rns_autotune")
    return v.value


@dataclass
class MatmulProblem:
    """C = A @ B over the integers: A (m, k), B (k, n) int64 device tensors;
    C int64 (m, n) for W == 1 or (m, n, W) words."""
    A: object
    B: object
    C: object
    prime_begin: int = 0
    L: int = 24
    bound: int = 0


class MatmulPlan:
    """rns_matmul_plan: reduce -> products -> CRT for a batch, with resident
    tiled operands and C residue planes; execute() is three kernel launches
    (conversion of the int64 operands, GEMM, CRT)."""

    def __init__(self, ctx: Context, problems: Sequence[MatmulProblem], path="auto", W: int = 1):
        self.ctx = ctx
        self._keep = list(problems)
        arr = (RnsMatmulDesc * max(1, len(problems)))()
        for i, p in enumerate(problems):
            m, k = p.A.shape
            k2, n = p.B.shape
            assert k == k2 and p.A.stride(1) == 1 and p.B.stride(1) == 1 and p.C.is_contiguous()
            d = arr[i]
            d.m, d.n, d.k = m, n, k
            d.A, d.lda = _dev_ptr(p.A), p.A.stride(0)
            d.B, d.ldb = _dev_ptr(p.B), p.B.stride(0)
            d.C, d.ldc = _dev_ptr(p.C), n
            d.prime_begin, d.L, d.bound = p.prime_begin, p.L, int(p.bound)
        h = _P()
        _check(_lib_mplan_create(ctx.handle, arr, len(problems), _path(path), W, ctypes.byref(h)),
               "rns_matmul_plan_create")
        self.handle = h

    def execute(self, stream=None):
        _check(_lib_mplan_execute(self.handle, _stream(stream)), "rns_matmul_plan_execute")

    def info(self) -> dict:
        return _info(_lib_mplan_info, self.handle)

    def set_variant(self, v: int):
        _check(_lib_gplan_set_variant(_lib_mplan_gemm(self.handle), v), "rns_gemm_plan_set_variant")

    def autotune(self, stream=None) -> int:
        """Time the INT8 GEMM variants on this plan's products and keep the fastest."""
        v = _I32()
        _check(_lib_gplan_autotune(_lib_mplan_gemm(self.handle), _stream(stream), ctypes.byref(v)),
               "rns_gemm_plan_autotune")
        return v.value

    def close(self):
        if self.handle:
            _lib_mplan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def crt_reconstruct(ctx: Context, res, prime_begin: int = 0, L: Optional[int] = None,
                    bound: Optional[int] = None, W: int = 1, out=None, status=None, stream=None):
    """res: int32 planes [L, rows, cols].  Returns int64 [rows, cols, W] words
    (two's complement, little-endian); for W == 1 a [rows, cols] tensor."""
    import torch
    L = res.shape[0] if L is None else L
    _, rows, cols = res.shape
    assert res.dtype == torch.int32 and res.stride(2) == 1
    if out is None:
        out = torch.empty((rows, cols, W), dtype=torch.int64, device=res.device)
    assert out.dtype == torch.int64 and out.is_contiguous()
    if bound is not None:
        w = _words(bound)
        barr = (ctypes.c_uint64 * len(w))(*w)
        bptr, bw = ctypes.cast(barr, _P), len(w)
    else:
        bptr, bw = None, 0
    sptr = _dev_ptr(status) if status is not None else None
    _check(_lib_crt(ctx.handle, _dev_ptr(res), rows, cols, res.stride(1), res.stride(0),
                    prime_begin, L, bptr, bw, _dev_ptr(out), W, cols, sptr, _stream(stream)),
           "crt_reconstruct")
    return out[:, :, 0] if W == 1 else out


def base_convert(ctx: Context, res, prime_begin: int, prime_begin_out: int, L_out: int,
                 L: Optional[int] = None, bound: Optional[int] = None, out=None, status=None, stream=None):
    """Residues [L, rows, cols] in the primes range (prime_begin, L) ->
    residues [L_out, rows, cols] of the same symmetric integer in the range
    (prime_begin_out, L_out) (rns_base_convert); int32 device tensors."""
    import torch
    L = res.shape[0] if L is None else L
    _, rows, cols = res.shape
    assert res.dtype == torch.int32 and res.stride(2) == 1
    if out is None:
        out = torch.empty((L_out, rows, cols), dtype=torch.int32, device=res.device)
    assert out.dtype == torch.int32 and out.stride(2) == 1
    if bound is not None:
        w = _words(bound)
        barr = (ctypes.c_uint64 * len(w))(*w)
        bptr, bw = ctypes.cast(barr, _P), len(w)
    else:
        bptr, bw = None, 0
    sptr = _dev_ptr(status) if status is not None else None
    _check(_lib_convert(ctx.handle, _dev_ptr(res), rows, cols, res.stride(1), res.stride(0), prime_begin, L,
                        bptr, bw, _dev_ptr(out), out.stride(1), out.stride(0), prime_begin_out, L_out, sptr,
                        _stream(stream)), "rns_base_convert")
    return out


def words_to_ints(words: np.ndarray) -> np.ndarray:
    """int64 [..., W] two's-complement words -> object array of Python ints."""
    w = np.ascontiguousarray(np.asarray(words).astype("<u8"))
    W = w.shape[-1]
    flat = w.reshape(-1, W)
    out = np.empty(flat.shape[0], dtype=object)
    for e in range(flat.shape[0]):
        out[e] = int.from_bytes(flat[e].tobytes(), "little", signed=True)
    return out.reshape(w.shape[:-1])


@dataclass
class SmithResult:
    s: List[int]
    stats: dict


def _smith_result(h) -> SmithResult:
    try:
        return _smith_result_keep(h)
    finally:
        _lib_smith_free(h)


def smith_form(ctx: Context, a: np.ndarray, seed: int = 0) -> SmithResult:
    a = np.ascontiguousarray(a, dtype=np.int64)
    n = a.shape[0]
    assert a.shape == (n, n)
    h = _P()
    _check(_lib_smith(ctx.handle, a.ctypes.data, n, seed, ctypes.byref(h)), "smith_form")
    return _smith_result(h)


MASSAGER_U, MASSAGER_M, MASSAGER_T = 0, 1, 2


@dataclass
class MassagerResult:
    """S (list of ints) and the Smith massager U (rows), M and T (columns) as
    n x n object arrays of Python ints (rns_smith_massager); a matrix not
    asked for is None, and m_columns holds the columns of M asked for alone."""
    s: List[int]
    U: Optional[np.ndarray]
    M: Optional[np.ndarray]
    T: Optional[np.ndarray]
    stats: dict
    m_columns: Optional[dict] = None


def _massager_vector(h, which, idx, n):
    w = _lib_massager_width(h, which, idx)
    if w < 1:
        raise RnsError(-w, "rns_smith_massager_width")
    buf = np.zeros(n * w, dtype=np.uint64)
    _check(_lib_massager_vector(h, which, idx, buf.ctypes.data, w), "rns_smith_massager_vector")
    return words_to_uints(buf.reshape(n, w))


def smith_massager(ctx: Context, a: np.ndarray, seed: int = 0, fetch=("U", "M", "T"),
                   m_columns=None) -> MassagerResult:
    a = np.ascontiguousarray(a, dtype=np.int64)
    n = a.shape[0]
    assert a.shape == (n, n)
    h = _P()
    _check(_lib_massager(ctx.handle, a.ctypes.data, n, seed, ctypes.byref(h)), "rns_smith_massager")
    try:
        mats = {}
        for name, which in (("U", MASSAGER_U), ("M", MASSAGER_M), ("T", MASSAGER_T)):
            if name not in fetch:
                mats[name] = None
                continue
            out = np.empty((n, n), dtype=object)
            for idx in range(n):
                vals = _massager_vector(h, which, idx, n)
                if which == MASSAGER_U:
                    out[idx, :] = vals
                else:
                    out[:, idx] = vals
            mats[name] = out
        cols = {j: _massager_vector(h, MASSAGER_M, j, n) for j in (m_columns or [])}
        res = _smith_result_keep(h)
    finally:
        _lib_smith_free(h)
    return MassagerResult(res.s, mats["U"], mats["M"], mats["T"], res.stats, cols)


@dataclass
class UnimodularResult:
    """rns_unimodular_certify: verdict (True, False, or None when the steps
    ran out before the bound's precision), the last residue Z (int64 array,
    if asked for) and the call's info fields (x_prime / q_prime as lists)."""
    verdict: Optional[bool]
    Z: Optional[np.ndarray]
    info: dict


def unimodular_certify(ctx: Context, d: np.ndarray, max_steps: int = -1, want_z: bool = False) -> UnimodularResult:
    d = np.ascontiguousarray(d, dtype=np.int64)
    n = d.shape[0]
    assert d.shape == (n, n)
    z = np.zeros((n, n), dtype=np.int64) if want_z else None
    info = RnsUnimodInfo()
    _check(_lib_unimodular(ctx.handle, d.ctypes.data if n else None, n, max_steps,
                           z.ctypes.data if want_z and n else None, ctypes.byref(info)),
           "rns_unimodular_certify")
    out = {f: getattr(info, f) for f, _ in RnsUnimodInfo._fields_}
    out["x_prime"] = list(info.x_prime)[:info.x_primes]
    out["q_prime"] = list(info.q_prime)[:info.q_primes]
    verdict = {1: True, 0: False}.get(info.verdict)
    return UnimodularResult(verdict, z, out)


def words_to_uints(w: np.ndarray) -> np.ndarray:
    """Rows of little-endian 64-bit words as non-negative Python ints (an
    object array)."""
    w = np.ascontiguousarray(w, dtype="<u8")
    out = np.empty(w.shape[0], dtype=object)
    for i in range(w.shape[0]):            # linear in the words, unlike shifts
        out[i] = int.from_bytes(w[i].tobytes(), "little")
    return out


def _smith_result_keep(h) -> SmithResult:
    s = []
    words = ctypes.POINTER(ctypes.c_uint64)()
    nw = _I32()
    for i in range(_lib_smith_size(h)):
        _check(_lib_smith_get(h, i, ctypes.byref(words), ctypes.byref(nw)), "rns_smith_get")
        s.append(int.from_bytes(ctypes.string_at(words, 8 * nw.value), "little") if nw.value else 0)
    st = RnsSmithStats()
    _check(_lib_smith_stats(h, ctypes.byref(st)), "rns_smith_stats_get")
    return SmithResult(s, {f: getattr(st, f) for f, _ in RnsSmithStats._fields_})


def largest_invariant(ctx: Context, a: np.ndarray, seed: int = 0) -> SmithResult:
    """Phase 1 alone: s_n by p-adic lifting (Monte Carlo); result.s == [s_n]."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    n = a.shape[0]
    assert a.shape == (n, n)
    h = _P()
    _check(_lib_lif(ctx.handle, a.ctypes.data, n, seed, ctypes.byref(h)), "rns_largest_invariant")
    return _smith_result(h)


LIFT_C_MFMA, LIFT_AX_MFMA, LIFT_PACKED, LIFT_A_INT16 = 1, 2, 4, 8


def lift_step(C, A, R, p: int, form: str = "mfma", device: int = 0, stream=None):
    """One Dixon lifting step on the GPU (rns_lift_step).  C: uint32 residues
    as int32 (n, n); A: int64 (n, n); R: int64 (t, n) -- device tensors.
    Returns (X int32 (t, n), R_next int64 (t, n), Rm_next int32 (t, n),
    inexact: bool, kernels: LIFT_* bits)."""
    import torch
    n = A.shape[0]
    t = R.shape[0]
    assert C.shape == (n, n) and A.shape == (n, n) and R.shape == (t, n)
    assert C.dtype == torch.int32 and A.dtype == torch.int64 and R.dtype == torch.int64
    assert C.is_contiguous() and A.is_contiguous() and R.is_contiguous()
    X = torch.empty((t, n), dtype=torch.int32, device=A.device)
    Rn = torch.empty((t, n), dtype=torch.int64, device=A.device)
    Rnm = torch.empty((t, n), dtype=torch.int32, device=A.device)
    bad = ctypes.c_int32()
    used = _I32()
    _check(_lib_lift_step(device, _dev_ptr(C), _dev_ptr(A), _dev_ptr(R), n, t, p,
                          {"vector": 0, "mfma": 1}[form], _dev_ptr(X), _dev_ptr(Rn), _dev_ptr(Rnm),
                          ctypes.byref(bad), ctypes.byref(used), _stream(stream)), "rns_lift_step")
    return X, Rn, Rnm, bool(bad.value), used.value


def server_footprint(n: int) -> int:
    out = ctypes.c_size_t()
    _check(_lib_srv_footprint(n, ctypes.byref(out)), "rns_server_footprint")
    return out.value


class Server:
    """rns_server: Smith-form requests served concurrently on one GPU."""

    def __init__(self, device: int = 0, workers: int = 4, hbm_budget: int = 0, aging: float = 2.0):
        h = _P()
        _check(_lib_srv_create(device, workers, hbm_budget, ctypes.byref(h)), "rns_server_create")
        self.handle = h
        _check(_lib_srv_aging(h, aging), "rns_server_set_aging")

    def submit(self, a: np.ndarray, seed: int = 0) -> int:
        a = np.ascontiguousarray(a, dtype=np.int64)
        t = ctypes.c_uint64()
        _check(_lib_srv_submit(self.handle, a.ctypes.data, a.shape[0], seed, ctypes.byref(t)),
               "rns_server_submit")
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """-> (status, SmithResult or None, info dict)."""
        h = _P()
        info = RnsRequestInfo()
        st = _lib_srv_wait(self.handle, ticket, timeout, ctypes.byref(h), ctypes.byref(info))
        d = {f: getattr(info, f) for f, _ in RnsRequestInfo._fields_}
        if st == OK:
            return st, _smith_result(h), d
        if h:
            _lib_smith_free(h)
        return st, None, d

    def stats(self) -> dict:
        s = RnsServerStats()
        _check(_lib_srv_stats(self.handle, ctypes.byref(s)), "rns_server_stats")
        return {f: getattr(s, f) for f, _ in RnsServerStats._fields_}

    def close(self):
        if self.handle:
            _lib_srv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
