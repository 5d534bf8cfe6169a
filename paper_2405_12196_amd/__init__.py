"""Python binding of the MI355X block-sparse tensordot library (libyastn.so).

Argument marshalling only: every step of the contraction (matching, fusing,
sector GEMMs, output scatter, norms) runs in the library's HIP kernels.
PyTorch supplies device memory and streams.  If the compiled library is
missing this package raises on first use; there is no fallback path.

Names follow the C ABI in include/yastn.h:
    plan(problems, ...)        -> Plan            (yastn_plan)
    Plan.output(p)             -> structure of C  (yastn_plan_output)
    Plan.contract(a, b, c, ws) -> None, async     (yastn_contract)
    Plan.contract_noalloc(a, b, c) -> None, async (yastn_contract_noalloc)
    contract_jobs(jobs)        -> None, async     (yastn_contract_jobs)
    norm(x, out, ws)           -> None, async     (yastn_norm)
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libyastn.so")

F64, F32, BF16X3, BF16X6 = 0, 1, 2, 3
FLAG_MFMA, FLAG_ROWS, FLAG_NOCACHE = 1, 2, 4
DTYPE_F64, DTYPE_F32, DTYPE_C128 = 0, 1, 2
CONJ_A, CONJ_B = 1, 2
SVD_RECOVER_V = 1
PRECISIONS = {"f64": F64, "f32": F32, "bf16x3": BF16X3, "bf16x6": BF16X6}
STATUS = ["OK", "ERR_ARG", "ERR_SYM", "ERR_CHARGE", "ERR_SIGNATURE", "ERR_SHAPE",
          "ERR_DUPLICATE", "ERR_NOMEM", "ERR_HIP", "ERR_STATE"]

EXPORTS = ["yastn_plan", "yastn_plan_profile", "yastn_plan_cache_clear", "yastn_tune_save", "yastn_tune_load",
           "yastn_tune_clear", "yastn_plan_output", "yastn_plan_workspace", "yastn_plan_stats", "yastn_plan_info",
           "yastn_contract", "yastn_contract_noalloc", "yastn_contract_norm", "yastn_contract_timed",
           "yastn_contract_jobs", "yastn_norm_workspace", "yastn_norm",
           "yastn_free", "yastn_last_error", "yastn_status_string", "yastn_abi_version",
           "yastn_plan_autotune", "yastn_plan_set_variant",
           "yastn_server_create", "yastn_server_submit", "yastn_server_step", "yastn_server_query",
           "yastn_server_forget", "yastn_server_drain", "yastn_server_get_stats", "yastn_server_destroy",
           "yastn_perm_plan", "yastn_perm_output", "yastn_permute", "yastn_perm_free",
           "yastn_grad_plan", "yastn_grad_output", "yastn_grad_workspace", "yastn_grad", "yastn_grad_free",
           "yastn_svd_plan", "yastn_svd_info", "yastn_svd_set_flags", "yastn_svd_sector", "yastn_svd",
           "yastn_svd_output", "yastn_svd_factors", "yastn_svd_factors_scaled", "yastn_svd_free",
           "yastn_ctm_plan", "yastn_ctm_move", "yastn_ctm_tensor", "yastn_ctm_copy", "yastn_ctm_info",
           "yastn_ctm_free", "yastn_zplan", "yastn_zplan_output", "yastn_zplan_workspace", "yastn_zplan_real",
           "yastn_zcontract", "yastn_zplan_autotune", "yastn_zplan_free", "yastn_swap_plan", "yastn_swap_info",
           "yastn_swap_gate", "yastn_swap_free"]
CTM_NAMES = ("Q1", "Q2", "Q3", "Q4", "Rup", "Rdn", "M", "Us", "Vts", "Pup", "Pdn", "C1T1", "C4T3", "Z1", "Z2",
             "Z3", "C1n", "T4n", "C4n", "C1", "T4", "C4")
CTM_INPUTS = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4", "A")
CTM_AUTOTUNE = 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE = 0, 1, 2
MAX_CHAIN = 8
NUM_VARIANTS = 25
SCRATCH_BYTES = 64 << 20


class YastnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = name


class TensorDesc(C.Structure):
    _fields_ = [("rank", C.c_int32), ("nsym", C.c_int32), ("sym_mod", C.POINTER(C.c_int32)),
                ("sig", C.POINTER(C.c_int8)), ("n", C.POINTER(C.c_int32)), ("nblocks", C.c_int64),
                ("charges", C.POINTER(C.c_int32)), ("shapes", C.POINTER(C.c_int64)),
                ("offsets", C.POINTER(C.c_int64))]


class Problem(C.Structure):
    _fields_ = [("a", TensorDesc), ("b", TensorDesc), ("ncontract", C.c_int32),
                ("axes_a", C.POINTER(C.c_int32)), ("axes_b", C.POINTER(C.c_int32))]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("in_dtype", C.c_int32), ("out_dtype", C.c_int32),
                ("tile_rows", C.c_int32), ("flags", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("blocks_a", "blocks_b", "pairs", "sectors", "c_blocks",
                                         "c_numel", "numel_a", "numel_b", "max_m", "max_k", "max_n",
                                         "tiles")] + \
               [("useful_flops", C.c_double), ("mfma_flops", C.c_double), ("alg_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("nsteps", C.c_int32), ("plans", C.POINTER(C.c_void_p)), ("a0", C.c_void_p),
                ("b", C.POINTER(C.c_void_p)), ("out", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "admitted", "completed", "ticks", "launched_steps",
                                         "max_batch", "queued", "running")] + \
               [(n, C.c_size_t) for n in ("pool_bytes", "pool_used", "pool_peak")] + \
               [(n, C.c_int64) for n in ("bypasses", "queued_peak")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Job(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("a", C.POINTER(C.c_void_p)), ("b", C.POINTER(C.c_void_p)),
                ("c", C.POINTER(C.c_void_p)), ("workspace", C.c_void_p)]


_LIB = None


def lib():
    """Load libyastn.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with paper_2405_12196_amd/build.py "
                              "(no fallback path exists)")
        L = C.CDLL(LIB_PATH)
        L.yastn_plan.argtypes = [C.POINTER(Problem), C.c_int32, C.POINTER(Options), C.c_void_p,
                                 C.POINTER(C.c_void_p)]
        L.yastn_plan_profile.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.yastn_plan_profile.restype = C.c_int32
        L.yastn_plan_cache_clear.argtypes = []
        L.yastn_plan_cache_clear.restype = None
        L.yastn_tune_save.argtypes = [C.c_char_p]
        L.yastn_tune_save.restype = C.c_int32
        L.yastn_tune_load.argtypes = [C.c_char_p, C.POINTER(C.c_int32)]
        L.yastn_tune_load.restype = C.c_int32
        L.yastn_tune_clear.argtypes = []
        L.yastn_tune_clear.restype = None
        L.yastn_plan_output.argtypes = [C.c_void_p, C.c_int32, C.POINTER(TensorDesc), C.POINTER(C.c_int64)]
        L.yastn_plan_workspace.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.yastn_plan_stats.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Stats)]
        L.yastn_contract.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]
        L.yastn_contract_noalloc.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                             C.POINTER(C.c_void_p), C.c_void_p]
        L.yastn_contract_norm.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_void_p]
        L.yastn_contract_timed.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
        L.yastn_contract_jobs.argtypes = [C.POINTER(Job), C.c_int32, C.c_void_p]
        L.yastn_plan_autotune.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_int32,
                                          C.POINTER(C.c_int32), C.POINTER(C.c_float)]
        L.yastn_plan_set_variant.argtypes = [C.c_void_p, C.c_int32]
        L.yastn_plan_info.argtypes = [C.c_void_p, C.POINTER(Options), C.POINTER(C.c_int32)]
        L.yastn_server_create.argtypes = [C.c_size_t, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
        L.yastn_server_submit.argtypes = [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_int64)]
        L.yastn_server_step.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.yastn_server_query.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.yastn_server_forget.argtypes = [C.c_void_p, C.c_int64]
        L.yastn_server_drain.argtypes = [C.c_void_p]
        L.yastn_server_get_stats.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
        L.yastn_server_destroy.argtypes = [C.c_void_p]
        L.yastn_server_destroy.restype = None
        L.yastn_norm_workspace.restype = C.c_size_t
        L.yastn_norm.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.yastn_free.argtypes = [C.c_void_p]
        L.yastn_free.restype = None
        L.yastn_last_error.restype = C.c_char_p
        L.yastn_status_string.restype = C.c_char_p
        L.yastn_status_string.argtypes = [C.c_int32]
        L.yastn_perm_plan.argtypes = [C.POINTER(TensorDesc), C.POINTER(C.c_int32), C.c_void_p, C.POINTER(C.c_void_p)]
        L.yastn_perm_output.argtypes = [C.c_void_p, C.POINTER(TensorDesc), C.POINTER(C.c_int64)]
        L.yastn_permute.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.yastn_perm_free.argtypes = [C.c_void_p]
        L.yastn_perm_free.restype = None
        L.yastn_grad_plan.argtypes = [C.POINTER(Problem), C.c_int32, C.POINTER(Options), C.c_void_p,
                                      C.POINTER(C.c_void_p)]
        L.yastn_grad_output.argtypes = [C.c_void_p, C.POINTER(TensorDesc), C.POINTER(C.c_int64)]
        L.yastn_grad_workspace.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.yastn_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.yastn_grad_free.argtypes = [C.c_void_p]
        L.yastn_grad_free.restype = None
        L.yastn_svd_plan.argtypes = [C.POINTER(TensorDesc), C.c_int32, C.POINTER(C.c_int32), C.c_void_p,
                                     C.POINTER(C.c_void_p)]
        L.yastn_svd_info.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
        L.yastn_svd_set_flags.argtypes = [C.c_void_p, C.c_int32]
        L.yastn_svd_sector.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.yastn_svd.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_void_p,
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p, C.c_void_p]
        L.yastn_svd_output.argtypes = [C.c_void_p, C.POINTER(TensorDesc), C.POINTER(C.c_int64),
                                       C.POINTER(TensorDesc), C.POINTER(C.c_int64)]
        L.yastn_svd_factors.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.yastn_svd_factors_scaled.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                               C.c_void_p, C.c_void_p]
        L.yastn_svd_free.argtypes = [C.c_void_p]
        L.yastn_svd_free.restype = None
        L.yastn_ctm_plan.argtypes = [C.POINTER(TensorDesc), C.c_void_p, C.POINTER(C.c_void_p)]
        L.yastn_ctm_move.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.c_int32, C.c_double, C.c_double,
                                     C.c_int32, C.c_void_p]
        L.yastn_ctm_tensor.argtypes = [C.c_void_p, C.c_int32, C.POINTER(TensorDesc), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_void_p)]
        L.yastn_ctm_copy.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.yastn_ctm_info.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.yastn_ctm_free.argtypes = [C.c_void_p]
        L.yastn_ctm_free.restype = None
        L.yastn_zplan.argtypes = [C.POINTER(Problem), C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
        L.yastn_zplan_output.argtypes = [C.c_void_p, C.c_int32, C.POINTER(TensorDesc), C.POINTER(C.c_int64)]
        L.yastn_zplan_workspace.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.yastn_zplan_real.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        L.yastn_zcontract.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]
        L.yastn_zplan_autotune.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_int32,
                                           C.POINTER(C.c_int32), C.POINTER(C.c_float)]
        L.yastn_zplan_free.argtypes = [C.c_void_p]
        L.yastn_zplan_free.restype = None
        L.yastn_swap_plan.argtypes = [C.POINTER(TensorDesc), C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_void_p)]
        L.yastn_swap_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.yastn_swap_gate.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.yastn_swap_free.argtypes = [C.c_void_p]
        L.yastn_swap_free.restype = None
        for f in ("yastn_perm_plan", "yastn_perm_output", "yastn_permute", "yastn_grad_plan", "yastn_grad_output",
                  "yastn_grad_workspace", "yastn_grad", "yastn_svd_plan", "yastn_svd_info", "yastn_svd_set_flags",
                  "yastn_svd_sector",
                  "yastn_svd", "yastn_svd_output", "yastn_svd_factors", "yastn_svd_factors_scaled",
                  "yastn_ctm_plan", "yastn_ctm_move", "yastn_ctm_tensor", "yastn_ctm_copy", "yastn_ctm_info",
                  "yastn_zplan", "yastn_zplan_output", "yastn_zplan_workspace", "yastn_zplan_real", "yastn_zcontract",
                  "yastn_zplan_autotune", "yastn_swap_plan", "yastn_swap_info", "yastn_swap_gate"):
            getattr(L, f).restype = C.c_int32
        for f in ("yastn_plan", "yastn_plan_output", "yastn_plan_workspace", "yastn_plan_stats",
                  "yastn_contract", "yastn_contract_noalloc", "yastn_contract_norm", "yastn_contract_timed",
                  "yastn_contract_jobs", "yastn_norm",
                  "yastn_plan_autotune", "yastn_plan_set_variant", "yastn_plan_info", "yastn_server_create",
                  "yastn_server_submit", "yastn_server_step", "yastn_server_query", "yastn_server_forget",
                  "yastn_server_drain", "yastn_server_get_stats"):
            getattr(L, f).restype = C.c_int32
        _LIB = L
    return _LIB


def _check(status: int):
    if status != 0:
        raise YastnError(status, lib().yastn_last_error().decode())


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x), dtype=dtype)


class _Keep:
    """Holds numpy arrays alive while a descriptor points at them."""

    def __init__(self):
        self.items = []

    def ptr(self, arr, ctype):
        self.items.append(arr)
        return arr.ctypes.data_as(C.POINTER(ctype))


def _desc(t, keep: _Keep) -> TensorDesc:
    """Descriptor of anything with sym_mod, sig, n, charges, shapes, offsets."""
    charges = _arr(t.charges, np.int32)
    shapes = _arr(t.shapes, np.int64)
    offsets = _arr(t.offsets, np.int64)
    sig = _arr(t.sig, np.int8)
    sym = _arr(t.sym_mod, np.int32)
    n = _arr(t.n, np.int32)
    d = TensorDesc()
    d.rank = int(sig.shape[0])
    d.nsym = int(sym.shape[0])
    d.sym_mod = keep.ptr(sym, C.c_int32)
    d.sig = keep.ptr(sig, C.c_int8)
    d.n = keep.ptr(n, C.c_int32)
    d.nblocks = int(offsets.shape[0])
    d.charges = keep.ptr(charges, C.c_int32)
    d.shapes = keep.ptr(shapes, C.c_int64)
    d.offsets = keep.ptr(offsets, C.c_int64)
    return d


@dataclass
class Structure:
    """Block structure of a tensor (no data): what yastn_plan_output returns."""

    sym_mod: tuple
    sig: np.ndarray
    n: np.ndarray
    charges: np.ndarray
    shapes: np.ndarray
    offsets: np.ndarray
    numel: int

    @property
    def nblocks(self):
        return int(self.offsets.shape[0])


def _ptr(x) -> int:
    """Device address of a torch tensor or an int."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return 0
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _structure(d, n) -> Structure:
    """Copy a descriptor the library owns into a Structure."""
    nb, r, s = d.nblocks, d.rank, d.nsym

    def cp(ptr, count, dtype):
        if count == 0:
            return np.zeros(0, dtype=dtype)
        return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)
    return Structure(tuple(int(v) for v in cp(d.sym_mod, s, np.int32)),
                     cp(d.sig, r, np.int8) if r else np.zeros(0, np.int8),
                     cp(d.n, s, np.int32),
                     cp(d.charges, nb * r * s, np.int32).reshape(nb, r, s),
                     cp(d.shapes, nb * r, np.int64).reshape(nb, r),
                     cp(d.offsets, nb, np.int64), int(n.value))


class Plan:
    """A validated, matched and tiled set of tensordot problems (yastn_plan)."""

    def __init__(self, problems, precision="f64", in_dtype=None, out_dtype=None, tile_rows=0, stream=None,
                 flags=0):
        L = lib()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if in_dtype is None:
            in_dtype = DTYPE_F64 if prec == F64 else DTYPE_F32
        if out_dtype is None:
            out_dtype = DTYPE_F64 if prec == F64 else DTYPE_F32
        self.precision, self.in_dtype, self.out_dtype = prec, in_dtype, out_dtype
        keep = _Keep()
        arr = (Problem * max(1, len(problems)))()
        for i, (a, b, axes_a, axes_b) in enumerate(problems):
            arr[i].a = _desc(a, keep)
            arr[i].b = _desc(b, keep)
            xa, xb = _arr(list(axes_a), np.int32), _arr(list(axes_b), np.int32)
            arr[i].ncontract = int(len(axes_a)) if len(axes_a) == len(axes_b) else -1
            arr[i].axes_a = keep.ptr(xa, C.c_int32)
            arr[i].axes_b = keep.ptr(xb, C.c_int32)
        opts = Options(prec, in_dtype, out_dtype, tile_rows, flags)
        h = C.c_void_p()
        _check(L.yastn_plan(arr, len(problems), C.byref(opts), C.c_void_p(_stream(stream)),
                            C.byref(h)))
        self._h = h
        self.nprob = len(problems)
        self.variant_id = 0
        ws = C.c_size_t()
        _check(L.yastn_plan_workspace(h, C.byref(ws)))
        self.workspace_bytes = int(ws.value)

    @property
    def handle(self):
        return self._h

    def output(self, p: int = 0) -> Structure:
        d = TensorDesc()
        n = C.c_int64()
        _check(lib().yastn_plan_output(self._h, p, C.byref(d), C.byref(n)))
        return _structure(d, n)

    def profile(self):
        """(ms of validation, join, host tables, upload; from the cache?)."""
        ms = (C.c_double * 4)()
        cached = C.c_int32()
        _check(lib().yastn_plan_profile(self._h, ms, C.byref(cached)))
        return [float(v) for v in ms], bool(cached.value)

    def stats(self, p: int = 0) -> dict:
        st = Stats()
        _check(lib().yastn_plan_stats(self._h, p, C.byref(st)))
        return st.as_dict()

    def contract(self, a, b, c, workspace=None, stream=None):
        """a, b, c: sequences (one per problem) of device buffers (torch tensors
        or addresses).  Asynchronous on ``stream`` (torch's current by default)."""
        n = self.nprob
        pa = (C.c_void_p * max(1, n))(*[_ptr(x) for x in a])
        pb = (C.c_void_p * max(1, n))(*[_ptr(x) for x in b])
        pc = (C.c_void_p * max(1, n))(*[_ptr(x) for x in c])
        _check(lib().yastn_contract(self._h, pa, pb, pc, C.c_void_p(_ptr(workspace)),
                                    C.c_void_p(_stream(stream))))

    def contract_noalloc(self, a, b, c, stream=None):
        """As contract(), with the library's fixed per-GPU scratch as the
        workspace (yastn_contract_noalloc: no device allocation; calls that
        may overlap on one GPU race on the scratch)."""
        n = self.nprob
        pa = (C.c_void_p * max(1, n))(*[_ptr(x) for x in a])
        pb = (C.c_void_p * max(1, n))(*[_ptr(x) for x in b])
        pc = (C.c_void_p * max(1, n))(*[_ptr(x) for x in c])
        _check(lib().yastn_contract_noalloc(self._h, pa, pb, pc, C.c_void_p(_stream(stream))))

    def contract_norm(self, a, b, c, workspace, norm_out, stream=None):
        """As contract() for a single-problem plan; also writes norm_out[0] =
        ||C||_F and norm_out[1] = max |C| (FP64, on the device)."""
        pa = (C.c_void_p * 1)(_ptr(a[0]))
        pb = (C.c_void_p * 1)(_ptr(b[0]))
        pc = (C.c_void_p * 1)(_ptr(c[0]))
        _check(lib().yastn_contract_norm(self._h, pa, pb, pc, C.c_void_p(_ptr(workspace)),
                                         C.c_void_p(_ptr(norm_out)), C.c_void_p(_stream(stream))))

    def contract_timed(self, a, b, c, workspace, events, stream=None):
        """As contract(); records ``events`` (3 raw hipEvent_t handles or None)
        before the pack kernel, between pack and GEMM, and after the GEMM."""
        n = self.nprob
        pa = (C.c_void_p * max(1, n))(*[_ptr(x) for x in a])
        pb = (C.c_void_p * max(1, n))(*[_ptr(x) for x in b])
        pc = (C.c_void_p * max(1, n))(*[_ptr(x) for x in c])
        ev = (C.c_void_p * 3)(*[e or 0 for e in events])
        _check(lib().yastn_contract_timed(self._h, pa, pb, pc, C.c_void_p(_ptr(workspace)),
                                          C.c_void_p(_stream(stream)), ev))

    def autotune(self, a, b, c, workspace, reps=5, stream=None):
        """Time every kernel variant that fits on these buffers, keep the
        fastest; returns (variant, per-variant ms list, -1 = not applicable)."""
        n = self.nprob
        pa = (C.c_void_p * max(1, n))(*[_ptr(x) for x in a])
        pb = (C.c_void_p * max(1, n))(*[_ptr(x) for x in b])
        pc = (C.c_void_p * max(1, n))(*[_ptr(x) for x in c])
        ch = C.c_int32()
        times = (C.c_float * NUM_VARIANTS)()
        _check(lib().yastn_plan_autotune(self._h, pa, pb, pc, C.c_void_p(_ptr(workspace)),
                                         C.c_void_p(_stream(stream)), int(reps), C.byref(ch), times))
        self.variant_id = int(ch.value)
        return int(ch.value), [float(t) for t in times]

    def set_variant(self, v: int):
        _check(lib().yastn_plan_set_variant(self._h, int(v)))
        self.variant_id = int(v)

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def plan(problems, **kw) -> Plan:
    return Plan(problems, **kw)


def plan_cache_clear():
    """Drop every entry of the library's plan structure cache."""
    lib().yastn_plan_cache_clear()


class Perm:
    """Leg permutation of a block tensor (yastn_perm_plan / yastn_permute)."""

    def __init__(self, x, perm, stream=None):
        keep = _Keep()
        d = _desc(x, keep)
        pa = _arr(list(perm), np.int32)
        h = C.c_void_p()
        _check(lib().yastn_perm_plan(C.byref(d), keep.ptr(pa, C.c_int32), C.c_void_p(_stream(stream)),
                                     C.byref(h)))
        self._h = h

    def output(self) -> Structure:
        d, n = TensorDesc(), C.c_int64()
        _check(lib().yastn_perm_output(self._h, C.byref(d), C.byref(n)))
        return _structure(d, n)

    def permute(self, x, y, dtype=DTYPE_F64, stream=None):
        _check(lib().yastn_permute(self._h, int(dtype), C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)),
                                   C.c_void_p(_stream(stream))))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_perm_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Grad:
    """Gradient of C = tensordot(A, B, axes) with respect to A (wrt=0) or B
    (wrt=1), given dC (yastn_grad_plan / yastn_grad)."""

    def __init__(self, a, b, axes_a, axes_b, wrt, precision="f64", in_dtype=None, out_dtype=None, stream=None):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if in_dtype is None:
            in_dtype = DTYPE_F64 if prec == F64 else DTYPE_F32
        if out_dtype is None:
            out_dtype = DTYPE_F64 if prec == F64 else DTYPE_F32
        self.in_dtype, self.out_dtype = in_dtype, out_dtype
        keep = _Keep()
        pr = Problem()
        pr.a, pr.b = _desc(a, keep), _desc(b, keep)
        xa, xb = _arr(list(axes_a), np.int32), _arr(list(axes_b), np.int32)
        pr.ncontract = int(len(axes_a)) if len(axes_a) == len(axes_b) else -1
        pr.axes_a, pr.axes_b = keep.ptr(xa, C.c_int32), keep.ptr(xb, C.c_int32)
        opts = Options(prec, in_dtype, out_dtype, 0, 0)
        h = C.c_void_p()
        _check(lib().yastn_grad_plan(C.byref(pr), int(wrt), C.byref(opts), C.c_void_p(_stream(stream)),
                                     C.byref(h)))
        self._h = h
        ws = C.c_size_t()
        _check(lib().yastn_grad_workspace(h, C.byref(ws)))
        self.workspace_bytes = int(ws.value)

    def output(self) -> Structure:
        d, n = TensorDesc(), C.c_int64()
        _check(lib().yastn_grad_output(self._h, C.byref(d), C.byref(n)))
        return _structure(d, n)

    def run(self, dc, other, out, workspace, stream=None):
        _check(lib().yastn_grad(self._h, C.c_void_p(_ptr(dc)), C.c_void_p(_ptr(other)), C.c_void_p(_ptr(out)),
                                C.c_void_p(_ptr(workspace)), C.c_void_p(_stream(stream))))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_grad_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Svd:
    """Block-sparse truncated SVD of a block tensor (yastn_svd_*): rows = the
    legs ``row_legs`` (in that order), columns = the others; one sector per
    row-leg charge X = sum s_i rho_i.  ``sectors``: [(X, m, n, sv0)]."""

    def __init__(self, t, row_legs, stream=None):
        keep = _Keep()
        d = _desc(t, keep)
        rl = _arr(list(row_legs), np.int32)
        h = C.c_void_p()
        _check(lib().yastn_svd_plan(C.byref(d), len(rl), keep.ptr(rl, C.c_int32), C.c_void_p(_stream(stream)),
                                    C.byref(h)))
        self._h = h
        ns, nsv, ws = C.c_int32(), C.c_int64(), C.c_size_t()
        _check(lib().yastn_svd_info(h, C.byref(ns), C.byref(nsv), C.byref(ws)))
        self.nsectors, self.nsv, self.workspace_bytes = int(ns.value), int(nsv.value), int(ws.value)
        nsym = len(t.sym_mod)
        self.sectors = []
        for k in range(self.nsectors):
            q = (C.c_int32 * nsym)()
            m, n, s0 = C.c_int64(), C.c_int64(), C.c_int64()
            _check(lib().yastn_svd_sector(h, k, q, C.byref(m), C.byref(n), C.byref(s0)))
            self.sectors.append((tuple(int(v) for v in q), int(m.value), int(n.value), int(s0.value)))

    def set_flags(self, flags: int):
        """SVD_RECOVER_V: kept right vectors formed after the sweeps (0: accumulated)."""
        _check(lib().yastn_svd_set_flags(self._h, int(flags)))

    def run(self, t, sv, workspace, chi, tol=0.0, deg_tol=1e-10, stream=None):
        """Singular values into ``sv`` (device, nsv FP64), each sector's
        descending; returns (kept per sector, sweeps).  Synchronises."""
        kept = (C.c_int32 * max(1, self.nsectors))()
        sweeps = C.c_int32()
        _check(lib().yastn_svd(self._h, C.c_void_p(_ptr(t)), int(chi), float(tol), float(deg_tol),
                               C.c_void_p(_ptr(sv)), kept, C.byref(sweeps), C.c_void_p(_ptr(workspace)),
                               C.c_void_p(_stream(stream))))
        return [int(kept[k]) for k in range(self.nsectors)], int(sweeps.value)

    def output(self):
        """(U structure, V^T structure) of the last run's kept factors."""
        du, dv, nu, nv = TensorDesc(), TensorDesc(), C.c_int64(), C.c_int64()
        _check(lib().yastn_svd_output(self._h, C.byref(du), C.byref(nu), C.byref(dv), C.byref(nv)))
        return _structure(du, nu), _structure(dv, nv)

    def factors(self, u, vt, workspace, stream=None, pu=0.0, pv=0.0):
        """Kept factors into u and vt (device); U's column t times S_t^pu,
        V^T's row t times S_t^pv."""
        _check(lib().yastn_svd_factors_scaled(self._h, C.c_void_p(_ptr(u)), C.c_void_p(_ptr(vt)), float(pu),
                                              float(pv), C.c_void_p(_ptr(workspace)),
                                              C.c_void_p(_stream(stream))))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_svd_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _problems(problems, keep):
    arr = (Problem * max(1, len(problems)))()
    for i, (a, b, axes_a, axes_b) in enumerate(problems):
        arr[i].a = _desc(a, keep)
        arr[i].b = _desc(b, keep)
        xa, xb = _arr(list(axes_a), np.int32), _arr(list(axes_b), np.int32)
        arr[i].ncontract = int(len(axes_a)) if len(axes_a) == len(axes_b) else -1
        arr[i].axes_a = keep.ptr(xa, C.c_int32)
        arr[i].axes_b = keep.ptr(xb, C.c_int32)
    return arr


def _ptrs(xs, n):
    return (C.c_void_p * max(1, n))(*[_ptr(x) for x in xs])


def tune_save(path):
    """Write the process's tuning store (every autotuned choice) to a JSON file."""
    _check(lib().yastn_tune_save(os.fsencode(path)))


def tune_load(path) -> int:
    """Add a saved tuning store; returns the number of entries read."""
    n = C.c_int32()
    _check(lib().yastn_tune_load(os.fsencode(path), C.byref(n)))
    return int(n.value)


def tune_clear():
    lib().yastn_tune_clear()


class ZPlan:
    """Complex128 tensordot (yastn_zplan_*): problems as for Plan, values
    complex (interleaved); ``conj`` = CONJ_A | CONJ_B conjugates the operands."""

    def __init__(self, problems, conj=0, stream=None):
        keep = _Keep()
        arr = _problems(problems, keep)
        h = C.c_void_p()
        _check(lib().yastn_zplan(arr, len(problems), int(conj), C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h
        self.nprob = len(problems)
        ws = C.c_size_t()
        _check(lib().yastn_zplan_workspace(h, C.byref(ws)))
        self.workspace_bytes = int(ws.value)
        r = C.c_void_p()
        _check(lib().yastn_zplan_real(h, C.byref(r)))
        self._real = r

    def output(self, p: int = 0) -> Structure:
        d, n = TensorDesc(), C.c_int64()
        _check(lib().yastn_zplan_output(self._h, p, C.byref(d), C.byref(n)))
        return _structure(d, n)

    def stats(self, p: int = 0) -> dict:
        """Stats of the real form (useful_flops = 8 m k n per matched pair)."""
        st = Stats()
        _check(lib().yastn_plan_stats(self._real, p, C.byref(st)))
        return st.as_dict()

    def contract(self, a, b, c, workspace, stream=None):
        n = self.nprob
        _check(lib().yastn_zcontract(self._h, _ptrs(a, n), _ptrs(b, n), _ptrs(c, n), C.c_void_p(_ptr(workspace)),
                                     C.c_void_p(_stream(stream))))

    def autotune(self, a, b, c, workspace, reps=5, stream=None):
        n = self.nprob
        ch = C.c_int32()
        times = (C.c_float * NUM_VARIANTS)()
        _check(lib().yastn_zplan_autotune(self._h, _ptrs(a, n), _ptrs(b, n), _ptrs(c, n),
                                          C.c_void_p(_ptr(workspace)), C.c_void_p(_stream(stream)), int(reps),
                                          C.byref(ch), times))
        return int(ch.value), [float(t) for t in times]

    def set_variant(self, v: int):
        _check(lib().yastn_plan_set_variant(self._real, int(v)))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_zplan_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class SwapGate:
    """Fermionic swap gate between leg groups legs1, legs2 of a tensor
    structure (yastn_swap_*); ``fermionic``: 0/1 per charge component."""

    def __init__(self, t, legs1, legs2, fermionic):
        keep = _Keep()
        d = _desc(t, keep)
        l1, l2 = _arr(list(legs1) or [0], np.int32), _arr(list(legs2) or [0], np.int32)
        fm = _arr(list(fermionic), np.int32)
        h = C.c_void_p()
        _check(lib().yastn_swap_plan(C.byref(d), len(legs1), keep.ptr(l1, C.c_int32), len(legs2),
                                     keep.ptr(l2, C.c_int32), keep.ptr(fm, C.c_int32), C.byref(h)))
        self._h = h
        nb, ne = C.c_int64(), C.c_int64()
        _check(lib().yastn_swap_info(h, C.byref(nb), C.byref(ne)))
        self.blocks, self.elements = int(nb.value), int(ne.value)

    def apply(self, data, dtype=DTYPE_F64, stream=None):
        """Negate the odd-odd blocks of ``data`` in place (asynchronous)."""
        _check(lib().yastn_swap_gate(self._h, C.c_void_p(_ptr(data)), int(dtype), C.c_void_p(_stream(stream))))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_swap_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Ctm:
    """One CTM left move on the device (yastn_ctm_*).  ``env``: the nine
    input structures C1, C2, C3, C4, T1, T2, T3, T4, A (CTM_INPUTS order)."""

    def __init__(self, env, stream=None):
        keep = _Keep()
        arr = (TensorDesc * 9)(*[_desc(t, keep) for t in env])
        h = C.c_void_p()
        _check(lib().yastn_ctm_plan(arr, C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h

    def move(self, env, chi, tol=0.0, deg_tol=1e-10, autotune=False, stream=None):
        """Run one move on the nine device buffers ``env``; returns when done."""
        ptrs = (C.c_void_p * 9)(*[_ptr(x) for x in env])
        _check(lib().yastn_ctm_move(self._h, ptrs, int(chi), float(tol), float(deg_tol),
                                    CTM_AUTOTUNE if autotune else 0, C.c_void_p(_stream(stream))))

    def tensor(self, name):
        """(structure, numel) of a tensor of the move (CTM_NAMES)."""
        d, n, p = TensorDesc(), C.c_int64(), C.c_void_p()
        _check(lib().yastn_ctm_tensor(self._h, CTM_NAMES.index(name), C.byref(d), C.byref(n), C.byref(p)))
        return _structure(d, n)

    def copy(self, name, dst, stream=None):
        """Copy a tensor's values into dst (device, >= numel FP64)."""
        _check(lib().yastn_ctm_copy(self._h, CTM_NAMES.index(name), C.c_void_p(_ptr(dst)),
                                    C.c_void_p(_stream(stream))))

    def info(self):
        """(kept values, Jacobi sweeps, [ms: corners, halves + product, SVD,
        plans after the SVD + scaled factors, projectors + column,
        normalisation], [useful flops before the SVD, after]) of the last move."""
        k, sw = C.c_int32(), C.c_int32()
        ms = (C.c_double * 6)()
        fl = (C.c_double * 2)()
        _check(lib().yastn_ctm_info(self._h, C.byref(k), C.byref(sw), ms, fl))
        return int(k.value), int(sw.value), [float(x) for x in ms], [float(x) for x in fl]

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_ctm_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def contract_jobs(jobs, stream=None):
    """jobs: list of (Plan, a_list, b_list, c_list, workspace): one grouped launch."""
    keep = []
    arr = (Job * max(1, len(jobs)))()
    for i, (pl, a, b, c, ws) in enumerate(jobs):
        n = pl.nprob
        pa = (C.c_void_p * max(1, n))(*[_ptr(x) for x in a])
        pb = (C.c_void_p * max(1, n))(*[_ptr(x) for x in b])
        pc = (C.c_void_p * max(1, n))(*[_ptr(x) for x in c])
        keep += [pa, pb, pc]
        arr[i].plan = pl.handle
        arr[i].a = C.cast(pa, C.POINTER(C.c_void_p))
        arr[i].b = C.cast(pb, C.POINTER(C.c_void_p))
        arr[i].c = C.cast(pc, C.POINTER(C.c_void_p))
        arr[i].workspace = _ptr(ws)
    _check(lib().yastn_contract_jobs(arr, len(jobs), C.c_void_p(_stream(stream))))


def norm_workspace_bytes() -> int:
    return int(lib().yastn_norm_workspace())


def norm(x, n: int, out, workspace, dtype=DTYPE_F64, stream=None):
    """out[0] = ||x[:n]||_F, out[1] = max |x[:n]| (FP64, on the device)."""
    _check(lib().yastn_norm(C.c_void_p(_ptr(x)), int(n), int(dtype), C.c_void_p(_ptr(out)),
                            C.c_void_p(_ptr(workspace)), C.c_void_p(_stream(stream))))


class Server:
    """Continuous-batching request loop (yastn_server_*).  A request is a chain
    of single-problem plans over resident device tensors; see include/yastn.h.

    Lifetime: the C server holds the plans' handles and the device addresses
    of a0, bs and out until the request completes, so ``submit`` keeps a
    reference to every one of them (plans and tensors) until ``query`` reports
    the request done, ``forget`` drops it, or the server is closed."""

    def __init__(self, pool_bytes: int, max_ahead: int = 2, stream=None):
        h = C.c_void_p()
        _check(lib().yastn_server_create(int(pool_bytes), int(max_ahead), C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h
        self._held = {}

    def submit(self, plans, a0, bs, out) -> int:
        n = len(plans)
        pl = (C.c_void_p * n)(*[p.handle.value for p in plans])
        pb = (C.c_void_p * n)(*[_ptr(b) for b in bs])
        rq = Request(n, C.cast(pl, C.POINTER(C.c_void_p)), _ptr(a0), C.cast(pb, C.POINTER(C.c_void_p)), _ptr(out))
        rid = C.c_int64()
        _check(lib().yastn_server_submit(self._h, C.byref(rq), C.byref(rid)))
        self._held[int(rid.value)] = (list(plans), a0, list(bs), out)
        return int(rid.value)

    def held(self) -> int:
        """Requests whose plans and tensors this object still keeps alive."""
        return len(self._held)

    def step(self) -> int:
        n = C.c_int32()
        _check(lib().yastn_server_step(self._h, C.byref(n)))
        return int(n.value)

    def query(self, rid: int):
        st, lat = C.c_int32(), C.c_double()
        _check(lib().yastn_server_query(self._h, int(rid), C.byref(st), C.byref(lat)))
        if st.value == REQ_DONE:
            self._held.pop(int(rid), None)
        return int(st.value), float(lat.value)

    def forget(self, rid: int):
        _check(lib().yastn_server_forget(self._h, int(rid)))
        self._held.pop(int(rid), None)

    def drain(self):
        _check(lib().yastn_server_drain(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().yastn_server_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yastn_server_destroy(self._h)  # waits for outstanding launches
            self._h = C.c_void_p()
        self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
