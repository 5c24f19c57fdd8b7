"""Thin ctypes binding of libtnamp.so (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of its own.  Device memory for the arena can come from PyTorch
(a uint8 CUDA tensor, passed by pointer); all contraction work runs in the
HIP library.  A missing library raises instead of falling back to anything.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; TNAMP_LIB names another build of the same sources
LIB_PATH = os.environ.get("TNAMP_LIB") or os.path.join(HERE, "libtnamp.so")

TN_OK, TN_PENDING = 0, 1
TN_EINVAL, TN_ENOMEM, TN_EBUSY, TN_EDEVICE, TN_ECANCELLED, TN_ENOTFOUND = -1, -2, -3, -4, -5, -6
TN_FP32_4M, TN_FP32_3M, TN_SPLIT_BF16, TN_SPLIT_FP16, TN_BF16_1TERM = 0, 1, 2, 3, 4
PRECISIONS = {"fp32": TN_FP32_4M, "fp32_3m": TN_FP32_3M, "bf16x3": TN_SPLIT_BF16,
              "fp16x3": TN_SPLIT_FP16, "bf16x1": TN_BF16_1TERM}

EXPORTED = ["tn_ctx_create", "tn_ctx_destroy", "tn_plan_load", "tn_plan_validate",
            "tn_plan_info", "tn_plan_unload", "tn_contract_amplitudes", "tn_submit",
            "tn_poll", "tn_cancel", "tn_server_config", "tn_server_set_heavy", "tn_server_stop",
            "tn_last_exec_stats", "tn_ctx_set_profiling", "tn_ctx_set_slice_block", "tn_ctx_set_graphs", "tn_kernel_cgemm", "tn_kernel_cgemm_scratch_bytes", "tn_kernel_cgemm_shape",
            "tn_kernel_cgemm_noalloc", "tn_kernel_cgemm_noalloc_max_scratch", "tn_kernel_permute",
            "tn_last_error"]


class TnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tnamp error %d: %s" % (code, msg))
        self.code = code


class tn_plan_info_t(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_sliced", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("flops_per_slice_per_b", ctypes.c_double),
                ("flops_total_per_b", ctypes.c_double),
                ("peak_bytes_fixed", ctypes.c_uint64), ("peak_bytes_per_b", ctypes.c_uint64)]


class tn_req_stats(ctypes.Structure):
    _fields_ = [("t_arrive_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_end_ns", ctypes.c_int64),
                ("batch", ctypes.c_int32), ("plan_id", ctypes.c_int32)]


class tn_exec_stats(ctypes.Structure):
    _fields_ = [("kernels_gemm", ctypes.c_int64), ("kernels_permute", ctypes.c_int64),
                ("kernels_gather", ctypes.c_int64), ("steps_executed", ctypes.c_int64),
                ("steps_reused", ctypes.c_int64), ("chunk", ctypes.c_int32),
                ("n_chunks", ctypes.c_int32), ("slice_block", ctypes.c_int32),
                ("graph_replays", ctypes.c_int32), ("algorithmic_flops", ctypes.c_double),
                ("permute_bytes", ctypes.c_double), ("launches", ctypes.c_int64 * 7),
                ("time_ms", ctypes.c_double * 7), ("flops", ctypes.c_double * 7),
                ("bytes", ctypes.c_double * 7)]

KERNEL_CLASSES = ["cgemm_dot", "cgemm_mfma_64x64", "cgemm_mfma_128x128", "cgemm_mfma_128x16",
                  "permute", "gather", "cgemm_wave_32x32"]
GEMM_CLASSES = [0, 1, 2, 3, 6]


_lib = None


def load_library(path=LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtnamp.so is not built (run paper_2208_01498_amd.build); "
                           "there is no fallback path")
    # PyTorch ships its own HIP runtime and asks for it by a name
    # (libamdhip64.so) that differs from the runtime's soname
    # (libamdhip64.so.7).  Loaded after torch, the library binds to torch's
    # runtime; loaded before, it brings in the system runtime and torch then
    # loads a second one, and the library's runtime finds no device.  So torch,
    # when present, is loaded first: one HIP runtime per process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, sz, i32, u64p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "tn_ctx_create": [ctypes.c_int, vp, sz, ctypes.POINTER(vp)],
        "tn_ctx_destroy": [vp],
        "tn_plan_load": [vp, ctypes.c_char_p, sz, ctypes.POINTER(vp)],
        "tn_plan_validate": [ctypes.c_char_p, sz, ctypes.POINTER(tn_plan_info_t)],
        "tn_plan_info": [vp, ctypes.POINTER(tn_plan_info_t)],
        "tn_plan_unload": [vp, vp],
        "tn_contract_amplitudes": [vp, vp, u64p, i32, i32, vp, dp],
        "tn_submit": [vp, vp, u64p, i32, i32, u64p],
        "tn_poll": [vp, ctypes.c_uint64, dp, ctypes.POINTER(tn_req_stats)],
        "tn_cancel": [vp, ctypes.c_uint64],
        "tn_server_config": [vp, i32, i32],
        "tn_server_set_heavy": [vp, ctypes.c_double, i32],
        "tn_server_stop": [vp],
        "tn_last_exec_stats": [vp, ctypes.POINTER(tn_exec_stats)],
        "tn_ctx_set_profiling": [vp, i32],
        "tn_ctx_set_slice_block": [vp, i32],
        "tn_ctx_set_graphs": [vp, i32],
        "tn_kernel_cgemm": [vp, vp, vp, i32, i32, i32, i32, i32, i32, i32, ctypes.c_int64,
                            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                            ctypes.c_int64, i32, vp, sz, vp],
        "tn_kernel_permute": [vp, vp, i32, ctypes.POINTER(ctypes.c_int32), i32, vp],
        "tn_kernel_cgemm_shape": [i32, i32, i32, i32, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)],
        "tn_kernel_cgemm_noalloc": [vp, vp, vp, i32, i32, i32, i32, i32, i32, i32,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, i32, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.tn_kernel_cgemm_scratch_bytes.argtypes = [i32, i32, i32, i32, i32]
    lib.tn_kernel_cgemm_scratch_bytes.restype = ctypes.c_size_t
    lib.tn_kernel_cgemm_noalloc_max_scratch.argtypes = []
    lib.tn_kernel_cgemm_noalloc_max_scratch.restype = ctypes.c_size_t
    lib.tn_last_error.argtypes = []
    lib.tn_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        raise TnError(rc, load_library().tn_last_error().decode(errors="replace"))
    return rc


def tn_last_error():
    return load_library().tn_last_error().decode(errors="replace")


def tn_plan_validate(blob):
    info = tn_plan_info_t()
    _check(load_library().tn_plan_validate(blob, len(blob), ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def tn_ctx_create(device=0, arena_bytes=1 << 30, arena_ptr=None):
    h = ctypes.c_void_p()
    _check(load_library().tn_ctx_create(device, arena_ptr, arena_bytes, ctypes.byref(h)))
    return h


def tn_ctx_destroy(ctx):
    _check(load_library().tn_ctx_destroy(ctx))


def tn_plan_load(ctx, blob):
    h = ctypes.c_void_p()
    _check(load_library().tn_plan_load(ctx, blob, len(blob), ctypes.byref(h)))
    return h


def tn_plan_info(plan):
    info = tn_plan_info_t()
    _check(load_library().tn_plan_info(plan, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def tn_plan_unload(ctx, plan):
    _check(load_library().tn_plan_unload(ctx, plan))


def _bits(words):
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    return w, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def tn_contract_amplitudes(ctx, plan, words, precision=TN_FP32_4M, stream=None):
    w, wp = _bits(words)
    out = np.zeros(2 * len(w), dtype=np.float64)
    _check(load_library().tn_contract_amplitudes(
        ctx, plan, wp, len(w), precision, stream,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.view(np.complex128)


def tn_submit(ctx, plan, words, precision=TN_FP32_4M):
    w, wp = _bits(words)
    t = ctypes.c_uint64()
    _check(load_library().tn_submit(ctx, plan, wp, len(w), precision, ctypes.byref(t)))
    return t.value


def tn_poll(ctx, ticket, nb):
    """Returns None while pending, else (amplitudes, stats dict)."""
    out = np.zeros(2 * nb, dtype=np.float64)
    st = tn_req_stats()
    rc = load_library().tn_poll(ctx, ticket, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.byref(st))
    if rc == TN_PENDING:
        return None
    _check(rc)
    return out.view(np.complex128), {k: getattr(st, k) for k, _ in st._fields_}


def tn_cancel(ctx, ticket):
    _check(load_library().tn_cancel(ctx, ticket))


def tn_server_config(ctx, n_slots, max_batch):
    _check(load_library().tn_server_config(ctx, n_slots, max_batch))


def tn_server_set_heavy(ctx, heavy_flops, max_heavy):
    _check(load_library().tn_server_set_heavy(ctx, float(heavy_flops), max_heavy))


def tn_server_stop(ctx):
    _check(load_library().tn_server_stop(ctx))


def tn_kernel_cgemm_scratch_bytes(M, N, K, nbatch=1, nb=1):
    return load_library().tn_kernel_cgemm_scratch_bytes(M, N, K, nbatch, nb)


def tn_kernel_cgemm_shape(M, N, K, nbatch=1):
    """(kernel class, K ranges) of the GEMM of this shape; host only."""
    kind, splits = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().tn_kernel_cgemm_shape(M, N, K, nbatch, ctypes.byref(kind),
                                                ctypes.byref(splits)))
    return kind.value, splits.value


def tn_kernel_cgemm(A, B, C, M, N, K, transA=0, transB=0, nbatch=1, nb=1, sAb=0, sBb=0,
                    sCb=0, sAi=0, sBi=0, sCi=0, precision=TN_FP32_4M, scratch=None,
                    scratch_bytes=0, stream=None):
    """A, B, C, scratch: device pointers (ints), complex64 elements."""
    _check(load_library().tn_kernel_cgemm(A, B, C, M, N, K, transA, transB, nbatch, nb, sAb,
                                          sBb, sCb, sAi, sBi, sCi, precision, scratch,
                                          scratch_bytes, stream))


def tn_kernel_cgemm_noalloc(A, B, C, M, N, K, transA=0, transB=0, nbatch=1, nb=1, sAb=0,
                            sBb=0, sCb=0, sAi=0, sBi=0, sCi=0, precision=TN_FP32_4M,
                            stream=None):
    """tn_kernel_cgemm with the library's own scratch array (allocates nothing)."""
    _check(load_library().tn_kernel_cgemm_noalloc(A, B, C, M, N, K, transA, transB, nbatch, nb,
                                                  sAb, sBb, sCb, sAi, sBi, sCi, precision,
                                                  stream))


def tn_kernel_cgemm_noalloc_max_scratch():
    return load_library().tn_kernel_cgemm_noalloc_max_scratch()


def tn_kernel_permute(src, dst, rank, perm, nb=1, stream=None):
    """dst bit p takes src bit perm[p]; src, dst: device pointers (ints)."""
    arr = (ctypes.c_int32 * max(1, len(perm)))(*perm)
    _check(load_library().tn_kernel_permute(src, dst, rank, arr, nb, stream))


def tn_last_exec_stats(ctx):
    st = tn_exec_stats()
    _check(load_library().tn_last_exec_stats(ctx, ctypes.byref(st)))
    out = {}
    for k, _ in st._fields_:
        v = getattr(st, k)
        out[k] = list(v) if hasattr(v, "__len__") else v
    return out


def tn_ctx_set_slice_block(ctx, log2_block):
    _check(load_library().tn_ctx_set_slice_block(ctx, log2_block))


def tn_ctx_set_graphs(ctx, on):
    _check(load_library().tn_ctx_set_graphs(ctx, 1 if on else 0))


def tn_ctx_set_profiling(ctx, on):
    _check(load_library().tn_ctx_set_profiling(ctx, 1 if on else 0))


class Engine:
    """Context with a PyTorch-allocated arena on one GPU."""

    def __init__(self, device=0, arena_bytes=1 << 30, use_torch=True):
        self.arena = None
        ptr = None
        if use_torch:
            import torch
            self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda:%d" % device)
            ptr = ctypes.c_void_p(self.arena.data_ptr())
        self.ctx = tn_ctx_create(device, arena_bytes, ptr)
        self.plans = []

    def load(self, blob):
        p = tn_plan_load(self.ctx, blob)
        self.plans.append(p)
        return p

    def unload(self, plan):
        tn_plan_unload(self.ctx, plan)
        self.plans.remove(plan)

    def amplitudes(self, plan, words, precision=TN_FP32_4M):
        return tn_contract_amplitudes(self.ctx, plan, words, precision)

    def close(self):
        if self.ctx is not None:
            for p in self.plans:
                try:
                    tn_plan_unload(self.ctx, p)
                except TnError:
                    pass
            self.plans = []
            tn_ctx_destroy(self.ctx)
            self.ctx = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
