"""ctypes binding of libeis.so: argument marshalling only.

Every computation happens inside libeis.so on the GPU.  If the library is
missing, loading fails loudly; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import enum
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libeis.so")

EIS_MAX_D = 10**12
ABI_VERSION = 8  # must match EIS_ABI_VERSION of include/eis.h
EIS_SET_SQUAREFREE = 0
EIS_SET_PRIME = 1
EIS_FLAG_NO_GRAPHS = 1
EIS_FLAG_KERNEL_TIMES = 2
EIS_FLAG_NO_CONJUGATE_LOOKUPS = 4
EIS_FLAG_NO_SMALL_NORM_PRODUCT = 8
# eis_kernel: index of the per-kernel entries of the stats
KERNELS = ["prime_offsets", "sieve", "walk_plain", "walk_window", "build_tables", "walk_giant",
           "walk_handoff", "popcount", "giant_square", "giant_retry"]

EXPORTED_SYMBOLS = [
    "eis_config_default", "eis_create", "eis_destroy", "eis_num_candidates",
    "eis_first_candidate", "eis_count", "eis_classify", "eis_classify_async",
    "eis_last_error", "eis_count_batch", "eis_submit", "eis_wait", "eis_cancel",
    "eis_get_stats", "eis_strerror", "eis_abi_version", "eis_tune", "eis_tuned_choice",
    "eis_count_set", "eis_count_batch_set", "eis_classify_async_noalloc", "eis_tuned_shape",
]
# eis_classify_async_noalloc's limit (EIS_NOALLOC_MAX_CANDIDATES)
NOALLOC_MAX_CANDIDATES = 1 << 20


class Status(enum.IntEnum):
    OK = 0
    EINVAL = -1
    ERANGE = -2
    ENOMEM = -3
    EDEVICE = -4
    EBUSY = -5
    ECANCELED = -6
    ETIMEDOUT = -7
    EINTERNAL = -8


class Method(enum.IntEnum):
    BABY = 0
    INFRA = 1
    AUTO = 2


class EisConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("method", ctypes.c_int),
        ("mem_budget_bytes", ctypes.c_uint64),
        ("max_steps_per_d", ctypes.c_uint64),
        ("window_scale", ctypes.c_double),
        ("serve_slots", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("tune_cache_path", ctypes.c_char_p),
    ]


class EisStats(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_uint64),
        ("discriminants", ctypes.c_uint64),
        ("baby_steps", ctypes.c_uint64),
        ("giant_steps", ctypes.c_uint64),
        ("refills", ctypes.c_uint64),
        ("fallbacks", ctypes.c_uint64),
        ("requests_done", ctypes.c_uint64),
        ("last_walk_ms", ctypes.c_double),
        ("last_total_ms", ctypes.c_double),
        ("kernel_steps", ctypes.c_uint64 * len(KERNELS)),
        ("kernel_launches", ctypes.c_uint64 * len(KERNELS)),
        ("kernel_ms", ctypes.c_double * len(KERNELS)),
        ("giant_compositions", ctypes.c_uint64),
        ("giant_euclid_steps", ctypes.c_uint64),
        ("giant_reduce_steps", ctypes.c_uint64),
        ("giant_gcd_branches", ctypes.c_uint64),
        ("giant_lookups", ctypes.c_uint64),
        ("window_entries", ctypes.c_uint64),
        ("giant_retries", ctypes.c_uint64),
        ("giant_compose_phases", ctypes.c_uint64),
        ("giant_compose_lanes", ctypes.c_uint64),
        ("giant_walk_phases", ctypes.c_uint64),
        ("giant_walk_lanes", ctypes.c_uint64),
        ("serve_bytes_reserved", ctypes.c_uint64),
        ("serve_bytes_budget", ctypes.c_uint64),
        ("giant_xgcd_steps", ctypes.c_uint64),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name.startswith("kernel_") else v
        return out


class EisError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = int(status)
        try:
            name = Status(self.status).name
        except ValueError:
            name = str(self.status)
        super().__init__(f"{where}: {name} ({eis_strerror(self.status)})")


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libeis.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise OSError(f"{_LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch ships its own HIP runtime (same soname).  Load it first so that
    # libeis.so binds to that copy and the process has ONE HIP runtime,
    # whose device memory and streams both sides then share.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(_LIB_PATH)
    u64, c_int, vp, sz = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    L.eis_config_default.argtypes = [P(EisConfig)]; L.eis_config_default.restype = None
    L.eis_create.argtypes = [P(EisConfig), P(vp)]; L.eis_create.restype = c_int
    L.eis_destroy.argtypes = [vp]; L.eis_destroy.restype = None
    L.eis_num_candidates.argtypes = [u64, u64]; L.eis_num_candidates.restype = u64
    L.eis_first_candidate.argtypes = [u64]; L.eis_first_candidate.restype = u64
    L.eis_count.argtypes = [vp, u64, u64, P(u64), P(u64)]; L.eis_count.restype = c_int
    L.eis_classify.argtypes = [vp, u64, u64, vp, vp, sz, P(u64), P(u64)]
    L.eis_classify.restype = c_int
    L.eis_classify_async.argtypes = [vp, u64, u64, vp, vp, vp, vp]
    L.eis_classify_async.restype = c_int
    L.eis_classify_async_noalloc.argtypes = [vp, u64, u64, vp, vp, vp, vp]
    L.eis_classify_async_noalloc.restype = c_int
    L.eis_last_error.argtypes = [vp]; L.eis_last_error.restype = c_int
    L.eis_count_batch.argtypes = [vp, vp, vp, sz, vp, vp]; L.eis_count_batch.restype = c_int
    L.eis_submit.argtypes = [vp, u64, u64, P(u64)]; L.eis_submit.restype = c_int
    L.eis_wait.argtypes = [vp, u64, ctypes.c_int64, P(u64), P(u64)]; L.eis_wait.restype = c_int
    L.eis_cancel.argtypes = [vp, u64]; L.eis_cancel.restype = c_int
    L.eis_get_stats.argtypes = [vp, P(EisStats)]; L.eis_get_stats.restype = c_int
    L.eis_strerror.argtypes = [c_int]; L.eis_strerror.restype = ctypes.c_char_p
    L.eis_abi_version.argtypes = []; L.eis_abi_version.restype = c_int
    L.eis_tune.argtypes = [vp]; L.eis_tune.restype = c_int
    L.eis_count_set.argtypes = [vp, c_int, u64, u64, P(u64), P(u64)]
    L.eis_count_set.restype = c_int
    L.eis_count_batch_set.argtypes = [vp, c_int, vp, vp, sz, vp, vp]
    L.eis_count_batch_set.restype = c_int
    L.eis_tuned_choice.argtypes = [vp, u64, P(c_int), P(ctypes.c_double)]
    L.eis_tuned_choice.restype = c_int
    L.eis_tuned_shape.argtypes = [vp, u64, P(ctypes.c_uint32), P(u64)]
    L.eis_tuned_shape.restype = c_int
    if L.eis_abi_version() != ABI_VERSION:
        raise OSError(f"{_LIB_PATH} has ABI version {L.eis_abi_version()}, this binding "
                      f"expects {ABI_VERSION}: rebuild it")
    _lib = L
    return L


def eis_num_candidates(a: int, b: int) -> int:
    return int(lib().eis_num_candidates(a, b))


def eis_first_candidate(a: int) -> int:
    return int(lib().eis_first_candidate(a))


def eis_strerror(status: int) -> str:
    return lib().eis_strerror(int(status)).decode()


def eis_abi_version() -> int:
    return int(lib().eis_abi_version())


def _check(rc: int, where: str):
    if rc != 0:
        raise EisError(rc, where)


class Context:
    """Owns an ``eis_ctx``.  Methods mirror the C calls of the same names."""

    def __init__(self, device: int = 0, method: int = Method.AUTO, mem_budget_bytes: int = 0,
                 max_steps_per_d: int = 0, window_scale: float = 0.0, serve_slots: int = 0,
                 flags: int = 0, tune_cache_path: str | None = None):
        L = lib()
        cfg = EisConfig()
        L.eis_config_default(ctypes.byref(cfg))
        cfg.device = device
        cfg.method = int(method)
        cfg.mem_budget_bytes = mem_budget_bytes
        cfg.max_steps_per_d = max_steps_per_d
        cfg.window_scale = window_scale
        cfg.serve_slots = serve_slots
        cfg.flags = flags
        path = tune_cache_path.encode() if tune_cache_path else None
        cfg.tune_cache_path = path
        h = ctypes.c_void_p()
        _check(L.eis_create(ctypes.byref(cfg), ctypes.byref(h)), "eis_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().eis_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    # -- calls ----------------------------------------------------------
    def eis_count(self, a: int, b: int):
        s, e = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().eis_count(self._h, a, b, ctypes.byref(s), ctypes.byref(e)), "eis_count")
        return int(s.value), int(e.value)

    def eis_classify(self, a: int, b: int):
        """(sqfree_bits, eis_bits, n_sqfree, n_eis) with numpy uint8 bitmaps."""
        import numpy as np
        nb = max(1, (eis_num_candidates(a, b) + 7) // 8)
        sq = np.zeros(nb, dtype=np.uint8)
        eb = np.zeros(nb, dtype=np.uint8)
        s, e = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().eis_classify(self._h, a, b, sq.ctypes.data, eb.ctypes.data, nb,
                                  ctypes.byref(s), ctypes.byref(e)), "eis_classify")
        return sq, eb, int(s.value), int(e.value)

    def eis_classify_async(self, a: int, b: int, sq_ptr: int, eis_ptr: int, counts_ptr: int,
                           stream: int = 0):
        """Device-pointer variant (e.g. torch tensors' data_ptr(), and
        torch.cuda.current_stream().cuda_stream)."""
        _check(lib().eis_classify_async(self._h, a, b, sq_ptr or None, eis_ptr or None,
                                        counts_ptr or None, stream or None),
               "eis_classify_async")

    def eis_classify_async_noalloc(self, a: int, b: int, sq_ptr: int, eis_ptr: int,
                                   counts_ptr: int, stream: int = 0):
        """Like eis_classify_async, but the library allocates nothing (its
        kernels work in a fixed device scratch; at most
        EIS_NOALLOC_MAX_CANDIDATES candidates)."""
        _check(lib().eis_classify_async_noalloc(self._h, a, b, sq_ptr or None, eis_ptr or None,
                                                counts_ptr or None, stream or None),
               "eis_classify_async_noalloc")

    def eis_last_error(self) -> int:
        return int(lib().eis_last_error(self._h))

    def eis_count_batch(self, a, b):
        import numpy as np
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.uint64))
        if a.shape != b.shape:
            raise ValueError("a and b must have the same length")
        n = a.size
        s = np.zeros(max(1, n), dtype=np.uint64)
        e = np.zeros(max(1, n), dtype=np.uint64)
        _check(lib().eis_count_batch(self._h, a.ctypes.data, b.ctypes.data, n, s.ctypes.data,
                                     e.ctypes.data), "eis_count_batch")
        return s[:n], e[:n]

    def eis_count_set(self, set_: int, a: int, b: int):
        s, e = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().eis_count_set(self._h, int(set_), a, b, ctypes.byref(s), ctypes.byref(e)),
               "eis_count_set")
        return int(s.value), int(e.value)

    def eis_count_batch_set(self, set_: int, a, b):
        import numpy as np
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.uint64))
        if a.shape != b.shape:
            raise ValueError("a and b must have the same length")
        n = a.size
        s = np.zeros(max(1, n), dtype=np.uint64)
        e = np.zeros(max(1, n), dtype=np.uint64)
        _check(lib().eis_count_batch_set(self._h, int(set_), a.ctypes.data, b.ctypes.data, n,
                                         s.ctypes.data, e.ctypes.data), "eis_count_batch_set")
        return s[:n], e[:n]

    def eis_submit(self, a: int, b: int) -> int:
        t = ctypes.c_uint64(0)
        _check(lib().eis_submit(self._h, a, b, ctypes.byref(t)), "eis_submit")
        return int(t.value)

    def eis_wait(self, ticket: int, timeout_us: int = -1):
        s, e = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().eis_wait(self._h, ticket, timeout_us, ctypes.byref(s), ctypes.byref(e)),
               "eis_wait")
        return int(s.value), int(e.value)

    def eis_wait_status(self, ticket: int, timeout_us: int = -1):
        s, e = ctypes.c_uint64(0), ctypes.c_uint64(0)
        rc = lib().eis_wait(self._h, ticket, timeout_us, ctypes.byref(s), ctypes.byref(e))
        return int(rc), int(s.value), int(e.value)

    def eis_cancel(self, ticket: int):
        _check(lib().eis_cancel(self._h, ticket), "eis_cancel")

    def eis_tune(self):
        _check(lib().eis_tune(self._h), "eis_tune")

    def eis_tuned_choice(self, d: int):
        """(method, window_scale) in force for height d."""
        m, w = ctypes.c_int(0), ctypes.c_double(0.0)
        _check(lib().eis_tuned_choice(self._h, d, ctypes.byref(m), ctypes.byref(w)),
               "eis_tuned_choice")
        return Method(m.value), float(w.value)

    def eis_tuned_shape(self, d: int):
        """(walk chunk, candidates per pass) in force for height d."""
        ch, ps = ctypes.c_uint32(0), ctypes.c_uint64(0)
        _check(lib().eis_tuned_shape(self._h, d, ctypes.byref(ch), ctypes.byref(ps)),
               "eis_tuned_shape")
        return int(ch.value), int(ps.value)

    def eis_get_stats(self):
        st = EisStats()
        _check(lib().eis_get_stats(self._h, ctypes.byref(st)), "eis_get_stats")
        return st.as_dict()
