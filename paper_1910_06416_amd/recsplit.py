"""Python binding of librecsplit (argument marshalling only).

Every step of construction and lookup runs in the HIP kernels of
``librecsplit.so``; PyTorch only provides device memory and the current
stream.  There is no CPU fallback: if the library is missing or no GPU is
present the calls raise.

Keys are either a CUDA tensor of 64-bit integers (int64 or uint64, viewed as
unsigned) or a pair ``(data, offsets)`` of CUDA tensors for byte strings:
``data`` uint8 with the concatenated bytes, ``offsets`` int64/uint64 with n+1
non-decreasing entries.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librecsplit.so")
TORCH_ALLOC_PATH = os.path.join(HERE, "libtorchalloc.so")

RS_OK, RS_EINVAL, RS_EDUPLICATE, RS_ENOMEM, RS_EDEVICE, RS_ESEARCH, RS_EFORMAT, RS_EBUSY = range(8)
RS_KEYS_U64, RS_KEYS_BYTES = 1, 2
STATUS_NAMES = {0: "RS_OK", 1: "RS_EINVAL", 2: "RS_EDUPLICATE", 3: "RS_ENOMEM", 4: "RS_EDEVICE", 5: "RS_ESEARCH",
                6: "RS_EFORMAT", 7: "RS_EBUSY"}


class RecSplitError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class rs_keys(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n", ctypes.c_uint64)]


class rs_options(ctypes.Structure):
    _fields_ = [("seed_cap", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("stage_from", ctypes.c_uint32),
                ("group_max", ctypes.c_uint32), ("waves", ctypes.c_uint32), ("wait_limit", ctypes.c_uint32),
                ("gr_table_max", ctypes.c_uint32), ("leaf_slack", ctypes.c_uint32)]


RS_OPT_TIMING, RS_OPT_TUNED, RS_OPT_NO_SAMPLES = 1, 2, 4


class rs_schedule(ctypes.Structure):
    _fields_ = [("stage_from", ctypes.c_uint32), ("group_max", ctypes.c_uint32), ("waves", ctypes.c_uint32),
                ("variants", ctypes.c_uint32), ("search_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("tune_ms", ctypes.c_double)]


class rs_build_stats(ctypes.Structure):
    _fields_ = [("ms_signature", ctypes.c_double), ("ms_scatter", ctypes.c_double), ("ms_search", ctypes.c_double),
                ("ms_offsets", ctypes.c_double), ("ms_fill", ctypes.c_double), ("ms_device", ctypes.c_double),
                ("n", ctypes.c_uint64), ("nb", ctypes.c_uint64), ("maxm", ctypes.c_uint64),
                ("tree_bits", ctypes.c_uint64), ("blob_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("refills", ctypes.c_uint64)]


class rs_server_stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("batched_requests", ctypes.c_uint64), ("max_batch", ctypes.c_uint64),
                ("max_concurrent_batches", ctypes.c_uint64), ("peak_in_flight_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("max_queue", ctypes.c_uint32), ("lookup_cus", ctypes.c_uint32)]


class rs_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("build_workers", ctypes.c_uint32),
                ("lookup_cus", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 4)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librecsplit.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch brings its own HIP runtime; loading it first makes the library
        # bind to that same runtime, so streams and memory from torch are valid
        # in the library (two runtimes in one process do not share them)
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.rs_build.argtypes = [ctypes.POINTER(rs_keys), U32, U32, P, ctypes.POINTER(P)]
        L.rs_build_ex.argtypes = [ctypes.POINTER(rs_keys), U32, U32, ctypes.POINTER(rs_options), P,
                                  ctypes.POINTER(P)]
        L.rs_lookup.argtypes = [P, ctypes.POINTER(rs_keys), P, P]
        L.rs_blob_bytes.argtypes = [P]
        L.rs_blob_bytes.restype = U64
        L.rs_blob_to_host.argtypes = [P, P, U64]
        L.rs_blob_from_host.argtypes = [P, U64, P, ctypes.POINTER(P)]
        L.rs_blob_device_ptr.argtypes = [P]
        L.rs_blob_device_ptr.restype = P
        L.rs_blob_info.argtypes = [P, ctypes.POINTER(U64), ctypes.POINTER(U32), ctypes.POINTER(U32)]
        L.rs_blob_free.argtypes = [P]
        L.rs_blob_free.restype = None
        L.rs_last_error.restype = ctypes.c_char_p
        L.rs_version.restype = ctypes.c_char_p
        L.rs_tables.argtypes = [U32, U32, P, P, P]
        L.rs_tables_ex.argtypes = [U32, U32, U32, P, P, P]
        L.rs_tables_packed.argtypes = [U32, U32, U32, P]
        L.rs_tables_range.argtypes = [U32, U32, U32, U32, P, P, P, P]
        L.rs_last_build_stats.argtypes = [ctypes.POINTER(rs_build_stats)]
        L.rs_build_batch.argtypes = [ctypes.POINTER(rs_keys), U32, P, P, ctypes.POINTER(rs_options), P, P, P]
        PU64, PI, PD, PU32 = (ctypes.POINTER(U64), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(U32))
        L.rs_server_create.argtypes = [U64, U32, ctypes.POINTER(rs_options), ctypes.POINTER(P)]
        L.rs_server_create_ex.argtypes = [ctypes.POINTER(rs_server_config), ctypes.POINTER(rs_options),
                                          ctypes.POINTER(P)]
        L.rs_server_submit_build.argtypes = [P, ctypes.POINTER(rs_keys), U32, U32, PU64]
        L.rs_server_submit_lookup.argtypes = [P, P, ctypes.POINTER(rs_keys), P, PU64]
        L.rs_server_poll.argtypes = [P, U64, PI, PI, ctypes.POINTER(P), PD, PU32]
        L.rs_server_wait.argtypes = [P, U64, PI, ctypes.POINTER(P), PD, PU32]
        L.rs_server_get_stats.argtypes = [P, ctypes.POINTER(rs_server_stats)]
        L.rs_server_destroy.argtypes = [P]
        L.rs_server_destroy.restype = None
        L.rs_autotune.argtypes = [U32, U32, U64, ctypes.c_double, P, ctypes.POINTER(rs_schedule)]
        L.rs_schedule_get.argtypes = [U32, U32, ctypes.POINTER(rs_schedule)]
        L.rs_schedule_set.argtypes = [U32, U32, ctypes.POINTER(rs_schedule)]
        L.rs_schedule_clear.argtypes = []
        L.rs_schedule_clear.restype = None
        L.rs_plan_create.argtypes = [ctypes.POINTER(rs_keys), U32, P, P, ctypes.POINTER(rs_options), P,
                                     ctypes.POINTER(P), P, P]
        L.rs_plan_run.argtypes = [P, P, P, P]
        L.rs_plan_info.argtypes = [P, ctypes.POINTER(U32), ctypes.POINTER(U64), ctypes.POINTER(U64),
                                   ctypes.POINTER(U64)]
        L.rs_plan_destroy.argtypes = [P]
        L.rs_plan_destroy.restype = None
        L.rs_set_allocator.argtypes = [P, P, P]
        L.rs_build_noalloc.argtypes = [ctypes.POINTER(rs_keys), U32, U32, P, U64, ctypes.POINTER(U64), P]
        for f in ("rs_build", "rs_build_ex", "rs_lookup", "rs_blob_to_host", "rs_blob_from_host", "rs_blob_info",
                  "rs_tables", "rs_last_build_stats", "rs_build_batch", "rs_server_create", "rs_server_create_ex", "rs_server_submit_build",
                  "rs_server_submit_lookup", "rs_server_poll", "rs_server_wait", "rs_server_get_stats", "rs_autotune",
                  "rs_schedule_get", "rs_schedule_set", "rs_plan_create", "rs_plan_run", "rs_plan_info",
                  "rs_set_allocator", "rs_tables_ex", "rs_tables_packed", "rs_tables_range", "rs_build_noalloc"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
        use_torch_allocator()
    return _lib


_torch_alloc = None


def use_torch_allocator():
    """Give the library's device memory to PyTorch's caching allocator (the
    default of this binding): workspaces and blobs then come from torch's pool
    and count in torch.cuda.memory_allocated().  The allocation functions are
    native (libtorchalloc.so), so no Python runs per allocation."""
    global _torch_alloc
    import torch

    if torch.cuda.is_available():
        torch.cuda.init()  # the caching allocator serves devices only after torch's lazy init
    if _torch_alloc is None:
        if not os.path.exists(TORCH_ALLOC_PATH):
            raise RuntimeError(f"{TORCH_ALLOC_PATH} is not built; run __graft_entry__.build() first")
        _torch_alloc = ctypes.CDLL(TORCH_ALLOC_PATH)
    alloc = ctypes.cast(_torch_alloc.rs_torch_alloc, ctypes.c_void_p)
    free = ctypes.cast(_torch_alloc.rs_torch_free, ctypes.c_void_p)
    _check(lib().rs_set_allocator(alloc, free, None))


def use_default_allocator():
    """The library's own stream-ordered hipMallocAsync / hipFreeAsync."""
    _check(lib().rs_set_allocator(None, None, None))


def set_allocator(alloc, free, ctx=None):
    """Install an allocator given as ctypes function pointers matching
    rs_alloc_fn / rs_free_fn (the caller keeps them alive)."""
    _check(lib().rs_set_allocator(ctypes.cast(alloc, ctypes.c_void_p), ctypes.cast(free, ctypes.c_void_p), ctx))


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _check(rc: int):
    if rc != RS_OK:
        raise RecSplitError(rc, lib().rs_last_error().decode())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_keys(keys) -> rs_keys:
    import torch

    if isinstance(keys, tuple):
        data, offsets = keys
        if not (data.is_cuda and offsets.is_cuda):
            raise ValueError("keys must be CUDA tensors")
        if data.dtype != torch.uint8 or offsets.dtype not in (torch.int64, torch.uint64):
            raise ValueError("byte keys need (uint8 data, int64/uint64 offsets)")
        if not (data.is_contiguous() and offsets.is_contiguous()):
            raise ValueError("key tensors must be contiguous")
        return rs_keys(RS_KEYS_BYTES, data.data_ptr(), offsets.data_ptr(), offsets.numel() - 1)
    if not keys.is_cuda or keys.dtype not in (torch.int64, torch.uint64) or not keys.is_contiguous():
        raise ValueError("u64 keys must be a contiguous CUDA int64/uint64 tensor")
    return rs_keys(RS_KEYS_U64, keys.data_ptr(), None, keys.numel())


class Blob:
    """A built structure resident in device memory."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise RuntimeError("blob was freed")
        return self._h

    @property
    def nbytes(self) -> int:
        return int(lib().rs_blob_bytes(self.handle))

    def info(self):
        n, leaf, bucket = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().rs_blob_info(self.handle, ctypes.byref(n), ctypes.byref(leaf), ctypes.byref(bucket)))
        return n.value, leaf.value, bucket.value

    def bits_per_key(self) -> float:
        return 8.0 * self.nbytes / self.info()[0]

    def to_bytes(self) -> bytes:
        buf = np.zeros(self.nbytes, dtype=np.uint8)
        _check(lib().rs_blob_to_host(self.handle, buf.ctypes.data, buf.size))
        return buf.tobytes()

    def lookup(self, keys, out=None, stream=None):
        return lookup(self, keys, out=out, stream=stream)

    def free(self):
        if self._h:
            lib().rs_blob_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _options(seed_cap=0, timing=False, tuned=False, stage_from=0, group_max=0, waves=0, wait_limit=0,
             gr_table_max=0, leaf_slack=0, samples=True) -> rs_options:
    flags = (RS_OPT_TIMING if timing else 0) | (RS_OPT_TUNED if tuned else 0) | (0 if samples else RS_OPT_NO_SAMPLES)
    return rs_options(seed_cap, flags, stage_from, group_max, waves, wait_limit, gr_table_max, leaf_slack)


def build(keys, leaf: int, bucket: int, seed_cap: int = 0, timing: bool = False, stage_from: int = 0,
          group_max: int = 0, waves: int = 0, tuned: bool = False, wait_limit: int = 0, gr_table_max: int = 0,
          leaf_slack: int = 0, samples: bool = True, stream=None) -> Blob:
    """Build the minimal perfect hash function of a device key set.  With
    timing=True the per-phase device times are available from last_build_stats().
    tuned=True takes the search schedule of (leaf, bucket) from the schedule
    table (see autotune); stage_from / group_max / waves override it.  Schedules
    never change the result.  wait_limit, gr_table_max and leaf_slack are the
    rs_options fields of those names; samples=False sets RS_OPT_NO_SAMPLES."""
    k = _as_keys(keys)
    h = ctypes.c_void_p()
    opts = _options(seed_cap, timing, tuned, stage_from, group_max, waves, wait_limit, gr_table_max, leaf_slack,
                    samples)
    _check(lib().rs_build_ex(ctypes.byref(k), leaf, bucket, ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
    return Blob(h)


def build_batch(key_sets, leafs, buckets, seed_cap: int = 0, timing: bool = False, stage_from: int = 0,
                group_max: int = 0, waves: int = 0, tuned: bool = False, gr_table_max: int = 0, leaf_slack: int = 0,
                stream=None):
    """Build many MPHFs in one call.  Returns (blobs, statuses): blobs[i] is a
    Blob or None when statuses[i] != RS_OK.  Raises only when the call itself
    fails (no build could be attempted)."""
    count = len(key_sets)
    if isinstance(leafs, int):
        leafs = [leafs] * count
    if isinstance(buckets, int):
        buckets = [buckets] * count
    arr = (rs_keys * count)(*[_as_keys(k) for k in key_sets])
    lf = np.ascontiguousarray(leafs, dtype=np.uint32)
    bk = np.ascontiguousarray(buckets, dtype=np.uint32)
    outs = (ctypes.c_void_p * count)()
    status = np.zeros(count, dtype=np.int32)
    opts = _options(seed_cap, timing, tuned, stage_from, group_max, waves, 0, gr_table_max, leaf_slack)
    rc = lib().rs_build_batch(arr, count, lf.ctypes.data, bk.ctypes.data, ctypes.byref(opts), _stream(stream),
                              ctypes.cast(outs, ctypes.c_void_p), status.ctypes.data)
    blobs = [Blob(ctypes.c_void_p(outs[i])) if outs[i] else None for i in range(count)]
    if rc != RS_OK and not any(b is not None for b in blobs) and not status.any():
        _check(rc)
    return blobs, [int(x) for x in status]


def _schedule_dict(sc: rs_schedule) -> dict:
    return {name: getattr(sc, name) for name, _ in rs_schedule._fields_}


def autotune(leaf: int, bucket: int, keys_hint: int = 0, budget_ms: float = 0.0, stream=None) -> dict:
    """Time the seed search of (leaf, bucket) on synthetic calibration keys
    (about keys_hint of them) with several schedules, store the fastest in the
    schedule table and return it."""
    sc = rs_schedule()
    _check(lib().rs_autotune(leaf, bucket, keys_hint, float(budget_ms), _stream(stream), ctypes.byref(sc)))
    return _schedule_dict(sc)


def get_schedule(leaf: int, bucket: int):
    """The table's schedule of (leaf, bucket), or None."""
    sc = rs_schedule()
    if lib().rs_schedule_get(leaf, bucket, ctypes.byref(sc)) != RS_OK:
        return None
    return _schedule_dict(sc)


def set_schedule(leaf: int, bucket: int, stage_from: int, group_max: int, waves: int):
    """Store a schedule (for example one saved from an earlier autotune)."""
    sc = rs_schedule(stage_from, group_max, waves)
    _check(lib().rs_schedule_set(leaf, bucket, ctypes.byref(sc)))


def clear_schedules():
    lib().rs_schedule_clear()


class Plan:
    """The construction of a fixed batch shape captured into one HIP graph
    (rs_plan_* in recsplit.h).  The key tensors must stay alive, at the same
    addresses, until close(); run() rebuilds from their current contents."""

    def __init__(self, key_sets, leafs, buckets, seed_cap: int = 0, stage_from: int = 0, group_max: int = 0,
                 waves: int = 0, tuned: bool = False, stream=None):
        count = len(key_sets)
        if isinstance(leafs, int):
            leafs = [leafs] * count
        if isinstance(buckets, int):
            buckets = [buckets] * count
        self._keep = list(key_sets)
        self._count = count
        arr = (rs_keys * count)(*[_as_keys(k) for k in key_sets])
        lf = np.ascontiguousarray(leafs, dtype=np.uint32)
        bk = np.ascontiguousarray(buckets, dtype=np.uint32)
        first = (ctypes.c_void_p * count)()
        status = np.zeros(count, dtype=np.int32)
        opts = _options(seed_cap, False, tuned, stage_from, group_max, waves)
        self._h = ctypes.c_void_p()
        _check(lib().rs_plan_create(arr, count, lf.ctypes.data, bk.ctypes.data, ctypes.byref(opts),
                                    _stream(stream), ctypes.byref(self._h), ctypes.cast(first, ctypes.c_void_p),
                                    status.ctypes.data))
        self.first = [Blob(ctypes.c_void_p(first[i])) if first[i] else None for i in range(count)]

    def run(self, stream=None):
        """Rebuild every set; returns (blobs, statuses) like build_batch."""
        outs = (ctypes.c_void_p * self._count)()
        status = np.zeros(self._count, dtype=np.int32)
        rc = lib().rs_plan_run(self._h, _stream(stream), ctypes.cast(outs, ctypes.c_void_p), status.ctypes.data)
        blobs = [Blob(ctypes.c_void_p(outs[i])) if outs[i] else None for i in range(self._count)]
        if rc != RS_OK and not any(b is not None for b in blobs) and not status.any():
            _check(rc)
        return blobs, [int(x) for x in status]

    def info(self) -> dict:
        cap, words, runs, fb = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().rs_plan_info(self._h, ctypes.byref(cap), ctypes.byref(words), ctypes.byref(runs),
                                  ctypes.byref(fb)))
        return {"bucket_cap": cap.value, "capacity_words": words.value, "runs": runs.value, "fallbacks": fb.value}

    def close(self):
        if self._h:
            lib().rs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_noalloc(keys, leaf: int, bucket: int, out, stream=None) -> int:
    """rs_build_noalloc: write the serialized structure into `out` (a CUDA
    uint8 tensor) without any device allocation by the library; returns its
    size in bytes."""
    k = _as_keys(keys)
    size = ctypes.c_uint64()
    _check(lib().rs_build_noalloc(ctypes.byref(k), leaf, bucket, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                  ctypes.byref(size), _stream(stream)))
    return size.value


def lookup(blob: Blob, keys, out=None, stream=None):
    """Ranks of the keys (a CUDA int64 tensor holding the unsigned values)."""
    import torch

    k = _as_keys(keys)
    if out is None:
        out = torch.empty(int(k.n), dtype=torch.int64, device="cuda")
    if out.numel() != k.n or not out.is_contiguous():
        raise ValueError("output tensor has the wrong shape")
    _check(lib().rs_lookup(blob.handle, ctypes.byref(k), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def from_bytes(data: bytes, stream=None) -> Blob:
    buf = np.frombuffer(data, dtype=np.uint8).copy()
    h = ctypes.c_void_p()
    _check(lib().rs_blob_from_host(buf.ctypes.data, buf.size, _stream(stream), ctypes.byref(h)))
    return Blob(h)


def packed_table(leaf: int, maxm: int, gr_table_max: int = 0):
    """The library's per-size words r | N << 5 | F << 16, or None when some
    size up to maxm does not fit."""
    out = np.zeros(maxm + 1, dtype=np.uint32)
    rc = lib().rs_tables_packed(leaf, maxm, gr_table_max, out.ctypes.data)
    if rc == RS_EINVAL:
        return None
    _check(rc)
    return out


def tables(leaf: int, maxm: int, gr_table_max: int = 0):
    """The library's per-size tables (Golomb-Rice parameter, fixed bits and
    coded nodes of a subtree) for sizes 0..maxm."""
    r = np.zeros(maxm + 1, dtype=np.uint32)
    F = np.zeros(maxm + 1, dtype=np.uint32)
    N = np.zeros(maxm + 1, dtype=np.uint32)
    _check(lib().rs_tables_ex(leaf, maxm, gr_table_max, r.ctypes.data, F.ctypes.data, N.ctypes.data))
    return r, F, N


def range_tables(leaf: int, maxm: int, leaf_slack: int, gr_table_max: int = 0):
    """rs_tables_range: (r, F, N, Q) of the non-minimal variant with the given
    slack, Q[m] being the output values of a subtree of m keys."""
    out = [np.zeros(maxm + 1, dtype=np.uint32) for _ in range(4)]
    _check(lib().rs_tables_range(leaf, maxm, gr_table_max, leaf_slack, *[a.ctypes.data for a in out]))
    return tuple(out)


class Server:
    """Continuous-batching build/lookup server (see rs_server_* in recsplit.h).
    Key tensors passed to submit_* must stay alive until the request completes;
    the server keeps a reference to them until then."""

    def __init__(self, budget_bytes: int, build_workers: int = 2, stage_from: int = 0, group_max: int = 0,
                 waves: int = 0, tuned: bool = False, lookup_cus: int = 0):
        self._h = ctypes.c_void_p()
        opts = _options(0, False, tuned, stage_from, group_max, waves)
        cfg = rs_server_config(budget_bytes, build_workers, lookup_cus)
        _check(lib().rs_server_create_ex(ctypes.byref(cfg), ctypes.byref(opts), ctypes.byref(self._h)))
        self._keep = {}

    def submit_build(self, keys, leaf: int, bucket: int) -> int:
        k = _as_keys(keys)
        t = ctypes.c_uint64()
        _check(lib().rs_server_submit_build(self._h, ctypes.byref(k), leaf, bucket, ctypes.byref(t)))
        self._keep[t.value] = keys
        return t.value

    def submit_lookup(self, blob: Blob, keys, out) -> int:
        k = _as_keys(keys)
        t = ctypes.c_uint64()
        _check(lib().rs_server_submit_lookup(self._h, blob.handle, ctypes.byref(k), ctypes.c_void_p(out.data_ptr()),
                                             ctypes.byref(t)))
        self._keep[t.value] = (keys, out, blob)
        return t.value

    def _result(self, t, status, h, lat, bs):
        self._keep.pop(t, None)
        blob = Blob(ctypes.c_void_p(h.value)) if h.value else None
        return {"status": status.value, "blob": blob, "latency_ms": lat.value, "batch_size": bs.value}

    def poll(self, ticket: int):
        done, status, h, lat, bs = ctypes.c_int(), ctypes.c_int(), ctypes.c_void_p(), ctypes.c_double(), U32()
        _check(lib().rs_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(status), ctypes.byref(h),
                                    ctypes.byref(lat), ctypes.byref(bs)))
        return self._result(ticket, status, h, lat, bs) if done.value else None

    def wait(self, ticket: int):
        status, h, lat, bs = ctypes.c_int(), ctypes.c_void_p(), ctypes.c_double(), U32()
        _check(lib().rs_server_wait(self._h, ticket, ctypes.byref(status), ctypes.byref(h), ctypes.byref(lat),
                                    ctypes.byref(bs)))
        return self._result(ticket, status, h, lat, bs)

    def stats(self) -> dict:
        st = rs_server_stats()
        _check(lib().rs_server_get_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in rs_server_stats._fields_}

    def close(self):
        if self._h:
            lib().rs_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


U32 = ctypes.c_uint32


def last_build_stats() -> dict:
    st = rs_build_stats()
    _check(lib().rs_last_build_stats(ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in rs_build_stats._fields_}


def version() -> str:
    return lib().rs_version().decode()


def device_keys(keys):
    """Copy host keys (numpy uint64 array, or (uint8 data, uint64 offsets)) to the GPU."""
    import torch

    if isinstance(keys, tuple):
        data, offsets = keys
        d = torch.from_numpy(np.ascontiguousarray(data, dtype=np.uint8)).cuda()
        o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).cuda()
        return d, o
    return torch.from_numpy(np.ascontiguousarray(keys, dtype=np.uint64).view(np.int64)).cuda()
