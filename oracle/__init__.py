"""RecSplit CPU oracle (test infrastructure only).

ctypes binding of ``recsplit_oracle.c``: a plain, single-threaded C
implementation of the whole RecSplit construction and lookup, written from the
paper (Esposito, Mueller Graf, Vigna 2019).  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may use this package; the GPU
library never imports, links or calls it.

Keys are passed either as a ``numpy.uint64`` array, or as a pair
``(data: uint8[], offsets: uint64[n+1])`` for byte strings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "recsplit_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, EDUPLICATE, ENOMEM, ESEARCH, EFORMAT = 0, 1, 2, 3, 5, 6
KEYS_U64, KEYS_BYTES = 1, 2


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def compile_library() -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation flags)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            compile_library()
        _lib = ctypes.CDLL(LIB)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
U32, U64, F64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double


def _declare(L):
    L.orc_splitmix64_stream.argtypes = [U64, U64, P]
    L.orc_fingerprint_u64.argtypes = [P, U64, P, P]
    L.orc_fingerprint_bytes.argtypes = [P, P, U64, P, P]
    L.orc_phi.argtypes = [U64, U32, U64, U32]
    L.orc_phi.restype = U32
    L.orc_ln_success.argtypes = [U32, U32]
    L.orc_ln_success.restype = F64
    L.orc_tables.argtypes = [U32, U32, P, P, P]
    L.orc_strategy.argtypes = [U32, P, P]
    L.orc_split_parts.argtypes = [U32, U32, P]
    L.orc_split_parts.restype = U32
    L.orc_tree.argtypes = [P, U32, U32, U64, P, P, P, P]
    L.orc_build.argtypes = [U32, P, P, U64, U32, U32, U64, P, U64, P]
    L.orc_build_ex.argtypes = [U32, P, P, U64, U32, U32, U64, U32, U32, P, U64, P]
    L.orc_tables_slack.argtypes = [U32, U32, U32, U32, P, P, P, P]
    L.orc_tree_slack.argtypes = [P, U32, U32, U32, U64, P, P, P, P]
    L.orc_tables_ex.argtypes = [U32, U32, U32, P, P, P]
    L.orc_packed_table.argtypes = [U32, U32, U32, P]
    L.orc_lambda.argtypes = [U64]
    L.orc_lambda.restype = U32
    L.orc_gr_param_approx.argtypes = [U32, U32]
    L.orc_gr_param_approx.restype = U32
    L.orc_lookup.argtypes = [P, U64, U32, P, P, U64, P]
    L.orc_bucket_sizes.argtypes = [U32, P, P, U64, U64, P]
    L.orc_bucket_keys.argtypes = [U32, P, P, U64, U64, U64, P, U64]
    L.orc_bucket_keys.restype = U64
    L.orc_bucket_members.argtypes = [U32, P, P, U64, U64, U64, P, U64]
    L.orc_bucket_members.restype = U64
    L.orc_blob_bucket.argtypes = [P, U64, U64, P, P, P, P, U64, P]
    L.orc_bucket_ranks.argtypes = [P, U32, U32, U64, P]
    L.orc_blob_prefix.argtypes = [P, U64, P, P]
    L.orc_blob_check_inventory.argtypes = [P, U64, P]
    L.orc_inventory_build.argtypes = [P, U64, P, P, U32]
    L.orc_inventory_build.restype = None
    L.orc_inventory_select.argtypes = [P, P, P, U32, U64]
    L.orc_inventory_select.restype = U64
    L.orc_trees.argtypes = [P, P, U64, U64, U32, U64, P, P, P, P]
    L.orc_build_with_trees.argtypes = [U32, P, P, U64, U32, U32, P, P, P, P, U64, P]
    L.orc_bucket_layout.argtypes = [U32, P, P, U64, U64, P, P]
    L.orc_ranks_from_tree.argtypes = [P, U32, U32, P, P]
    L.orc_bucket_ids.argtypes = [P, U64, U64, P]
    L.orc_bucket_ids.restype = None
    for f in ("orc_tables", "orc_tree", "orc_build", "orc_lookup", "orc_bucket_sizes", "orc_blob_bucket",
              "orc_bucket_ranks", "orc_blob_prefix", "orc_blob_check_inventory", "orc_trees",
              "orc_build_with_trees", "orc_bucket_layout", "orc_ranks_from_tree", "orc_build_ex",
              "orc_tables_ex", "orc_packed_table", "orc_tables_slack", "orc_tree_slack"):
        getattr(L, f).restype = ctypes.c_int


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _keys(keys):
    """-> (kind, data array, offsets array or None, n)"""
    if isinstance(keys, tuple):
        data, offsets = keys
        data = np.ascontiguousarray(data, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        if data.size == 0:
            data = np.zeros(1, dtype=np.uint8)
        return KEYS_BYTES, data, offsets, len(offsets) - 1
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    return KEYS_U64, keys, None, len(keys)


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    lib().orc_splitmix64_stream(seed, count, _ptr(out))
    return out


def fingerprint(keys):
    kind, data, offs, n = _keys(keys)
    hi = np.zeros(n, dtype=np.uint64)
    lo = np.zeros(n, dtype=np.uint64)
    if kind == KEYS_U64:
        lib().orc_fingerprint_u64(_ptr(data), n, _ptr(hi), _ptr(lo))
    else:
        lib().orc_fingerprint_bytes(_ptr(data), _ptr(offs), n, _ptr(hi), _ptr(lo))
    return hi, lo


def phi(x: int, depth: int, v: int, m: int) -> int:
    return int(lib().orc_phi(x, depth, v, m))


def range_tables(leaf: int, maxm: int, leaf_slack: int, gr_table_max: int = 0):
    """Tables of the non-minimal variant: (r, F, N, Q), Q[m] the output range
    of a subtree of m keys."""
    r = np.zeros(maxm + 1, dtype=np.uint32)
    F = np.zeros(maxm + 1, dtype=np.uint32)
    N = np.zeros(maxm + 1, dtype=np.uint32)
    Q = np.zeros(maxm + 1, dtype=np.uint64)
    rc = lib().orc_tables_slack(leaf, maxm, gr_table_max, leaf_slack, _ptr(r), _ptr(F), _ptr(N), _ptr(Q))
    if rc:
        raise OracleError(rc, "tables_slack")
    return r, F, N, Q


def packed_table(leaf: int, maxm: int, gr_table_max: int = 0):
    """One 32-bit word per size (r | N << 5 | F << 16), or None when some
    size does not fit."""
    out = np.zeros(maxm + 1, dtype=np.uint32)
    rc = lib().orc_packed_table(leaf, maxm, gr_table_max, _ptr(out))
    if rc == EINVAL:
        return None
    if rc:
        raise OracleError(rc, "packed_table")
    return out


def lam(x: int) -> int:
    """lambda(x) = floor(lg x), the index of the highest set bit (Sec. 2)."""
    return int(lib().orc_lambda(x))


def gr_param_approx(leaf: int, m: int) -> int:
    """The Sec. 7.2 integer approximation of a split node's Golomb-Rice
    parameter (0 for leaves)."""
    return int(lib().orc_gr_param_approx(leaf, m))


def ln_success(leaf: int, m: int) -> float:
    return float(lib().orc_ln_success(leaf, m))


def strategy(leaf: int):
    lo, up = U32(), U32()
    lib().orc_strategy(leaf, ctypes.byref(lo), ctypes.byref(up))
    return lo.value, up.value


def split_parts(leaf: int, m: int) -> list:
    parts = np.zeros(16, dtype=np.uint32)
    f = lib().orc_split_parts(leaf, m, _ptr(parts))
    return [int(x) for x in parts[:f]]


def tables(leaf: int, maxm: int, gr_table_max: int = 0):
    """Per-size tables r, F, N for sizes 0..maxm; splits of more than
    gr_table_max keys (if nonzero) take the Sec. 7.2 approximation."""
    r = np.zeros(maxm + 1, dtype=np.uint32)
    F = np.zeros(maxm + 1, dtype=np.uint32)
    N = np.zeros(maxm + 1, dtype=np.uint32)
    rc = lib().orc_tables_ex(leaf, maxm, gr_table_max, _ptr(r), _ptr(F), _ptr(N))
    if rc:
        raise OracleError(rc, "tables")
    return r, F, N


def tree(lo: np.ndarray, leaf: int, seed_cap: int = 0, leaf_slack: int = 0):
    """Splitting tree of one bucket: (v, m, depth) arrays in preorder."""
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    m = len(lo)
    cap = max(m, 1)
    v = np.zeros(cap, dtype=np.uint64)
    mm = np.zeros(cap, dtype=np.uint32)
    d = np.zeros(cap, dtype=np.uint32)
    cnt = U64()
    rc = lib().orc_tree_slack(_ptr(lo if m else np.zeros(1, np.uint64)), m, leaf, leaf_slack, seed_cap, _ptr(v),
                              _ptr(mm), _ptr(d), ctypes.byref(cnt))
    if rc:
        raise OracleError(rc, "tree")
    c = cnt.value
    return v[:c].copy(), mm[:c].copy(), d[:c].copy()


def build(keys, leaf: int, bucket: int, seed_cap: int = 0, gr_table_max: int = 0, leaf_slack: int = 0) -> bytes:
    """The serialized structure (gr_table_max: splits of more than that many
    keys take the integer Golomb-Rice approximation of Sec. 7.2; 0 = none;
    leaf_slack > 0: the non-minimal variant, leaves of m keys map into
    m + ceil(m leaf_slack / 256) values)."""
    kind, data, offs, n = _keys(keys)
    size = U64()
    op = _ptr(offs) if offs is not None else None
    args = (kind, _ptr(data), op, n, leaf, bucket, seed_cap, gr_table_max, leaf_slack)
    rc = lib().orc_build_ex(*args, None, 0, ctypes.byref(size))
    if rc:
        raise OracleError(rc, "build")
    out = np.zeros(size.value, dtype=np.uint8)
    rc = lib().orc_build_ex(*args, _ptr(out), size.value, ctypes.byref(size))
    if rc:
        raise OracleError(rc, "build")
    return out.tobytes()


def bucket_layout(keys, nb: int):
    """(sorted, s): the lower signature words in bucket order (each bucket
    ascending) and the nb+1 prefix sums of the bucket sizes."""
    kind, data, offs, n = _keys(keys)
    srt = np.zeros(max(n, 1), dtype=np.uint64)
    s_ = np.zeros(nb + 1, dtype=np.uint64)
    rc = lib().orc_bucket_layout(kind, _ptr(data), _ptr(offs) if offs is not None else None, n, nb, _ptr(srt),
                                 _ptr(s_))
    if rc:
        raise OracleError(rc, "bucket_layout")
    return srt[:n], s_


def trees(sorted_lo: np.ndarray, s_: np.ndarray, first: int, last: int, leaf: int, seed_cap: int = 0):
    """Trees of buckets [first, last) of a bucket layout: (node_v, node_m,
    node_count), node arrays of the layout's length (bucket i's coded nodes
    from slot s_i on; other slots untouched) and counts for all buckets."""
    sorted_lo = np.ascontiguousarray(sorted_lo, dtype=np.uint64)
    s_ = np.ascontiguousarray(s_, dtype=np.uint64)
    n = max(len(sorted_lo), 1)
    v = np.zeros(n, dtype=np.uint64)
    m = np.zeros(n, dtype=np.uint32)
    d = np.zeros(n, dtype=np.uint32)
    cnt = np.zeros(max(len(s_) - 1, 1), dtype=np.uint64)
    src = sorted_lo if len(sorted_lo) else np.zeros(1, np.uint64)
    rc = lib().orc_trees(_ptr(src), _ptr(s_), first, last, leaf, seed_cap, _ptr(v), _ptr(m), _ptr(d), _ptr(cnt))
    if rc:
        raise OracleError(rc, "trees")
    return v, m, cnt


def build_with_trees(keys, leaf: int, bucket: int, node_v, node_m, node_count) -> bytes:
    """The serialized structure from trees computed elsewhere (same bytes as
    build() when the trees are the oracle's)."""
    kind, data, offs, n = _keys(keys)
    node_v = np.ascontiguousarray(node_v, dtype=np.uint64)
    node_m = np.ascontiguousarray(node_m, dtype=np.uint32)
    node_count = np.ascontiguousarray(node_count, dtype=np.uint64)
    size = U64()
    op = _ptr(offs) if offs is not None else None
    args = (kind, _ptr(data), op, n, leaf, bucket, _ptr(node_v), _ptr(node_m), _ptr(node_count))
    rc = lib().orc_build_with_trees(*args, None, 0, ctypes.byref(size))
    if rc:
        raise OracleError(rc, "build_with_trees")
    out = np.zeros(size.value, dtype=np.uint8)
    rc = lib().orc_build_with_trees(*args, _ptr(out), size.value, ctypes.byref(size))
    if rc:
        raise OracleError(rc, "build_with_trees")
    return out.tobytes()


def lookup(blob: bytes, keys) -> np.ndarray:
    kind, data, offs, q = _keys(keys)
    b = np.frombuffer(blob, dtype=np.uint8).copy()
    ranks = np.zeros(max(q, 1), dtype=np.uint64)
    rc = lib().orc_lookup(_ptr(b), len(blob), kind, _ptr(data), _ptr(offs) if offs is not None else None, q,
                          _ptr(ranks))
    if rc:
        raise OracleError(rc, "lookup")
    return ranks[:q]


def bucket_sizes(keys, nb: int) -> np.ndarray:
    kind, data, offs, n = _keys(keys)
    out = np.zeros(nb, dtype=np.uint64)
    rc = lib().orc_bucket_sizes(kind, _ptr(data), _ptr(offs) if offs is not None else None, n, nb, _ptr(out))
    if rc:
        raise OracleError(rc, "bucket_sizes")
    return out


def bucket_keys(keys, nb: int, bucket: int, cap: int = 1 << 16) -> np.ndarray:
    """Sorted lower signature words of one bucket."""
    kind, data, offs, n = _keys(keys)
    out = np.zeros(cap, dtype=np.uint64)
    cnt = lib().orc_bucket_keys(kind, _ptr(data), _ptr(offs) if offs is not None else None, n, nb, bucket,
                                _ptr(out), cap)
    if cnt > cap:
        return bucket_keys(keys, nb, bucket, int(cnt))
    return out[:cnt].copy()


def bucket_members(keys, nb: int, bucket: int, cap: int = 1 << 16) -> np.ndarray:
    """Positions in the input of the keys that fall in one bucket, ascending."""
    kind, data, offs, n = _keys(keys)
    out = np.zeros(cap, dtype=np.uint64)
    cnt = lib().orc_bucket_members(kind, _ptr(data), _ptr(offs) if offs is not None else None, n, nb, bucket,
                                   _ptr(out), cap)
    if cnt > cap:
        return bucket_members(keys, nb, bucket, int(cnt))
    return out[:cnt].copy()


def bucket_ranks(lo: np.ndarray, leaf: int, seed_cap: int = 0) -> np.ndarray:
    """Rank inside the bucket (0..m-1) of each lower signature word, from the
    tree the oracle builds for the bucket."""
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    out = np.zeros(max(len(lo), 1), dtype=np.uint64)
    rc = lib().orc_bucket_ranks(_ptr(lo if len(lo) else np.zeros(1, np.uint64)), len(lo), leaf, seed_cap, _ptr(out))
    if rc:
        raise OracleError(rc, "bucket_ranks")
    return out[:len(lo)]


def ranks_from_tree(lo: np.ndarray, leaf: int, v: np.ndarray) -> np.ndarray:
    """In-bucket ranks of the lower words lo given the bucket tree's indices
    v in preorder (no search)."""
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    v = np.ascontiguousarray(v, dtype=np.uint64)
    out = np.zeros(max(len(lo), 1), dtype=np.uint64)
    rc = lib().orc_ranks_from_tree(_ptr(lo if len(lo) else np.zeros(1, np.uint64)), len(lo), leaf,
                                   _ptr(v if len(v) else np.zeros(1, np.uint64)), _ptr(out))
    if rc:
        raise OracleError(rc, "ranks_from_tree")
    return out[:len(lo)]


def bucket_ids(hi: np.ndarray, nb: int) -> np.ndarray:
    """Bucket of every upper signature word."""
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    out = np.zeros(max(len(hi), 1), dtype=np.uint64)
    lib().orc_bucket_ids(_ptr(hi if len(hi) else np.zeros(1, np.uint64)), len(hi), nb, _ptr(out))
    return out[:len(hi)]


def blob_bucket(blob: bytes, bucket: int):
    """Decode one bucket of a serialized structure: (s_i, o_i, indices, sizes),
    the coded nodes in preorder."""
    b = np.frombuffer(blob, dtype=np.uint8).copy()
    h = header(blob)
    cap = max(int(h["maxm"]), 1)
    v = np.zeros(cap, dtype=np.uint64)
    m = np.zeros(cap, dtype=np.uint32)
    s_i, o_i, cnt = U64(), U64(), U64()
    rc = lib().orc_blob_bucket(_ptr(b), len(blob), bucket, ctypes.byref(s_i), ctypes.byref(o_i), _ptr(v), _ptr(m),
                               cap, ctypes.byref(cnt))
    if rc:
        raise OracleError(rc, "blob_bucket")
    c = cnt.value
    return s_i.value, o_i.value, v[:c].copy(), m[:c].copy()


def blob_prefix(blob: bytes):
    """Both Elias-Fano lists of a serialized structure: (s, o), nb+1 entries
    each (first rank and first tree bit of every bucket)."""
    b = np.frombuffer(blob, dtype=np.uint8).copy()
    nb = header(blob)["nb"]
    s_ = np.zeros(nb + 1, dtype=np.uint64)
    o_ = np.zeros(nb + 1, dtype=np.uint64)
    rc = lib().orc_blob_prefix(_ptr(b), len(blob), _ptr(s_), _ptr(o_))
    if rc:
        raise OracleError(rc, "blob_prefix")
    return s_, o_


def blob_check_inventory(blob: bytes) -> int:
    """Number of ones of the two upper-bit arrays that the inventory search
    places differently from a plain scan (0 for a correct structure)."""
    b = np.frombuffer(blob, dtype=np.uint8).copy()
    bad = U64()
    rc = lib().orc_blob_check_inventory(_ptr(b), len(blob), ctypes.byref(bad))
    if rc:
        raise OracleError(rc, "blob_check_inventory")
    return bad.value


def ones_from_positions(pos: np.ndarray) -> np.ndarray:
    """A little-endian bit array (uint64 words) with ones at the given positions."""
    pos = np.asarray(pos, dtype=np.uint64)
    words = np.zeros(int(pos.max()) // 64 + 2, dtype=np.uint64)
    np.bitwise_or.at(words, (pos // np.uint64(64)).astype(np.int64), np.left_shift(np.uint64(1), pos % np.uint64(64)))
    return words


def inventory_build(bits: np.ndarray, ones: int):
    """Two-level inventory of a bit array: (64-bit anchors, 16-bit offsets)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    hi = np.zeros((ones >> 14) + 1, dtype=np.uint64)
    lo = np.zeros((ones >> 8) + 1, dtype=np.uint16)
    lib().orc_inventory_build(_ptr(bits), ones, _ptr(hi), _ptr(lo), 1)
    return hi[: (ones + (1 << 14) - 1) >> 14], lo[: (ones + 255) >> 8]


def inventory_select(bits: np.ndarray, hi: np.ndarray, lo: np.ndarray, k: int) -> int:
    return int(lib().orc_inventory_select(_ptr(np.ascontiguousarray(bits, dtype=np.uint64)),
                                          _ptr(np.ascontiguousarray(hi, dtype=np.uint64)),
                                          _ptr(np.ascontiguousarray(lo, dtype=np.uint16)), 1, k))


def header(blob: bytes) -> dict:
    w = np.frombuffer(blob[:128], dtype=np.uint64)
    return {
        "magic": int(w[0]), "version": int(w[1]) & 0xFFFFFFFF, "kind": int(w[1]) >> 32, "n": int(w[2]),
        "leaf": int(w[3]), "bucket": int(w[4]), "nb": int(w[5]), "maxm": int(w[6]), "Ws": int(w[7]) & 0xFF,
        "Wz": (int(w[7]) >> 8) & 0xFF, "gr_table_max": (int(w[7]) >> 16) & 0xFFFFFF,
        "leaf_slack": (int(w[7]) >> 40) & 0xFF, "delta_s": int(w[8]), "delta_z": int(np.int64(w[9])), "beta": int(w[10]),
        "us_words": int(w[11]), "uz_words": int(w[12]), "lower_words": int(w[13]), "tree_words": int(w[14]),
        "tree_bits": int(w[15]),
    }
