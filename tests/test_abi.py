"""The C-ABI library loads on the CPU and exports every entry point its
header declares; the library's host tables equal the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "recsplit.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1910_06416_amd import recsplit

    return recsplit.lib()


def test_binding_constants_match_the_header():
    """Status codes, key kinds and option flags: the Python binding's values
    are the header's."""
    from paper_1910_06416_amd import recsplit

    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {k: int(v) for k, v in re.findall(r"\b(RS_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    for name in ("RS_OK", "RS_EINVAL", "RS_EDUPLICATE", "RS_ENOMEM", "RS_EDEVICE", "RS_ESEARCH", "RS_EFORMAT",
                 "RS_EBUSY", "RS_KEYS_U64", "RS_KEYS_BYTES", "RS_OPT_TIMING", "RS_OPT_TUNED", "RS_OPT_NO_SAMPLES"):
        assert values[name] == getattr(recsplit, name), name
    assert recsplit._options(samples=False).flags == values["RS_OPT_NO_SAMPLES"]
    assert recsplit._options().flags == 0


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rs_build", "rs_lookup", "rs_blob_bytes", "rs_blob_to_host", "rs_blob_from_host",
                     "rs_blob_free", "rs_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing


def test_version_string(lib):
    assert b"gfx950" in lib.rs_version()


@pytest.mark.parametrize("leaf", range(1, 25))
def test_library_tables_equal_oracle_tables(orc, leaf):
    from paper_1910_06416_amd import recsplit

    r, F, N = recsplit.tables(leaf, 4096)
    r2, F2, N2 = orc.tables(leaf, 4096)
    assert np.array_equal(r, r2) and np.array_equal(F, F2) and np.array_equal(N, N2)


def test_argument_validation_without_device(lib):
    from paper_1910_06416_amd import recsplit

    keys = recsplit.rs_keys(recsplit.RS_KEYS_U64, None, None, 0)
    out = ctypes.c_void_p()
    assert lib.rs_build(ctypes.byref(keys), 8, 100, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    keys.n = 10
    assert lib.rs_build(ctypes.byref(keys), 8, 100, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    keys.data = 16
    assert lib.rs_build(ctypes.byref(keys), 25, 100, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    assert lib.rs_build(ctypes.byref(keys), 8, 0, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    assert b"bucket" in lib.rs_last_error()
    bad = np.zeros(16, dtype=np.uint64)
    assert lib.rs_blob_from_host(bad.ctypes.data, 128, None, ctypes.byref(out)) == recsplit.RS_EFORMAT
    assert out.value is None


def test_server_argument_validation(lib):
    import ctypes

    from paper_1910_06416_amd import recsplit

    out = ctypes.c_void_p()
    assert lib.rs_server_create(0, 2, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    assert lib.rs_server_create_ex(None, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    cfg = recsplit.rs_server_config(0, 2, 0)
    assert lib.rs_server_create_ex(ctypes.byref(cfg), None, ctypes.byref(out)) == recsplit.RS_EINVAL


def test_schedule_table_roundtrip_and_validation(lib):
    from paper_1910_06416_amd import recsplit

    recsplit.clear_schedules()
    assert recsplit.get_schedule(8, 100) is None
    recsplit.set_schedule(8, 100, stage_from=7, group_max=3, waves=2)
    got = recsplit.get_schedule(8, 100)
    assert (got["stage_from"], got["group_max"], got["waves"]) == (7, 3, 2)
    assert recsplit.get_schedule(8, 101) is None
    for bad in [(7, 3, 3), (7, 0, 1), (7, 8, 1), (1, 3, 1), (26, 3, 1)]:
        with pytest.raises(recsplit.RecSplitError):
            recsplit.set_schedule(8, 100, *bad)
    with pytest.raises(recsplit.RecSplitError):
        recsplit.set_schedule(25, 100, 9, 7, 4)
    with pytest.raises(recsplit.RecSplitError):
        recsplit.set_schedule(8, 0, 9, 7, 4)
    recsplit.clear_schedules()
    assert recsplit.get_schedule(8, 100) is None


def test_autotune_argument_validation(lib):
    from paper_1910_06416_amd import recsplit

    assert lib.rs_autotune(0, 100, 0, 10.0, None, None) == recsplit.RS_EINVAL
    assert lib.rs_autotune(8, 0, 0, 10.0, None, None) == recsplit.RS_EINVAL


def test_too_many_buckets_is_refused_before_any_device_work(lib):
    """More than 4096 bins of 65536 buckets is refused on the host."""
    from paper_1910_06416_amd import recsplit

    keys = recsplit.rs_keys(recsplit.RS_KEYS_U64, 16, None, 4096 * 65536 + 1)
    out = ctypes.c_void_p()
    assert lib.rs_build(ctypes.byref(keys), 8, 1, None, ctypes.byref(out)) == recsplit.RS_EINVAL
    assert b"too many buckets" in lib.rs_last_error()
    assert out.value is None


def test_set_allocator_validation_without_device(lib):
    """rs_set_allocator takes both functions or neither; no device is needed."""
    from paper_1910_06416_amd import recsplit

    fake = ctypes.c_void_p(0x1000)
    assert lib.rs_set_allocator(fake, None, None) == recsplit.RS_EINVAL
    assert lib.rs_set_allocator(None, fake, None) == recsplit.RS_EINVAL
    assert b"neither" in lib.rs_last_error()
    assert lib.rs_set_allocator(None, None, None) == recsplit.RS_OK
    # the binding's default: PyTorch's caching allocator through the native shim
    recsplit.use_torch_allocator()
    assert lib.rs_set_allocator(None, None, None) == recsplit.RS_OK
    recsplit.use_torch_allocator()


@pytest.mark.parametrize("leaf,T", [(8, 96), (8, 500), (16, 560), (16, 1200), (5, 31), (1, 4), (24, 216), (12, 97)])
def test_library_tables_with_large_split_approximation_equal_oracle(orc, leaf, T):
    """Splits above T take the integer approximation of Sec. 7.2 on both sides
    (written independently); every table of sizes 0..4096 agrees."""
    from paper_1910_06416_amd import recsplit

    r, F, N = recsplit.tables(leaf, 4096, T)
    r2, F2, N2 = orc.tables(leaf, 4096, T)
    assert np.array_equal(r, r2) and np.array_equal(F, F2) and np.array_equal(N, N2)
    r0, _, _ = recsplit.tables(leaf, 4096)
    assert (r != r0).any()  # the approximation is in use above T


@pytest.mark.parametrize("leaf,T", [(4, 0), (8, 0), (16, 0), (24, 0), (3, 0), (8, 500), (2, 0), (1, 0)])
def test_library_packed_table_equals_oracle(orc, leaf, T):
    """The packed per-size words (footnote of Sec. 7.2), written independently
    on both sides, agree; both refuse where a size does not fit."""
    from paper_1910_06416_amd import recsplit

    got = recsplit.packed_table(leaf, 2600, T)
    want = orc.packed_table(leaf, 2600, T)
    if want is None:
        assert got is None
    else:
        assert got is not None and np.array_equal(got, want)


@pytest.mark.parametrize("leaf,slack,T", [(8, 32, 0), (8, 255, 0), (5, 64, 0), (16, 16, 0), (16, 128, 500),
                                          (24, 85, 0), (12, 1, 0), (2, 100, 0), (1, 255, 0)])
def test_library_range_tables_equal_oracle(orc, leaf, slack, T):
    """Non-minimal variant (Sec. 9): leaf parameters from the injection
    probability into the larger range and the subtree ranges Q, written
    independently on both sides, agree for sizes 0..4096."""
    from paper_1910_06416_amd import recsplit

    got = recsplit.range_tables(leaf, 4096, slack, T)
    want = orc.range_tables(leaf, 4096, slack, T)
    for g, w in zip(got, want):
        assert np.array_equal(g.astype(np.uint64), w.astype(np.uint64))
    Q = got[3].astype(np.int64)
    assert (np.diff(Q) > 0).all() and Q[0] == 0 and Q[1] == 1
    if leaf >= 2:
        assert Q[leaf] == leaf + -(-leaf * slack // 256)


def test_range_tables_refuse_leaves_over_32_values(lib):
    from paper_1910_06416_amd import recsplit

    with pytest.raises(recsplit.RecSplitError):
        recsplit.range_tables(24, 100, 86)  # 24 + ceil(24 * 86 / 256) = 33 values
    with pytest.raises(recsplit.RecSplitError):
        recsplit.range_tables(8, 100, 256)
    recsplit.range_tables(24, 100, 85)


def test_build_option_validation_without_device(lib):
    """Options the library refuses on the host, before any device work."""
    from paper_1910_06416_amd import recsplit

    keys = recsplit.rs_keys(recsplit.RS_KEYS_U64, 16, None, 10)
    out = ctypes.c_void_p()
    for opts in (recsplit._options(leaf_slack=256), recsplit._options(gr_table_max=1 << 24)):
        assert lib.rs_build_ex(ctypes.byref(keys), 8, 100, ctypes.byref(opts), None, ctypes.byref(out)) == \
            recsplit.RS_EINVAL
    opts = recsplit._options(leaf_slack=86)
    assert lib.rs_build_ex(ctypes.byref(keys), 24, 100, ctypes.byref(opts), None, ctypes.byref(out)) == \
        recsplit.RS_EINVAL
    assert b"32 values" in lib.rs_last_error()
