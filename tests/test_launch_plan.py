"""Launch geometry (csrc/launch.h), checked on the CPU with a plain C++ program.

A dispatch carries its grid size in work-items as a 32-bit value.  The seed
search launches one workgroup of 64 * waves lanes per bucket, so a call with
more than (2^32 - 1) / (64 * waves) buckets must be split into several
launches; so must the Golomb-Rice writer (16 lanes per bucket) and lookups
(one lane per query).  This test runs the library's own chunking code
(`for_each_chunk`) for the bucket counts of the largest workloads and checks
that every chunk fits one launch and that the chunks cover every bucket once.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_1910_06416_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "launch.h"
int main(int argc, char** argv) {
    const unsigned long long units = std::strtoull(argv[1], nullptr, 10);
    const unsigned long long threads = std::strtoull(argv[2], nullptr, 10);
    const unsigned long long per_block = std::strtoull(argv[3], nullptr, 10);
    return rs::for_each_chunk(units, threads, per_block, [&](uint64_t first, uint64_t count, uint64_t blocks) {
        std::printf("%llu %llu %llu %d\n", (unsigned long long)first, (unsigned long long)count,
                    (unsigned long long)blocks, rs::grid_fits(blocks, threads) ? 1 : 0);
        return 0;
    });
}
"""


@pytest.fixture(scope="module")
def plan_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("launch")
    src = d / "plan.cpp"
    src.write_text(DRIVER)
    exe = d / "plan"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", HEADER_DIR, "-o", str(exe), str(src)], check=True)
    return str(exe)


def _chunks(exe, units, threads, per_block):
    out = subprocess.run([exe, str(units), str(threads), str(per_block)], check=True, capture_output=True,
                         text=True).stdout
    return [tuple(int(x) for x in line.split()) for line in out.splitlines()]


# 1.11e8 buckets: 10^9 keys at l=12, b=9; 67,108,864 = 4096 bins x 16384 buckets;
# 2e7 buckets: 2e7 keys at b=1 (four waves: 5.1e9 work-items in one grid).
BUCKETS = [111_111_112, 67_108_864, 20_000_000, 16_777_215, 16_777_216, 1, 1000]


@pytest.mark.parametrize("nb", BUCKETS)
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_search_chunks_fit_and_cover(plan_exe, nb, waves):
    threads = 64 * waves
    chunks = _chunks(plan_exe, nb, threads, 1)
    assert all(fits == 1 for *_, fits in chunks)
    assert all(blocks * threads <= 2**32 - 1 and blocks <= 2**31 - 1 for _, _, blocks, _ in chunks)
    # consecutive, disjoint, and covering [0, nb)
    pos = 0
    for first, count, blocks, _ in chunks:
        assert first == pos and count == blocks and count >= 1
        pos += count
    assert pos == nb
    # as few launches as the limit allows
    per = (2**32 - 1) // threads
    assert len(chunks) == -(-nb // per)


def test_old_single_grid_overflowed_at_the_faulted_shape():
    """The one-grid search launch of 1.11e8 buckets of four wavefronts asked
    for 2.8e10 work-items, far beyond the 32-bit grid size."""
    assert 111_111_112 * 256 > 2**32
    assert 20_000_000 * 256 > 2**32


@pytest.mark.parametrize("nb", [111_111_112, 268_435_456, 300_000_000])
def test_tree_writer_chunks(plan_exe, nb):
    chunks = _chunks(plan_exe, nb, 256, 16)
    pos = 0
    for first, count, blocks, fits in chunks:
        assert fits == 1 and first == pos and blocks == -(-count // 16)
        pos += count
    assert pos == nb


@pytest.mark.parametrize("q", [10**7, 2**32 - 1, 2**32, 5 * 10**9])
def test_lookup_chunks(plan_exe, q):
    chunks = _chunks(plan_exe, q, 256, 256)
    pos = 0
    for first, count, blocks, fits in chunks:
        assert fits == 1 and first == pos and blocks == -(-count // 256)
        pos += count
    assert pos == q


def test_grid_limits(plan_exe):
    # a grid of exactly 2^32 work-items does not fit; one less block does
    assert _chunks(plan_exe, 2**26, 64, 1) == [(0, 2**26 - 1, 2**26 - 1, 1), (2**26 - 1, 1, 1, 1)]
