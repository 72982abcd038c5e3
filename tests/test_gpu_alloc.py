"""Every device allocation of the library goes through the installed
allocator (rs_set_allocator), and the results do not depend on it."""
import numpy as np
import pytest

from paper_1910_06416_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch

    assert torch.cuda.is_available()
    from paper_1910_06416_amd import recsplit

    recsplit.lib()
    return recsplit


class CountingAllocator:
    """A caller-side allocator over torch's caching allocator that records
    every pointer the library takes and gives back."""

    def __init__(self, rs):
        import torch

        self.live, self.allocs, self.frees, self.ctx_seen = {}, 0, 0, set()

        def alloc(nbytes, stream, ctx):
            p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            self.live[p] = int(nbytes)
            self.allocs += 1
            self.ctx_seen.add(ctx)
            return p

        def free(ptr, stream, ctx):
            assert ptr in self.live, "freed a pointer the allocator never gave out"
            del self.live[ptr]
            self.frees += 1
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = rs.ALLOC_FN(alloc)
        self.free_fn = rs.FREE_FN(free)


def test_every_allocation_goes_through_the_callers_allocator(rs, orc):
    import torch

    ca = CountingAllocator(rs)
    rs.set_allocator(ca.alloc_fn, ca.free_fn, 1234)
    try:
        keys = inputs.u64_keys(50_000, 91)
        print("case counting allocator: build", flush=True)
        blob = rs.build(rs.device_keys(keys), 8, 100)
        torch.cuda.synchronize()
        # workspace, tables and blob arena; the workspace is already back
        assert ca.allocs >= 3 and len(ca.live) == 2 and ca.ctx_seen == {1234}
        assert sum(ca.live.values()) >= blob.nbytes
        assert blob.to_bytes() == orc.build(keys, 8, 100)
        ranks = rs.lookup(blob, rs.device_keys(keys)).cpu().numpy().view(np.uint64)
        assert np.array_equal(np.sort(ranks), np.arange(len(keys), dtype=np.uint64))
        blob.free()
        assert not ca.live, "blob memory not returned through the allocator"
        print("case counting allocator: batch, plan, from_bytes", flush=True)
        sets = [inputs.u64_keys(n, 92 + n) for n in (3000, 20_000, 7)]
        blobs, status = rs.build_batch([rs.device_keys(k) for k in sets], [8, 12, 5], [100, 1000, 5])
        assert status == [0, 0, 0]
        for b, k, (l, bb) in zip(blobs, sets, [(8, 100), (12, 1000), (5, 5)]):
            assert b.to_bytes() == orc.build(k, l, bb)
        plan = rs.Plan([rs.device_keys(sets[0])], 8, 100)
        pb, _ = plan.run()
        assert pb[0].to_bytes() == orc.build(sets[0], 8, 100)
        fb = rs.from_bytes(orc.build(sets[1], 12, 1000))
        assert fb.to_bytes() == orc.build(sets[1], 12, 1000)
        for b in blobs + pb + plan.first + [fb]:
            b.free()
        plan.close()
        torch.cuda.synchronize()
        assert not ca.live, f"{len(ca.live)} allocations not returned"
        assert ca.frees == ca.allocs
    finally:
        rs.use_torch_allocator()


def test_torch_allocator_counts_library_memory(rs, orc):
    """With the binding's default (PyTorch's caching allocator) a live blob is
    part of torch.cuda.memory_allocated()."""
    import torch

    rs.use_torch_allocator()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    keys = inputs.u64_keys(200_000, 93)
    dk = rs.device_keys(keys)
    print("case torch allocator", flush=True)
    mid = torch.cuda.memory_allocated()
    blob = rs.build(dk, 8, 100)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - mid >= blob.nbytes
    assert blob.to_bytes() == orc.build(keys, 8, 100)
    blob.free()
    del dk
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_default_allocator_still_builds(rs, orc):
    keys = inputs.u64_keys(30_000, 94)
    rs.use_default_allocator()
    try:
        print("case default allocator", flush=True)
        assert rs.build(rs.device_keys(keys), 8, 100).to_bytes() == orc.build(keys, 8, 100)
    finally:
        rs.use_torch_allocator()
