// Device memory for librecsplit from PyTorch's caching allocator.
//
// The two functions match rs_alloc_fn / rs_free_fn of recsplit.h; the Python
// binding passes their addresses to rs_set_allocator, so the library's
// workspaces and blobs come from the same pool as the caller's tensors (and
// show in torch.cuda.memory_allocated()) without a Python call per
// allocation.  The caching allocator is stream-aware: a block returned by
// rs_torch_free is reused only by later work on the stream it was allocated
// for, which is the ordering the library's stream-ordered releases need.
#include <c10/hip/HIPCachingAllocator.h>

#include <cstddef>

extern "C" void* rs_torch_alloc(size_t bytes, void* stream, void* /*ctx*/) {
    try {
        return c10::hip::HIPCachingAllocator::raw_alloc_with_stream(bytes, static_cast<hipStream_t>(stream));
    } catch (...) {
        return nullptr;  // out of memory: the library reports RS_ENOMEM
    }
}

extern "C" void rs_torch_free(void* ptr, void* /*stream*/, void* /*ctx*/) {
    try {
        c10::hip::HIPCachingAllocator::raw_delete(ptr);
    } catch (...) {
    }
}
