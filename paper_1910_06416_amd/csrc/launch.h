// Launch geometry of librecsplit (host only, no HIP types, so that it can be
// checked by a plain C++ program on a machine without a GPU).
//
// A dispatch holds its grid size in work-items as a 32-bit value, and HIP
// limits the blocks of a one-dimensional grid to 2^31 - 1.  Every launch of
// the library checks its grid against both limits, and launches over more
// items than one grid holds (the seed search over buckets, the Golomb-Rice
// writer, lookups) are split into chunks that each fit.
#pragma once

#include <cstdint>

namespace rs {

constexpr uint64_t kMaxGridItems = 0xffffffffull;   // work-items of one launch
constexpr uint64_t kMaxGridBlocks = 0x7fffffffull;  // blocks of a one-dimensional grid

// True if `blocks` blocks of `threads` work-items form a valid grid.
inline bool grid_fits(uint64_t blocks, uint64_t threads) {
    return blocks >= 1 && threads >= 1 && threads <= 1024 && blocks <= kMaxGridBlocks &&
           blocks <= kMaxGridItems / threads;
}

// Most blocks of `threads` work-items that one launch may hold.
inline uint64_t max_grid_blocks(uint64_t threads) {
    const uint64_t by_items = kMaxGridItems / threads;
    return by_items < kMaxGridBlocks ? by_items : kMaxGridBlocks;
}

// Units (buckets, queries) one launch covers when each block of `threads`
// work-items takes `per_block` of them.
inline uint64_t chunk_units(uint64_t threads, uint64_t per_block) { return max_grid_blocks(threads) * per_block; }

// Calls f(first, count, blocks) for consecutive chunks that cover units
// [0, units), each launched as `blocks` blocks of `threads` work-items taking
// `per_block` units each; stops at the first nonzero return of f.
template <class F>
int for_each_chunk(uint64_t units, uint64_t threads, uint64_t per_block, F&& f) {
    const uint64_t per = chunk_units(threads, per_block);
    for (uint64_t first = 0; first < units; first += per) {
        const uint64_t count = units - first < per ? units - first : per;
        if (int rc = f(first, count, (count + per_block - 1) / per_block)) return rc;
    }
    return 0;
}

}  // namespace rs
