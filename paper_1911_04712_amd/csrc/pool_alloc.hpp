// pool_alloc.hpp -- first-fit allocator of a request server's device pool.
//
// Plain host C++ (no HIP): the server carves each admitted request's
// workspace out of one caller-owned device pool with it, and the host tests
// drive it directly.  Blocks are 256-byte aligned; freed neighbours merge.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace dpd {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing free blocks.
class PoolAlloc {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto& f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t blocks() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;   // offset -> length of each free block
};

}  // namespace dpd
