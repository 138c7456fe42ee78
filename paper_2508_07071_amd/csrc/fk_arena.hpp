// fk_arena.hpp -- first-fit allocator of byte ranges with coalescing, used
// by the server to place requests in its device arena.  Plain C++ (no HIP),
// so the host-side tests can build it with g++.
#pragma once
#include <stdint.h>

#include <iterator>
#include <map>

namespace fk {

// First-fit allocator over [0, size) with coalescing free blocks.
class Arena {
public:
    explicit Arena(int64_t size) { free_[0] = size; }
    int64_t alloc(int64_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0)
                    free_[off + bytes] = rest;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

    int64_t free_bytes() const
    {
        int64_t t = 0;
        for (const auto &kv : free_)
            t += kv.second;
        return t;
    }
    size_t free_blocks() const { return free_.size(); }

private:
    std::map<int64_t, int64_t> free_;  // offset -> size of each free block
};

}  // namespace fk
