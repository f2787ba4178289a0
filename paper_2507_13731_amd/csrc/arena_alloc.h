// First-fit allocator of the server's HBM arena (host bookkeeping only: offsets into one device
// allocation).  Header-only so that a host-only test can exercise it under the address and
// undefined-behaviour sanitizers.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace qlra_impl {

// First-fit allocator over [0, cap) with 256-byte granules; adjacent free ranges merge.
class ArenaAlloc {
  public:
    explicit ArenaAlloc(size_t cap) { if (cap) free_[0] = cap; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
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
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

}  // namespace qlra_impl
