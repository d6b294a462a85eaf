// First-fit range allocator over the request arena of the serving engine
// (gf_engine.cpp): byte ranges [off, off + n) of [0, size), free ranges kept
// in offset order and merged with their neighbours on release.  Host code
// only; not public ABI.
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace gf {

class RangeAlloc {
  public:
    explicit RangeAlloc(size_t size) { free_[0] = size; }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
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
    size_t largest() const {
        size_t m = 0;
        for (auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace gf
