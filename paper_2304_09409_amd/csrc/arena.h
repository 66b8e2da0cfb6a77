// arena.h -- first-fit carving of one device allocation (host bookkeeping only; no HIP calls).
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace dpk {

// The HBM of a server under a budget: one device allocation of the budget less the model, made
// when the server is created, from which the slots' workspaces are carved (first fit over 256-B
// granules, free neighbours merged). Only the scheduler thread carves and releases, so a slot's
// workspace changes size without a device allocation or free (hipFree waits for the whole device,
// every slot's work included).
struct Arena {
    char* base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> holes;   // offset -> length: disjoint, never adjacent
    void reset(char* b, int64_t n) {
        base = b;
        size = n;
        holes.clear();
        if (n > 0) holes[0] = n;
    }
    bool owns(const void* p) const { return base && (const char*)p >= base && (const char*)p < base + size; }
    // offset of a carved range of at least `bytes`, or -1 if no hole holds it
    int64_t carve(int64_t bytes) {
        bytes = (bytes + 255) & ~(int64_t)255;
        for (auto it = holes.begin(); it != holes.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, rest = it->second - bytes;
            holes.erase(it);
            if (rest > 0) holes[off + bytes] = rest;
            return off;
        }
        return -1;
    }
    void give_back(int64_t off, int64_t bytes) {
        bytes = (bytes + 255) & ~(int64_t)255;
        auto next = holes.lower_bound(off);
        if (next != holes.end() && off + bytes == next->first) {
            bytes += next->second;
            next = holes.erase(next);
        }
        if (next != holes.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        holes[off] = bytes;
    }
};

}  // namespace dpk
