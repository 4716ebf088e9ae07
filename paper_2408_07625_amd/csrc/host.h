// Host helpers shared by the single-problem context and the batched launch:
// device buffers, the splitmix64 generator of hash words and salts, and the
// membership-table geometry.
#pragma once

#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace eloc {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

inline uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline int bits_for(uint64_t v) {   // smallest b with v < 2^b
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

inline uint64_t pow2_at_least(uint64_t v) {
    uint64_t c = 1;
    while (c < v) c <<= 1;
    return c;
}

inline Table make_table(uint32_t* slots, uint32_t* stash, uint64_t capacity, int64_t n, uint64_t salt) {
    Table T;
    T.stash = stash;
    T.slots = slots;
    T.mask = static_cast<uint32_t>(capacity - 1);
    T.ibits = std::max(1, bits_for(static_cast<uint64_t>(n)));   // index + 1 <= n
    T.imask = (T.ibits >= 32) ? 0xFFFFFFFFu : ((1u << T.ibits) - 1u);
    T.fpshift = 32 + T.ibits;
    T.altshift = bits_for(capacity - 1);
    T.salt = salt;
    return T;
}

}  // namespace eloc
