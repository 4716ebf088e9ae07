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

// part_bits = 0: not partitioned.
inline Table make_table(void* slots, Stash* stash, uint64_t capacity, int64_t n, uint64_t salt,
                        int part_shift = kPartShiftLarge, int part_bits = 0) {
    Table T;
    T.stash = stash;
    T.slots = slots;
    T.mask = static_cast<uint32_t>(capacity - 1);
    T.ibits = std::max(1, bits_for(static_cast<uint64_t>(n)));   // index + 1 <= n
    T.imask = (T.ibits >= 32) ? 0xFFFFFFFFu : ((1u << T.ibits) - 1u);
    T.fpshift = 32 + T.ibits;
    T.capbits = bits_for(capacity - 1);
    T.pmask = part_bits > 0 && capacity >= part_min_slots(part_shift, part_bits)
                  ? (((1u << part_bits) - 1u) << part_shift)
                  : 0u;
    T.salt = salt;
    return T;
}

// Slots of a membership table for n keys: a power of two, load <= 1/4.
inline uint64_t table_capacity(int64_t n) { return pow2_at_least(static_cast<uint64_t>(4 * std::max<int64_t>(n, 1))); }

// Adds v to a GF(2) basis (basis[b]: reduced vector with leading bit b);
// false if v depends on it.
template <class T, int B>
inline bool gf2_insert(T (&basis)[B], T v) {
    for (int b = B - 1; b >= 0 && v; --b) {
        if (!((v >> b) & 1u)) continue;
        if (!basis[b]) {
            basis[b] = v;
            return true;
        }
        v ^= basis[b];
    }
    return false;
}

// The 128 words R of the linear hash.  R[0..31] are drawn until their low
// 32 bits are linearly independent over GF(2), and R[0..63] until they are
// independent as 64-bit words: the low half of the hash is then a bijection
// of keys of up to 32 qubits and the whole hash a bijection of one-word
// keys, which makes those lookups exact without a key compare.
inline void make_hash_words(uint64_t R[128]) {
    uint64_t s = 0x2408076250ull;
    uint32_t b32[32] = {};
    uint64_t b64[64] = {};
    int q = 0;
    while (q < 32) {
        const uint64_t v = splitmix64(s);
        if (gf2_insert(b32, static_cast<uint32_t>(v))) {
            (void)gf2_insert(b64, v);   // independent: its low half already is
            R[q++] = v;
        }
    }
    while (q < 64) {
        const uint64_t v = splitmix64(s);
        if (gf2_insert(b64, v)) R[q++] = v;
    }
    for (; q < 128; ++q) R[q] = splitmix64(s);
}

}  // namespace eloc
