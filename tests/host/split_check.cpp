// Host build of spin_split (csrc/internal.h), the key permutation the
// LoopOverTerms prefilter works on, exercised by tests/test_split_host.py.
#include "internal.h"

#include <cstdint>

extern "C" void spin_split_host(const uint64_t* x, int64_t n, uint64_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = eloc::spin_split(x[i]);
}
