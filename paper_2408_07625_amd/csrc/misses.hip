// The conventional local energy's extra states (Eq. local_energy summed over
// every x', the estimator that the sample-aware form replaces): the x' =
// x ^ XY_g, x in U, that are not in U and whose matrix element is non-zero.
//
// k_misses walks the same (row, XY group) candidates as LoopOverTerms: a
// wave owns kMissRows rows (keys in scalar registers), its lanes sweep 64
// groups of the row's chunk per step.  A candidate is looked up in U's
// table; one that is absent has its matrix element evaluated over the
// group's run, and is a miss when |H| > tol * sum |h_l| (strings that cancel
// exactly, e.g. hopping strings between particle-number sectors, give no
// state).  The misses of a step (all rows) take one range of the output
// from an atomic counter and are written there (ballot + mbcnt), those past
// the capacity only counted; the caller reruns with a larger buffer when the
// count exceeds it.  The list is then sorted and made unique, so the order
// in which waves append does not show in the result.  For one-word keys of
// at most 30 qubits the misses instead set their bit in a bitmap over the
// key space (one atomic OR each); the set bits, read in order, are the
// unique states already sorted.
#include "device.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

namespace {

constexpr int kMissRows = 8;

struct MissArgs {
    const void* groups;      // GroupRec<W>[G]
    const uint64_t* ghash;   // lin(XY_g)
    const void* terms;       // TermRec<W>[T]
    int n_groups;
    int per_chunk;
    int chunks;
    const uint64_t* keys;
    const uint64_t* khash;
    Table ktable;
    int64_t M;
    const uint32_t* prep_err;
    double tol;
};

// |H_xx'| > tol * sum |h_l| over the group's run [b, e) (real part [b, m),
// imaginary part [m, e)), H evaluated with the ket x'.
template <int W>
__device__ __forceinline__ bool nonzero_element(const TermRec<W>* __restrict__ terms, const GroupRec<W>& gr,
                                                const uint64_t* ket, double tol) {
    double hr = 0.0, hi = 0.0, sa = 0.0;
    for (int t = gr.begin; t < gr.mid; ++t) {
        const TermRec<W> tr = terms[t];
        hr += term_f64<W>(tr, ket);
        sa += fabs(tr.h);
    }
    for (int t = gr.mid; t < gr.end; ++t) {
        const TermRec<W> tr = terms[t];
        hi += term_f64<W>(tr, ket);
        sa += fabs(tr.h);
    }
    return hypot(hr, hi) > tol * sa;
}

__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u)));
}

template <int W, int TK>
__global__ __launch_bounds__(64) void k_misses(MissArgs A, unsigned long long* __restrict__ counter, int64_t capacity,
                                               uint64_t* __restrict__ out, uint32_t* __restrict__ bitmap) {
    const int lane = lane_id();
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kMissRows;
    const int chunk = static_cast<int>(blockIdx.y);
    if (row0 >= A.M) return;
    const int nr = static_cast<int>(min(static_cast<int64_t>(kMissRows), A.M - row0));
    if (__builtin_amdgcn_readfirstlane(static_cast<int>(*A.prep_err)) != 0) return;   // U invalid: no states
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(A.groups);
    const TermRec<W>* __restrict__ terms = static_cast<const TermRec<W>*>(A.terms);
    uint64_t x[kMissRows][W];
    uint64_t hx[kMissRows];
#pragma unroll
    for (int r = 0; r < kMissRows; ++r) {
        const int64_t row = min(row0 + r, A.M - 1);
#pragma unroll
        for (int w = 0; w < W; ++w) x[r][w] = A.keys[row * W + w];
        hx[r] = A.khash[row];
    }
    const int nstash = __builtin_amdgcn_readfirstlane(static_cast<int>(A.ktable.stash->count));
    const int g0 = chunk * A.per_chunk;
    const int g1 = min(A.n_groups, g0 + A.per_chunk);
    for (int base = g0; base < g1; base += 64) {
        const int g = base + lane;
        const bool valid = g < g1;
        const GroupRec<W> gr = groups[min(g, g1 - 1)];
        const uint64_t gh = A.ghash[min(g, g1 - 1)];
        uint64_t m[kMissRows];
        bool miss[kMissRows];
        int total = 0;
#pragma unroll
        for (int r = 0; r < kMissRows; ++r) {
            uint64_t xp[W];
#pragma unroll
            for (int w = 0; w < W; ++w) xp[w] = x[r][w] ^ gr.xy[w];
            miss[r] = false;
            if (valid && r < nr) {
                const auto hs = salted<TK>(A.ktable, hx[r] ^ gh);
                const int j = table_settle<TK, W>(A.ktable, A.keys, load_slot<TK>(A.ktable, slot1(A.ktable, hs)),
                                                  load_slot<TK>(A.ktable, slot2(A.ktable, hs)), hs, xp, nstash);
                if (j < 0) miss[r] = nonzero_element<W>(terms, gr, xp, A.tol);
            }
            m[r] = __ballot(miss[r]);
            total += __popcll(m[r]);
        }
        if (total == 0) continue;   // wave-uniform
        if (W == 1 && bitmap) {   // uniform
#pragma unroll
            for (int r = 0; r < kMissRows; ++r) {
                if (miss[r]) {
                    const uint64_t key = x[r][0] ^ gr.xy[0];
                    atomicOr(bitmap + (key >> 5), 1u << static_cast<uint32_t>(key & 31u));
                }
            }
            continue;
        }
        unsigned long long first = 0ull;
        if (lane == 0) first = atomicAdd(counter, static_cast<unsigned long long>(total));
        const int64_t at0 = static_cast<int64_t>(
            (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(first >> 32))))
             << 32) |
            static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(first))));
        int64_t run = 0;
#pragma unroll
        for (int r = 0; r < kMissRows; ++r) {
            if (miss[r]) {
                const int64_t at = at0 + run + lanes_below(m[r]);
                if (at < capacity) {
#pragma unroll
                    for (int w = 0; w < W; ++w) out[at * W + w] = x[r][w] ^ gr.xy[w];
                }
            }
            run += __popcll(m[r]);
        }
    }
}

// flags[i] = 1 if sorted key i differs from key i - 1 (first of its run)
template <int W>
__global__ void k_first_of_run(const uint64_t* __restrict__ sorted, int64_t n, int32_t* __restrict__ flags) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool first = i == 0;
    if (!first) {
#pragma unroll
        for (int w = 0; w < W; ++w) first = first || sorted[i * W + w] != sorted[(i - 1) * W + w];
    }
    flags[i] = first ? 1 : 0;
}

template <int W>
__global__ void k_scatter_unique(const uint64_t* __restrict__ sorted, int64_t n, const int32_t* __restrict__ flags,
                                 const int64_t* __restrict__ pos, uint64_t* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const int64_t o = pos[i];
#pragma unroll
    for (int w = 0; w < W; ++w) out[o * W + w] = sorted[i * W + w];
}

inline unsigned blocks256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

__global__ void k_bitmap_counts(const uint32_t* __restrict__ bitmap, int64_t nwords, int32_t* __restrict__ counts) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nwords) counts[i] = __popc(bitmap[i]);
}

__global__ void k_bitmap_keys(const uint32_t* __restrict__ bitmap, int64_t nwords, const int64_t* __restrict__ pos,
                              uint64_t* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nwords) return;
    uint32_t b = bitmap[i];
    int64_t o = pos[i];
    while (b) {
        const int k = __builtin_ctz(b);
        out[o++] = (static_cast<uint64_t>(i) << 5) | static_cast<uint64_t>(k);
        b &= b - 1u;
    }
}

template <int W, int TK>
hipError_t launch_misses_t(const MissArgs& A, unsigned long long* counter, int64_t capacity, uint64_t* out,
                           uint32_t* bitmap, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((A.M + kMissRows - 1) / kMissRows), static_cast<unsigned>(A.chunks));
    hipLaunchKernelGGL((k_misses<W, TK>), grid, dim3(64), 0, st, A, counter, capacity, out, bitmap);
    return hipGetLastError();
}

MissArgs miss_args(const HamDev& H, const SampleDev& S, int chunks, int per_chunk, double tol) {
    MissArgs A;
    A.groups = H.groups;
    A.ghash = H.group_hash;
    A.terms = H.terms;
    A.n_groups = static_cast<int>(H.n_groups);
    A.per_chunk = per_chunk;
    A.chunks = chunks;
    A.keys = S.keys;
    A.khash = S.hash;
    A.ktable = S.table;
    A.M = S.n;
    A.prep_err = S.prep_err;
    A.tol = tol;
    return A;
}

}  // namespace

hipError_t launch_misses(const HamDev& H, const SampleDev& S, int chunks, int per_chunk, double tol,
                         unsigned long long* counter, int64_t capacity, uint64_t* out, hipStream_t st) {
    const MissArgs A = miss_args(H, S, chunks, per_chunk, tol);
    const int tk = table_kind(H.W, H.narrow);
    if (H.W == 2) return launch_misses_t<2, kTabVerify>(A, counter, capacity, out, nullptr, st);
    if (tk == kTabNarrow) return launch_misses_t<1, kTabNarrow>(A, counter, capacity, out, nullptr, st);
    return launch_misses_t<1, kTabWide>(A, counter, capacity, out, nullptr, st);
}

hipError_t launch_misses_bitmap(const HamDev& H, const SampleDev& S, int chunks, int per_chunk, double tol,
                                uint32_t* bitmap, hipStream_t st) {
    if (H.W != 1 || H.n_qubits > kMissBitmapQubits || !bitmap) return hipErrorInvalidValue;
    const MissArgs A = miss_args(H, S, chunks, per_chunk, tol);
    if (table_kind(H.W, H.narrow) == kTabNarrow)
        return launch_misses_t<1, kTabNarrow>(A, nullptr, 0, nullptr, bitmap, st);
    return launch_misses_t<1, kTabWide>(A, nullptr, 0, nullptr, bitmap, st);
}

hipError_t launch_bitmap_counts(const uint32_t* bitmap, int64_t nwords, int32_t* counts, hipStream_t st) {
    hipLaunchKernelGGL(k_bitmap_counts, dim3(blocks256(nwords)), dim3(256), 0, st, bitmap, nwords, counts);
    return hipGetLastError();
}

hipError_t launch_bitmap_keys(const uint32_t* bitmap, int64_t nwords, const int64_t* pos, uint64_t* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_bitmap_keys, dim3(blocks256(nwords)), dim3(256), 0, st, bitmap, nwords, pos, out);
    return hipGetLastError();
}

hipError_t launch_unique_flags(int W, const uint64_t* sorted, int64_t n, int32_t* flags, hipStream_t st) {
    if (W == 2)
        hipLaunchKernelGGL(k_first_of_run<2>, dim3(blocks256(n)), dim3(256), 0, st, sorted, n, flags);
    else
        hipLaunchKernelGGL(k_first_of_run<1>, dim3(blocks256(n)), dim3(256), 0, st, sorted, n, flags);
    return hipGetLastError();
}

hipError_t launch_unique_scatter(int W, const uint64_t* sorted, int64_t n, const int32_t* flags, const int64_t* pos,
                                 uint64_t* out, hipStream_t st) {
    if (W == 2)
        hipLaunchKernelGGL(k_scatter_unique<2>, dim3(blocks256(n)), dim3(256), 0, st, sorted, n, flags, pos, out);
    else
        hipLaunchKernelGGL(k_scatter_unique<1>, dim3(blocks256(n)), dim3(256), 0, st, sorted, n, flags, pos, out);
    return hipGetLastError();
}

}  // namespace eloc
