// Shared declarations of the HIP engine: device data layouts, the
// membership tables and the kernel launchers used by api.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace eloc {

constexpr int kMaxWords = 2;     // N <= 128 qubits
constexpr int kSigRows = 65;     // popcount of even / odd qubit positions: 0..64
constexpr int kSigWords = 2 * kSigRows;

// ---------------------------------------------------------------------------
// Hamiltonian layout.  The unique XY set (first-appearance order) is an array
// of GroupRec; each group owns the run [begin, end) of TermRec (the paper's
// starts / nums arrays, as a CSR).  Inside a run the terms with an even
// |Y| = |XY & YZ| come first ([begin, mid), real matrix-element part), then
// those with odd |Y| ([mid, end), imaginary part), each in caller order.
// The stored coefficient already carries the sign of i^|Y|:
// h' = h (-1)^floor(|Y|/2), so <x|P|x'> h = h' (-1)^|x' & YZ| (times i for
// the odd part).
// ---------------------------------------------------------------------------
template <int W>
struct GroupRec {
    uint64_t xy[W];
    int32_t begin;
    int32_t mid;
    int32_t end;
    int32_t pad;
};

// Narrow keys (at most 32 qubits) also need every group's real and imaginary
// parts shorter than this: the hit queue carries their lengths in 16 bits.
constexpr int64_t kNarrowMaxPart = 65536;

template <int W>
struct TermRec {
    uint64_t yz[W];
    double h;
};

// FP32 form: signed coefficient split into hi + lo floats.
template <int W>
struct TermRecF {
    uint64_t yz[W];
    float h_hi;
    float h_lo;
};

// ---------------------------------------------------------------------------
// Membership tables.  Keys are looked up through a GF(2)-linear 64-bit hash
// lin(x) = XOR of R[q] over the set bits q of x, so lin(x ^ y) =
// lin(x) ^ lin(y): the hash of a candidate x ^ XY is one XOR of two
// precomputed hashes.  The table is a two-choice cuckoo table (load factor
// <= 1/4): a key sits in one of its two slots, so a lookup is exactly two
// independent loads.  With hs the salted hash and c = log2(capacity), slot 1
// is the low c bits of hs and slot 2 is slot 1 XOR ((hs >> c) | 1).
//
// Three formats, by key width:
//  * narrow (N <= 32): hs = low 32 bits of lin(x) ^ salt.  The low halves
//    of R[0..31] are linearly independent, so this is a bijection of 32-bit
//    keys; a 32-bit slot stores (hs >> c) << (ibits + 1) | which << ibits |
//    (index + 1).  Its position and contents give back all of hs, so equal
//    contents mean equal keys: a lookup is exact with no further load
//    (which = 1 marks a key sitting in its slot 2).
//  * wide (33 <= N <= 64): the same with the full 64-bit hash (R[0..63]
//    independent) and 64-bit slots.
//  * two words (N > 64): hs = lin(x) ^ salt; 32-bit slots hold
//    (fingerprint << ibits) | (index + 1), fingerprint = bits of hs above
//    bit 32 + ibits (never 0), and a match is confirmed by comparing the
//    stored key.
//
// Slots are 0 when empty.  A key whose insertion does not settle goes to a
// small stash (A. Kirsch, M. Mitzenmacher, U. Wieder, "More robust hashing:
// cuckoo hashing with a stash", 2009), scanned only when it is non-empty.
// ---------------------------------------------------------------------------
constexpr int kStash = 32;

enum TableKind : int { kTabNarrow = 0, kTabWide = 1, kTabVerify = 2 };

constexpr int table_kind(int W, bool narrow) { return W == 2 ? kTabVerify : (narrow ? kTabNarrow : kTabWide); }

template <int TK>
struct TabT {
    using slot = uint32_t;
    using hash = uint64_t;
};
template <>
struct TabT<kTabNarrow> {
    using slot = uint32_t;
    using hash = uint32_t;
};
template <>
struct TabT<kTabWide> {
    using slot = uint64_t;
    using hash = uint64_t;
};

inline size_t slot_bytes(int TK) { return TK == kTabWide ? sizeof(uint64_t) : sizeof(uint32_t); }

struct Stash {
    uint32_t count;
    uint32_t pad;
    uint32_t idx[kStash];     // key index
    uint64_t hs[kStash];      // salted hash of that key (narrow: low 32 bits)
};

struct Table {
    const void* slots;  // TabT<kind>::slot [capacity]
    uint32_t mask;      // capacity - 1
    int ibits;          // bits of index + 1
    uint32_t imask;     // (1 << ibits) - 1
    int fpshift;        // two-word keys: fingerprint = hs >> fpshift
    int capbits;        // log2(capacity)
    uint32_t pmask;     // partition bits of a slot index ((2^bits - 1) << shift, or 0: not partitioned)
    uint64_t salt;
    const Stash* stash;
};

// A table of at least 2^(shift + bits) slots is split into 2^bits
// partitions (bits = 3..5) by bits shift .. shift + bits - 1 of the slot
// index; both slots of a key lie in the partition of the key's salted hash.
// The hash is GF(2)-linear, so the partition of a candidate x ^ XY is part(x)
// ^ part(XY) ^ part(salt): a kernel can give each XCD the candidates of its
// partitions, one after another, whose slots then stay in that XCD's L2.
// Large tables use shift 16 (partitions made of blocks of 64K slots, so that
// every L2 channel and memory channel serves every partition: with low shift
// bits a partition would fall on a few channels only); shift 5 (runs of 32
// slots) lets small tables exercise the same path.
constexpr int kPartShiftLarge = 16;
constexpr int kPartShiftSmall = 5;
constexpr int kXcds = 8;
constexpr int kMaxPartBits = 5;
constexpr int kMaxParts = 1 << kMaxPartBits;
__host__ __device__ __forceinline__ int hash_part(uint64_t h, int shift, int bits) {
    return static_cast<int>((h >> shift) & ((1u << bits) - 1u));
}
__host__ __device__ __forceinline__ uint64_t part_min_slots(int shift, int bits) { return uint64_t(1) << (shift + bits); }
// Group buckets are ordered by the bit-reversed kMaxPartBits-bit partition
// field, so that for any bits the groups of one partition value p form one
// range: the buckets [r << (kMaxPartBits - bits), (r + 1) << (kMaxPartBits -
// bits)) with r = p reversed in bits bits.
__host__ __device__ __forceinline__ int rev_bits(int v, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

// Spin-split form of a key word: its even bits (spin-up orbitals under the
// interleaved Jordan-Wigner order) in order in the low half, its odd bits in
// the high half (an outer perfect unshuffle by five delta swaps).  A bit
// permutation commutes with XOR and keeps popcounts, so the LoopOverTerms
// prefilter can count both spin sectors of x ^ XY with one popcount per half
// word instead of a mask and two popcounts.
__host__ __device__ __forceinline__ uint64_t spin_split(uint64_t x) {
    uint64_t t;
    t = (x ^ (x >> 1)) & 0x2222222222222222ull;
    x ^= t ^ (t << 1);
    t = (x ^ (x >> 2)) & 0x0C0C0C0C0C0C0C0Cull;
    x ^= t ^ (t << 2);
    t = (x ^ (x >> 4)) & 0x00F000F000F000F0ull;
    x ^= t ^ (t << 4);
    t = (x ^ (x >> 8)) & 0x0000FF000000FF00ull;
    x ^= t ^ (t << 8);
    t = (x ^ (x >> 16)) & 0x00000000FFFF0000ull;
    x ^= t ^ (t << 16);
    return x;
}

template <int TK>
__host__ __device__ __forceinline__ typename TabT<TK>::hash salted(const Table& T, uint64_t h) {
    return static_cast<typename TabT<TK>::hash>(h ^ T.salt);
}
template <class HT>
__host__ __device__ __forceinline__ uint32_t slot1(const Table& T, HT hs) {
    return static_cast<uint32_t>(hs) & T.mask;
}
// The second slot keeps the first slot's partition bits; the other bits mix
// in the hash bits above the slot index (always odd, so the slots differ).
// Position and stored tag still determine the hash exactly.
template <class HT>
__host__ __device__ __forceinline__ uint32_t slot2(const Table& T, HT hs) {
    const uint32_t s = (static_cast<uint32_t>(hs) ^ (static_cast<uint32_t>(hs >> T.capbits) | 1u)) & T.mask;
    return (s & ~T.pmask) | (static_cast<uint32_t>(hs) & T.pmask);
}
// two-word keys; never 0, so an empty slot cannot match
__host__ __device__ __forceinline__ uint32_t fingerprint(const Table& T, uint64_t hs) {
    return static_cast<uint32_t>(hs >> T.fpshift) | 1u;
}

template <int W>
__device__ __forceinline__ bool keys_equal(const uint64_t* a, const uint64_t* b) {
    bool eq = a[0] == b[0];
    if (W == 2) eq = eq && (a[1] == b[1]);
    return eq;
}

template <int TK>
__device__ __forceinline__ typename TabT<TK>::slot load_slot(const Table& T, uint32_t s) {
    return static_cast<const typename TabT<TK>::slot*>(T.slots)[s];
}

// Slot loads through a bounds-checked raw buffer resource: an offset past the
// end of the slot array (kNoSlot) returns 0 without touching memory, so a
// filtered-out candidate needs no branch around its loads.  Dword 3 of the
// resource is the raw 32-bit format word of the gfx9 family.
constexpr uint32_t kNoSlot = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;

template <int TK>
struct SlotReader {
    using ST = typename TabT<TK>::slot;
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ explicit SlotReader(const Table& T)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(T.slots), static_cast<short>(0),
                                               static_cast<int>((T.mask + 1u) * sizeof(ST)), kRawBufferWord3)) {}
    __device__ __forceinline__ ST load(uint32_t slot, bool ok) const {
        const uint32_t off = ok ? slot * static_cast<uint32_t>(sizeof(ST)) : kNoSlot;
        if constexpr (sizeof(ST) == 4) {
            return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        } else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
            return (static_cast<uint64_t>(v[1]) << 32) | v[0];
        }
    }
};

// Whether a lookup must read the key's second slot, given its first: an
// insertion always claims the key's first slot before anything else, and a
// slot is never emptied again, so an empty first slot proves the key absent
// from both slots, and a first slot that holds the key settles the lookup.
// (Two-word keys: a fingerprint match at the first slot counts as settling;
// table_settle reads the second slot itself if the key compare then fails.)
template <int TK>
__device__ __forceinline__ bool need_slot2(const Table& T, typename TabT<TK>::slot v1, typename TabT<TK>::hash hs) {
    using ST = typename TabT<TK>::slot;
    if constexpr (TK != kTabVerify)
        return v1 != 0 && (v1 >> T.ibits) != static_cast<ST>((hs >> T.capbits) << 1);
    else
        return v1 != 0u && (v1 >> T.ibits) != fingerprint(T, hs);
}

// Second half of a lookup of a key with salted hash hs, given its two slot
// values (the second may be left 0 where need_slot2 is false); `nstash` is the stash count (wave-uniform).  Index of the key in
// `keys` (two-word format only), or -1.  A candidate that was filtered out
// (ok false: its slots read as empty) must not match the stash either, since
// the padded lanes past a chunk's end repeat a real candidate.
template <int TK, int W>
__device__ __forceinline__ int table_settle(const Table& T, const uint64_t* __restrict__ keys,
                                            typename TabT<TK>::slot v1, typename TabT<TK>::slot v2,
                                            typename TabT<TK>::hash hs, const uint64_t* key, int nstash,
                                            bool ok = true) {
    using ST = typename TabT<TK>::slot;
    int j = -1;
    if constexpr (TK != kTabVerify) {
        const ST t = static_cast<ST>((hs >> T.capbits) << 1);
        if ((v1 >> T.ibits) == t) j = static_cast<int>(v1 & T.imask) - 1;
        if ((v2 >> T.ibits) == (t | 1u)) j = static_cast<int>(v2 & T.imask) - 1;
        for (int k = 0; k < nstash && k < kStash; ++k)
            if (ok && T.stash->hs[k] == static_cast<uint64_t>(hs)) j = static_cast<int>(T.stash->idx[k]);
    } else {
        const uint32_t fp = fingerprint(T, hs);
        if ((v1 >> T.ibits) == fp) {
            const int j1 = static_cast<int>(v1 & T.imask) - 1;
            if (keys_equal<W>(keys + static_cast<size_t>(j1) * W, key)) j = j1;
        }
        if (j < 0 && (v1 >> T.ibits) == fp) v2 = load_slot<TK>(T, slot2(T, hs));   // rare: fingerprint clash
        if (j < 0 && (v2 >> T.ibits) == fp) {
            const int j2 = static_cast<int>(v2 & T.imask) - 1;
            if (keys_equal<W>(keys + static_cast<size_t>(j2) * W, key)) j = j2;
        }
        for (int k = 0; k < nstash && k < kStash; ++k) {
            if (ok && j < 0 && T.stash->hs[k] == hs) {
                const int js = static_cast<int>(T.stash->idx[k]);
                if (keys_equal<W>(keys + static_cast<size_t>(js) * W, key)) j = js;
            }
        }
    }
    return j;
}

// Full lookup of a key with (unsalted) hash h.
template <int TK, int W>
__device__ __forceinline__ int table_find(const Table& T, const uint64_t* __restrict__ keys, uint64_t h,
                                          const uint64_t* key) {
    const auto hs = salted<TK>(T, h);
    return table_settle<TK, W>(T, keys, load_slot<TK>(T, slot1(T, hs)), load_slot<TK>(T, slot2(T, hs)), hs, key,
                               static_cast<int>(T.stash->count));
}

// Cuckoo insertion of key i (hash hash[i]): place it in one of its two
// slots, evicting the occupant to its other slot; after kMaxKicks moves the
// key in hand goes to the stash, or the error bit is set if that is full.
constexpr int kMaxKicks = 256;

template <int TK>
__device__ __forceinline__ void table_insert_one(const uint64_t* __restrict__ hash, int64_t i, void* slots_v,
                                                 Stash* __restrict__ stash, const Table& T,
                                                 uint32_t* __restrict__ err, uint32_t err_bit) {
    const auto hs = salted<TK>(T, hash[i]);
    int64_t held = i;   // index of the key in hand
    if constexpr (TK != kTabVerify) {
        using ST = std::conditional_t<TK == kTabWide, unsigned long long, uint32_t>;
        auto* slots = static_cast<ST*>(slots_v);
        ST v = static_cast<ST>(((static_cast<ST>(hs) >> T.capbits) << (T.ibits + 1)) | static_cast<ST>(i + 1));
        uint32_t s = slot1(T, hs);
        for (int k = 0; k < kMaxKicks; ++k) {
            const ST old = atomicExch(slots + s, v);
            if (old == 0) return;
            // the evicted key moves to its other slot (the same XOR in both
            // directions; the partition bits are kept, as slot2 keeps them)
            s ^= (static_cast<uint32_t>(old >> (T.ibits + 1)) | 1u) & T.mask & ~T.pmask;
            v = old ^ (static_cast<ST>(1) << T.ibits);
        }
        held = static_cast<int64_t>(v & T.imask) - 1;
    } else {
        auto* slots = static_cast<uint32_t*>(slots_v);
        uint32_t v = (fingerprint(T, hs) << T.ibits) | static_cast<uint32_t>(i + 1);
        uint32_t s = slot1(T, hs);
        for (int k = 0; k < kMaxKicks; ++k) {
            const uint32_t old = atomicExch(slots + s, v);
            if (old == 0u) return;
            v = old;
            const uint64_t ho = hash[(old & T.imask) - 1u] ^ T.salt;
            const uint32_t a = slot1(T, ho);
            s = (s == a) ? slot2(T, ho) : a;
        }
        held = static_cast<int64_t>(v & T.imask) - 1;
    }
    const uint32_t k = atomicAdd(&stash->count, 1u);
    if (k < static_cast<uint32_t>(kStash)) {
        stash->idx[k] = static_cast<uint32_t>(held);
        stash->hs[k] = static_cast<uint64_t>(salted<TK>(T, hash[held]));
    } else {
        atomicOr(err, err_bit);
    }
}

// Blocked Bloom filter of U (LoopOverTerms): a key with linear hash h sets
// two bits of one 32-bit word, all chosen from hf = the high half of h, so
// the test of a candidate x ^ XY needs hf(x) ^ hf(XY) and one word.
constexpr uint32_t kBloomMaxWords = 8192;   // 32 KB of LDS

__host__ __device__ __forceinline__ uint32_t bloom_word(uint32_t hf, uint32_t fmask) { return (hf >> 10) & fmask; }
__host__ __device__ __forceinline__ uint32_t bloom_bits(uint32_t hf) {
    return (1u << (hf & 31u)) | (1u << ((hf >> 5) & 31u));
}

// ---------------------------------------------------------------------------
// Device state handed to kernels.
// ---------------------------------------------------------------------------
struct TNode;

// Prefix trees (sorted keys + radix-tree nodes).  XY trees are built per
// chunk of `chunk` consecutive sorted masks: chunk c owns leaves
// [c * chunk, min(G, (c + 1) * chunk)) and nodes from c * (chunk - 1).
struct XYTrieDev {
    const uint64_t* keys = nullptr;   // [G][W] sorted
    const int32_t* gid = nullptr;     // group id of each sorted mask
    const TNode* nodes = nullptr;
    const uint64_t* nkeys = nullptr;  // representative key of each node
    int chunk = 0;
    int chunks = 0;
};

struct UTrieDev {
    const uint64_t* keys = nullptr;   // [M][W] sorted
    const int32_t* perm = nullptr;    // sample index of each sorted key
    const TNode* nodes = nullptr;     // [M - 1]
    const uint64_t* nkeys = nullptr;  // [M - 1][W] representative key of each node
};

struct HamDev {
    int n_qubits = 0;
    int W = 0;
    bool narrow = false;       // n_qubits <= 32: narrow table format, 32-bit bit work
    int64_t n_terms = 0;
    int64_t n_groups = 0;
    int maxpop = 0;            // max popcount of an XY mask
    int diag_group = -1;       // group whose XY is 0, or -1
    const void* groups = nullptr;     // GroupRec<W>[G]
    const void* terms = nullptr;      // TermRec<W>[T]
    const void* terms_f = nullptr;    // TermRecF<W>[T]
    const int32_t* term_src = nullptr;     // caller index of every stored term [T]
    const uint8_t* term_ny = nullptr;      // its |Y| mod 4 [T]
    const uint64_t* group_hash = nullptr;  // lin(XY_g) [G]
    const uint64_t* group_keys = nullptr;  // XY_g [G][W] (table key array)
    const uint64_t* group_split = nullptr; // spin_split(XY_g) [G][W]
    Table group_table{};               // XY -> group id
    XYTrieDev xyt{};
    // the group records again, bucketed by the reversed kMaxPartBits-bit
    // partition field of their hash (stable), for LoopOverTerms over a
    // partitioned U table
    struct {
        const void* groups = nullptr;
        const uint64_t* ghash = nullptr;
        const uint64_t* gsplit = nullptr;
        const int32_t* gid = nullptr;          // group id of every record in bucket order
        int bucket[kMaxParts + 1] = {};        // bucket starts (host copy)
        const int32_t* bucket_dev = nullptr;   // the same [kMaxParts + 1] on the device
        int shift = kPartShiftLarge;   // first partition bit of U's tables for this Hamiltonian
    } part;
};

// Prefilter parameters of U for LoopOverTerms, derived on the device by
// eloc_set_samples and read by the pair kernels at their start (so that
// preparing U needs no host round trip): U's single (even-qubit, total)
// popcount signature, or sig_all = 1 when U has several; U's per-qubit
// majority key and its largest distance from it, or rad_max = 128 (off)
// when that radius is not under half the qubits.
struct SampleParams {
    int32_t sig_pa;
    int32_t sig_n;
    int32_t sig_all;
    int32_t rad_max;
    uint64_t rad_ref[kMaxWords];
};

struct SampleDev {
    int64_t n = 0;
    int64_t rows = 0;                       // rows the pair kernels evaluate: samples
                                            // 0 .. rows - 1 (0: all n); the conventional
                                            // local energy evaluates U's rows over U and
                                            // its coupled states
    const SampleParams* params = nullptr;   // device
    const uint32_t* prep_err = nullptr;     // device error word of the preparation: the
                                            // pair kernels do nothing while it is non-zero
    const uint64_t* keys = nullptr;    // [M][W] caller order
    const uint64_t* hash = nullptr;    // lin(x_i) [M]
    Table table{};
    const uint64_t* sig = nullptr;     // [kSigWords] signature bitmap
    UTrieDev ut{};                     // valid once built for this batch
    // rows ordered by hash_part of their (unsalted) hash, for the partitioned
    // LoopOverTerms: built with U's table when the table is partitioned
    struct {
        int bits = 0;                         // 2^bits partitions (0: not partitioned)
        const int32_t* row_perm = nullptr;
        const int64_t* class_off = nullptr;   // [2^bits + 1] (device)
        const int64_t* tile_off = nullptr;    // [2^bits + 1] (device), tiles of kRows rows
    } part;
};

// Amplitudes relative to the largest |psi|: a_i = exp(L_i - c), c = max Re L.
struct AmpDev {
    const double2* a = nullptr;        // FP64 form
    const float4* af = nullptr;        // FP32 form: (re_hi, re_lo, im_hi, im_lo)
    const double* shift = nullptr;     // device scalar c
};

// Launch geometry of the pair kernels.
struct Plan {
    int chunks = 1;            // group (or sample) chunks per row
    int per_chunk = 0;         // groups (or samples) per chunk
    bool sig_filter = true;    // exact LoopOverTerms prefilters on: U's single (even, total)
                               // popcount signature and / or its radius
    int sig_pa = 0;            // that signature: popcount on even qubits
    int sig_n = 0;             //                 total popcount
    bool sig_all = false;      // no single signature: the signature test passes everything
    uint64_t rad_ref[kMaxWords] = {0, 0};   // radius filter: reference key and
    int rad_max = 128;                      // max distance of U from it (128: off)
    int rows_per_block = 1;    // rows owned by one wave (TERMS, BATCH) or workgroup (TRIE)
    int waves_per_block = 1;   // waves of a TERMS / BATCH workgroup
    const uint32_t* bloom = nullptr;   // U's Bloom filter (LoopOverTerms), staged in LDS
    uint32_t bloom_words = 0;          // its size in words, a power of two (0: not used)
    bool part = false;                 // LoopOverTerms by U's table partitions (2^bits, kXcds at a time)
    int part_sub = 1;                  // chunks of a group bucket (chunks = 2^bits part_sub)
};

// Error bits latched in a device word, read by eloc_check / synchronising calls.
enum ErrBits : uint32_t {
    kErrDup = 1u,
    kErrBits = 2u,
    kErrWeights = 4u,
    kErrRange = 8u,
    kErrIndex = 16u,
    kErrTable = 32u,   // cuckoo insertion did not settle; rebuild with another salt
    kErrCapacity = 64u,   // a caller buffer of an asynchronous call was too small
};

// ---------------------------------------------------------------------------
// Batched launch: many (Hamiltonian, U) problems in one pipeline.  Samples of
// all problems share one global index space (problem k owns [s0, s0 + M));
// a per-problem descriptor holds the offsets into the concatenated buffers
// and the caller's own input / output pointers.  The pair kernel runs over
// work items (problem, row tile, chunk) in the order of the schedule: one
// workgroup per item, or a grid of a few per compute unit striding over them.
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 256;   // problems per batch (four lane registers of item starts)
constexpr int kBTile = 2048;     // samples per reduction tile

struct BatchProb {
    // Hamiltonian (run and group indices local to the problem)
    const void* groups;
    const uint64_t* ghash;
    const uint64_t* gsplit;   // spin_split of the XY masks [G][W]
    const void* terms;
    const void* terms_f;
    const uint64_t* gkeys;
    Table gtable;
    int32_t n_groups;
    int32_t maxpop;
    int32_t n_qubits;
    int32_t variant;       // 0 LoopOverTerms, 1 LoopOverBatch
    // samples
    int64_t s0;
    int64_t M;
    Table ktable;          // index values local to the problem
    void* kslots;          // writable views of ktable's arrays
    Stash* kstash;
    // schedule
    int32_t chunks;
    int32_t per_chunk;
    int64_t item0;         // first work item of the problem
    int64_t items;
    int64_t pbase;         // first partial of the problem; partial (c, row) at pbase + c * M + row
    int32_t rt0;           // reduction tiles [rt0, rt0 + rtn)
    int32_t rtn;
    // caller buffers (device)
    const uint64_t* keys_in;   // [M][w_in]
    int32_t w_in;
    int32_t narrow;            // one-word narrow tables and hit queue (at most 32 qubits, short runs)
    const double2* logpsi;
    const double* weights;     // null: |psi|^2 weights
    double2* eloc;
    double* stats;             // [4]
};

struct RTile {
    int32_t prob;
    int32_t pad;
    int64_t begin;   // global sample range
    int64_t end;
};

struct BatchDev {
    const BatchProb* probs;
    int n;
    int W;
    const int32_t* pid;        // [S] problem of every global sample
    int64_t S;
    const RTile* tiles;
    int n_tiles;
    const int32_t* sched;      // problems in schedule order (item0 ascending)
    int64_t total_items;
    const uint64_t* R;         // linear hash words [64 W]
    uint64_t* keys;            // [S][W] copy of the caller keys (zero-padded words)
    uint64_t* khash;           // [S]
    uint32_t* slots;           // all key-table slots (cleared per run)
    int64_t n_slot_words;      // their size in 32-bit words
    Stash* stash;              // [n]
    uint32_t* err;             // [n] error bits
    uint32_t* sigmin;          // [n] min / max of (even popcount << 8 | popcount) over U_k
    uint32_t* sigmax;
    uint32_t* bitcounts;       // [n][128] per-qubit counts of set bits over U_k
    unsigned long long* rad;   // [n][3] majority key of U_k (2 words), max distance from it
    double* shift;             // [n] max Re L
    double* scal;              // [n][3] E re, E im, sum w
    double* part;              // [n_tiles][3] reduction partials
    unsigned long long* pairs; // [n] coupled pairs found
    int64_t narrow_items;      // items [0, narrow_items) belong to narrow problems
    double2* a;
    double2* b;
    float4* af;
    float4* bf;
    void* partial;
};

// ---------------------------------------------------------------------------
// Launchers (kernels.hip).  All enqueue on `st` and return hipError_t.
// ---------------------------------------------------------------------------
hipError_t launch_sample_hash(int W, const uint64_t* keys, int64_t n, const uint64_t* R,
                              int n_qubits, uint64_t* hash, uint32_t* counts, uint32_t* err, hipStream_t st);
// rad[0..W-1] = per-qubit majority key of U (from the counts), rad[2] = max
// distance of U's keys from it (rad[2] must start at 0).
hipError_t launch_sample_radius(int W, const uint64_t* keys, int64_t n, const uint32_t* counts,
                                unsigned long long* rad, hipStream_t st);
hipError_t launch_bloom_build(const uint64_t* hash, int64_t n, uint32_t* filt, uint32_t words, hipStream_t st);
hipError_t launch_table_insert(int table_kind, const uint64_t* hash, int64_t n, void* slots, Stash* stash,
                               const Table& T, uint32_t* err, hipStream_t st);
hipError_t launch_sample_verify(int W, bool narrow, const SampleDev& S, uint64_t* sig, uint32_t* err,
                                hipStream_t st);
// SampleParams from the signature bitmap and the radius words (one thread).
hipError_t launch_sample_params(const uint64_t* sig, const unsigned long long* rad, int n_qubits,
                                SampleParams* out, hipStream_t st);
hipError_t launch_amp_prep(const double2* logpsi, int64_t n, bool fp32, double2* a, double2* b,
                           float4* af, float4* bf, double* shift, double* scratch, uint32_t* err,
                           hipStream_t st);
hipError_t launch_adj_vec(const double2* a, const double2* b, const double* weights, int64_t n,
                          bool fp32, double2* v, float4* vf, hipStream_t st);
hipError_t launch_pairs(bool adjoint, int variant, int precision, const HamDev& H,
                        const SampleDev& S, const Plan& P, const double2* vec, const float4* vecf,
                        void* partial, hipStream_t st);
hipError_t launch_finish(int precision, int64_t n, const Plan& P, const void* partial,
                         const double2* b, const float4* bf, double2* out, hipStream_t st);
hipError_t launch_adj_finish(int precision, int64_t n, const Plan& P, const void* partial,
                             const double2* a, const float4* af, const double2* eloc,
                             const double* weights, const double* stats, double* scratch,
                             double2 ge, double2* out, hipStream_t st);
hipError_t launch_energy(const double2* eloc, const double2* logpsi, const double* weights,
                         const double* shift, int64_t n, double* stats, double* scratch,
                         uint32_t* err, hipStream_t st);
hipError_t launch_pairs_count(int variant, const HamDev& H, const SampleDev& S, const Plan& P,
                              int32_t* counts, hipStream_t st);
hipError_t launch_pairs_fill(int variant, const HamDev& H, const SampleDev& S, const Plan& P,
                             int jbits, const int64_t* offsets, uint64_t* pkey, uint32_t* pval,
                             hipStream_t st);
hipError_t launch_scan_i32(const int32_t* in, int64_t n, int64_t* out, int64_t* scratch,
                           hipStream_t st);
hipError_t launch_radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                                   uint32_t* vals_alt, int64_t n, int end_bit, uint32_t* hist,
                                   int64_t* hist_off, int64_t* scan_scratch, int* result_in_alt,
                                   hipStream_t st);
hipError_t launch_split_pairs(const uint64_t* keys, const uint32_t* vals, int64_t n, int jbits,
                              int32_t* i_out, int32_t* j_out, int32_t* g_out, hipStream_t st);
// h_out[t] = H_{x_i x_j} for the pair t = (i_idx[t], j_idx[t]); with cnt /
// grp (both or neither) also the term count of the pair's group (0 if the
// pair is not coupled) and the group id (-1).
hipError_t launch_pair_elements(const HamDev& H, const SampleDev& S, int64_t n,
                                const int32_t* i_idx, const int32_t* j_idx, double2* h_out,
                                int32_t* cnt, int32_t* grp, uint32_t* err, hipStream_t st);
// Phase exponents k = (|Y_l| + 2 |x_j & YZ_l|) mod 4 of every term l of the
// pair's group, ascending l, at k_out[offsets[t] ..]; nothing is written
// and kErrCapacity is latched if offsets[n] > capacity.
hipError_t launch_pair_phases(const HamDev& H, const SampleDev& S, int64_t n, const int32_t* j_idx,
                              const int32_t* grp, const int64_t* offsets, uint8_t* k_out, int64_t capacity,
                              uint32_t* err, hipStream_t st);

hipError_t launch_pairs_to_csr(const HamDev& H, const SampleDev& S, int64_t n, const uint64_t* pkey,
                               const uint32_t* pval, int jbits, int32_t* col, double2* h, hipStream_t st);
hipError_t launch_rowptr(const int64_t* offsets, int64_t M, int chunks, int64_t* rowptr, hipStream_t st);
hipError_t launch_spmv(bool adjoint, int precision, int64_t M, const int64_t* rowptr, const int32_t* col,
                       const double2* h, const void* vec, void* partial, hipStream_t st);

struct SortScratch {
    uint64_t* key;
    uint32_t* val;
    uint64_t* key2;
    uint32_t* val2;
    uint32_t* hist;
    int64_t* hist_off;
    int64_t* scan;
};
hipError_t launch_sort_keys(int W, int n_bits, const uint64_t* keys, int64_t n, const SortScratch& S,
                            uint64_t* sorted, int32_t* perm, hipStream_t st);
hipError_t launch_trie_build(int W, const uint64_t* keys, int64_t n_total, int64_t per, TNode* nodes,
                             uint64_t* nkeys, hipStream_t st);
int rows_per_block(int variant, int requested);
constexpr int kPartRows = 8;   // rows of a tile of the partitioned LoopOverTerms
// Rows ordered by the partition class of their hash (stable), the first
// position and the first tile (kPartRows rows, classes padded to whole tiles)
// of every class: perm[n], class_off[2^bits + 1], tile_off[2^bits + 1];
// scratch as for the sort.
hipError_t launch_row_classes(const uint64_t* hash, int64_t n, int shift, int bits, uint64_t* key, uint32_t* val,
                              uint64_t* key2,
                              uint32_t* val2, uint32_t* hist, int64_t* hist_off, int64_t* scan, int32_t* perm,
                              int64_t* class_off, int64_t* tile_off, hipStream_t st);
// Node pairs (U node, XY node) the LoopOverTrie walk visits over all rows
// and XY chunks, added to *visits.
hipError_t launch_trie_visits(const HamDev& H, const SampleDev& S, const Plan& P, unsigned long long* visits,
                              hipStream_t st);

// Batched pipeline (batch.hip; the batched pair kernel in pairs.hip).
hipError_t launch_batch_prepare(const BatchDev& B, bool fp32, hipStream_t st);
hipError_t launch_batch_pairs(const BatchDev& B, int precision, int rows, int narrow_blocks, int wide_blocks,
                              hipStream_t st);
hipError_t launch_batch_finish(const BatchDev& B, int precision, hipStream_t st);
int batch_blocks_per_cu(int W, bool narrow, int precision, int rows);


// The conventional local energy's extra states: the x' = x ^ XY_g outside U
// with |H_xx'| > tol sum |h|, appended (in no particular order, duplicates
// included) as [n][W] keys to out at positions taken from *counter (which
// must start at 0 and ends at their number); those at positions >= capacity
// are counted but not written.
hipError_t launch_misses(const HamDev& H, const SampleDev& S, int chunks, int per_chunk, double tol,
                         unsigned long long* counter, int64_t capacity, uint64_t* out, hipStream_t st);
// One-word keys of at most kMissBitmapQubits qubits: the same states marked
// instead in a bitmap over the whole key space (bit x' of word x' >> 5; the
// bitmap must start cleared), which makes them unique and sorted at once.
constexpr int kMissBitmapQubits = 30;
hipError_t launch_misses_bitmap(const HamDev& H, const SampleDev& S, int chunks, int per_chunk, double tol,
                                uint32_t* bitmap, hipStream_t st);
// counts[w] = popcount(bitmap[w]); keys of the set bits in ascending order
// to out at the exclusive prefix sums pos of those counts
hipError_t launch_bitmap_counts(const uint32_t* bitmap, int64_t nwords, int32_t* counts, hipStream_t st);
hipError_t launch_bitmap_keys(const uint32_t* bitmap, int64_t nwords, const int64_t* pos, uint64_t* out,
                              hipStream_t st);
// flags[i] = 1 where sorted key i starts a run of equal keys
hipError_t launch_unique_flags(int W, const uint64_t* sorted, int64_t n, int32_t* flags, hipStream_t st);
// out[pos[i]] = sorted[i] where flags[i]
hipError_t launch_unique_scatter(int W, const uint64_t* sorted, int64_t n, const int32_t* flags, const int64_t* pos,
                                 uint64_t* out, hipStream_t st);

// Stochastic reconfiguration over the highest-probability samples: the
// indices of the nsr largest Re log psi (descending, ties to the lower
// index; sorts all n with the key scratch), and the shifted solve.
hipError_t launch_sr_select(const double2* logpsi, int64_t n, int nsr, uint64_t* key, uint32_t* val, uint64_t* key2,
                            uint32_t* val2, uint32_t* hist, int64_t* hist_off, int64_t* scan, int32_t* out,
                            hipStream_t st);
// Scratch: w[2 nsr], mean[2 np], partial[sr_partial_len(np, R16, R)] (per-block
// Gram partials [sr_partial_blocks(np)][R16][R16], then the reduction passes)
// (R16 = 2 nsr + 1 rounded up to 16), T[R][R], L[(2 nsr)^2], y[2 nsr].
hipError_t launch_sr_solve(int nsr, int64_t np, const double* ore, const double* oim, const double2* logpsi,
                           const double* F, double lambda, double* w, double* mean, double* partial, double* T,
                           double* L, double* y, double* d, uint32_t* err, hipStream_t st);
int64_t sr_partial_blocks(int64_t np);
int64_t sr_partial_len(int64_t np, int R16, int R);   // doubles of `partial`

// Autoregressive sampling without replacement: the ansatz of per-qudit
// perceptrons (hidden width 64) and one level of the Gumbel top-K search.
struct ArModelDev {
    int n_qubits;
    int qudit;
    int n_up, n_down;
    const double* W1;   // [Q][64][N]
    const double* b1;   // [Q][64]
    const double* W2;   // [Q][64][64]
    const double* b2;   // [Q][64]
    const double* W3;   // [Q][2^qudit][64]
    const double* b3;   // [Q][2^qudit]
};
hipError_t launch_ar_root(uint64_t* keys, int W, double* l, double* T, hipStream_t st);
// Candidates of level `level` for the B prefixes (keys, l, T): cand_* [B O],
// O = 2^(qudit width); *n_allowed += the unmasked ones.
hipError_t launch_ar_level(const ArModelDev& M, int level, int64_t B, uint64_t seed, const uint64_t* keys,
                           const double* l, const double* T, double* cand_l, double* cand_T, uint64_t* cand_key,
                           uint32_t* cand_idx, unsigned long long* n_allowed, hipStream_t st);
hipError_t launch_ar_gather(const uint64_t* keys, const uint32_t* sorted_idx, int64_t n, int O, int W, int q0,
                            const double* cand_l, const double* cand_T, uint64_t* out_keys, double* out_l, double* out_T,
                            hipStream_t st);
// The candidates that can be among the first `need` (1 <= need <= n) in
// (key, index) order: every candidate whose 24-bit key prefix is at most the
// need-th's, in index order, into okey / oidx (their count in off[n]).
// Scratch: hist[4096] (digit totals), sel[4], keep[n], off[n + 1],
// scan as for launch_scan_i32.
int64_t ar_select_blocks(int64_t n);
hipError_t launch_ar_select(const uint64_t* key, int64_t n, int64_t need, uint32_t* hist, int64_t* sel,
                            int32_t* keep, int64_t* off, int64_t* scan, uint64_t* okey, uint32_t* oidx,
                            hipStream_t st);

// Fixed workspace of the allocation-free forward pass (one per device).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
// Device address of this device's workspace (`device` must be current on
// the first call for it); cached per device.
hipError_t noalloc_workspace(int device, void** out);
// p[0..n) = v (a kernel, so that code under stream capture records no memset)
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

int64_t energy_scratch_len();
int64_t amp_scratch_len();
int64_t scan_scratch_len(int64_t n);
int64_t radix_tiles(int64_t n);

}  // namespace eloc
