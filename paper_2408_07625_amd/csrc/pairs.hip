// Pair kernels for gfx950: FindCoupledPairs (three variants) fused with
// MatrixElement and the ratio accumulation, plus the pair count / emission
// kernels that share the same enumeration.
//
// LoopOverTerms (Alg. 2A) and LoopOverBatch (Alg. 2B): a workgroup is one
// wave that owns kRows sample rows.  The rows' keys and linear hashes are
// wave-uniform (scalar registers); the lanes sweep the inner dimension - 64
// XY groups (TERMS) or 64 samples x' (BATCH) per step - so every lane has
// kRows independent table probes in flight.  Coupled pairs found in a step
// are compacted into an LDS queue with ballot + mbcnt.  Short term runs are
// evaluated 64 pairs at a time, one pair per lane; runs longer than kLongRun
// (the diagonal group, single excitations) are evaluated by the whole wave,
// 64 terms per step.  Accumulators live in LDS, kAccCols columns per row:
// lane l adds into column l % kAccCols, the lower half of the wave before the
// upper half, and at the end lane r adds row r's columns in order, so results
// are bitwise reproducible without atomics.
//
// LoopOverTrie (Alg. 2C, trees of Alg. 3): one lane per row walks the
// radix tree of U together with the radix tree of one chunk of the XY set
// (trie.h) and evaluates each pair it reaches.
//
// The grid's y dimension splits the inner loop into chunks; every
// (row, chunk) writes one partial sum that a second kernel adds in chunk
// order.
#include "device.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

namespace {

constexpr int kWave = 64;
constexpr int kRows = 8;                 // rows per wave (TERMS / BATCH)
static_assert(kRows == kPartRows, "the partitioned LoopOverTerms tiles are whole waves of rows");
constexpr int kLongRun = 16;             // longer term runs are split over the wave
constexpr int kTrieBlock = 256;

struct PairArgs {
    const void* groups;
    const uint64_t* ghash;
    const uint64_t* gsplit;     // spin_split of the groups' XY masks [G][W]
    const void* terms;
    const void* terms_f;
    const uint64_t* gkeys;
    Table gtable;
    int n_groups;
    int maxpop;
    const uint64_t* keys;
    const uint64_t* khash;
    Table ktable;
    // prefilter parameters of U: read from `sp` at kernel start (single
    // problem) or from the batch's per-problem arrays
    const SampleParams* sp;
    const uint32_t* prep_err;   // U's preparation error word (single problem; else null)
    int sig_pa;
    int sig_n;
    bool sig_all;
    int rad_max;
    uint64_t rad_ref[kMaxWords];
    const uint32_t* bloom;   // U's Bloom filter (global); staged in LDS by the kernel
    uint32_t bloom_words;
    uint32_t bloom_mask;
    int kstash;      // stash counts, read at kernel start
    int gstash;
    int64_t M;       // samples of U (table entries, LoopOverBatch's inner loop)
    int64_t rows;    // rows evaluated: samples 0 .. rows - 1 (rows <= M)
    int per_chunk;
    int chunks;      // LoopOverBatch forward / adjoint: chunks of the 1-D grid
    // prefix trees
    const uint64_t* u_keys;
    const int32_t* u_perm;
    const TNode* u_nodes;
    const uint64_t* u_nkeys;
    const uint64_t* xy_keys;
    const int32_t* xy_gid;
    const TNode* xy_nodes;
    const uint64_t* xy_nkeys;
    int xy_chunk;
    // LoopOverTerms split by U's table partitions (large tables): workgroup w
    // serves XCD w % 8, which probes only partitions w % 8 + 8 p, pass p
    // after pass; a tile's rows share one partition class, so its groups are
    // the bucket class ^ part ^ salt's
    bool part;
    int part_bits;              // 2^part_bits partitions
    int part_salt;              // partition bits of U's table salt
    int64_t part_tiles;         // workgroup rows of one pass (>= the tiles of all classes)
    const int32_t* row_perm;    // rows ordered by class (stable)
    const int64_t* class_off;   // [2^bits + 1] first position of each class in row_perm
    const int64_t* tile_off;    // [2^bits + 1] first tile of each class
    const void* groups_b;       // group records bucketed by the partition of their hash
    const uint64_t* ghash_b;
    const uint64_t* gsplit_b;
    const int32_t* gid_b;       // group id of every record in bucket order
    // bucket starts in groups_b [kMaxParts + 1], in device memory: a kernel
    // argument array indexed at run time would move the whole argument
    // block to the stack
    const int32_t* gbucket;
    int part_sub;               // chunks of a bucket
};

PairArgs make_args(const HamDev& H, const SampleDev& S, const Plan& P) {
    PairArgs a;
    a.groups = H.groups;
    a.ghash = H.group_hash;
    a.gsplit = H.group_split;
    a.terms = H.terms;
    a.terms_f = H.terms_f;
    a.gkeys = H.group_keys;
    a.gtable = H.group_table;
    a.n_groups = static_cast<int>(H.n_groups);
    a.maxpop = H.maxpop;
    a.keys = S.keys;
    a.khash = S.hash;
    a.ktable = S.table;
    a.sp = S.params;
    a.prep_err = S.prep_err;
    a.sig_pa = 0;
    a.sig_n = 0;
    a.sig_all = true;
    a.rad_max = 128;
    a.rad_ref[0] = 0;
    a.rad_ref[1] = 0;
    a.bloom = P.bloom;
    a.bloom_words = P.bloom_words;
    a.bloom_mask = P.bloom_words ? P.bloom_words - 1u : 0u;
    a.M = S.n;
    a.rows = S.rows > 0 ? S.rows : S.n;
    a.per_chunk = P.per_chunk;
    a.chunks = P.chunks;
    a.u_keys = S.ut.keys;
    a.u_perm = S.ut.perm;
    a.u_nodes = S.ut.nodes;
    a.u_nkeys = S.ut.nkeys;
    a.xy_keys = H.xyt.keys;
    a.xy_gid = H.xyt.gid;
    a.xy_nodes = H.xyt.nodes;
    a.xy_nkeys = H.xyt.nkeys;
    a.xy_chunk = H.xyt.chunk;
    a.part = P.part;
    a.part_bits = P.part ? S.part.bits : 0;
    a.part_salt = hash_part(S.table.salt, H.part.shift, a.part_bits);
    a.part_tiles = P.part ? (a.rows + kPartRows - 1) / kPartRows + (int64_t(1) << a.part_bits) : 0;
    a.row_perm = S.part.row_perm;
    a.class_off = S.part.class_off;
    a.tile_off = S.part.tile_off;
    a.groups_b = H.part.groups;
    a.ghash_b = H.part.ghash;
    a.gsplit_b = H.part.gsplit;
    a.gid_b = H.part.gid;
    a.gbucket = H.part.bucket_dev;
    a.part_sub = P.part_sub;
    return a;
}

// popcount(x) + c in one instruction (the optimizer would otherwise turn an
// addend that is a negated signature into a separate subtraction)
__device__ __forceinline__ uint32_t popc_plus(uint32_t x, uint32_t c) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "s"(c));
    return r;
}

__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u)));
}

template <int W, int NR>
struct Rows {
    static constexpr int kN = NR;
    int n;
    int64_t row0;
    int64_t id[NR];      // sample index of each row slot (clamped copies past n)
    uint64_t x[NR][W];
    uint64_t hx[NR];
};

__device__ __forceinline__ void read_stash_counts(PairArgs& A) {
    A.kstash = static_cast<int>(__builtin_amdgcn_readfirstlane(A.ktable.stash->count));
    A.gstash = static_cast<int>(__builtin_amdgcn_readfirstlane(A.gtable.stash->count));
}

// Kernel prologue of the single-problem pair kernels: false when U's
// preparation latched an error (duplicate keys, bits >= N, a table that did
// not settle), in which case the kernel does nothing and the outputs are
// unspecified; else the prefilter parameters are loaded (wave-uniform).
__device__ __forceinline__ bool read_sample_params(PairArgs& A) {
    if (__builtin_amdgcn_readfirstlane(static_cast<int>(*A.prep_err)) != 0) return false;
    const SampleParams& p = *A.sp;
    A.sig_pa = __builtin_amdgcn_readfirstlane(p.sig_pa);
    A.sig_n = __builtin_amdgcn_readfirstlane(p.sig_n);
    A.sig_all = __builtin_amdgcn_readfirstlane(p.sig_all) != 0;
    A.rad_max = __builtin_amdgcn_readfirstlane(p.rad_max);
#pragma unroll
    for (int w = 0; w < kMaxWords; ++w) {
        const uint64_t v = p.rad_ref[w];
        A.rad_ref[w] = (static_cast<uint64_t>(static_cast<uint32_t>(
                            __builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32)))) << 32) |
                       static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
    }
    read_stash_counts(A);
    return true;
}

// A wave's row buffer in LDS: the NR rows' keys [NR][W], then their
// unsalted hashes [NR].
template <int W, int NR>
constexpr int kRowBuf = NR * (W + 1);

template <int W, int NR>
__device__ __forceinline__ void load_rows(const PairArgs& A, Rows<W, NR>& R, uint64_t* rowkey, int64_t tile) {
    R.row0 = tile * NR;
    R.n = static_cast<int>(min(static_cast<int64_t>(NR), A.rows - R.row0));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int64_t row = min(R.row0 + r, A.rows - 1);
        R.id[r] = row;
#pragma unroll
        for (int w = 0; w < W; ++w) R.x[r][w] = A.keys[row * W + w];
        R.hx[r] = A.khash[row];
    }
    if (lane_id() < NR * W) {
        const int64_t row = min(R.row0 + lane_id() / W, A.rows - 1);
        rowkey[lane_id()] = A.keys[row * W + lane_id() % W];
    }
    if (lane_id() < NR) rowkey[NR * W + lane_id()] = A.khash[min(R.row0 + lane_id(), A.rows - 1)];
}

// Rows of a tile taken through a row order: positions [p0, p0 + n) of perm.
template <int W, int NR>
__device__ __forceinline__ void load_rows_perm(const PairArgs& A, Rows<W, NR>& R, uint64_t* rowkey, int64_t p0,
                                               int n, const int32_t* __restrict__ perm) {
    R.row0 = p0;
    R.n = n;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int64_t row = perm[p0 + min(r, n - 1)];
        R.id[r] = row;
#pragma unroll
        for (int w = 0; w < W; ++w) R.x[r][w] = A.keys[row * W + w];
        R.hx[r] = A.khash[row];
    }
    if (lane_id() < NR * W) {
        const int64_t row = perm[p0 + min(lane_id() / W, n - 1)];
        rowkey[lane_id()] = A.keys[row * W + lane_id() % W];
    }
    if (lane_id() < NR) rowkey[NR * W + lane_id()] = A.khash[perm[p0 + min(lane_id(), n - 1)]];
}

// A group's term run as the hit queue carries it for narrow keys: first
// term and the real / imaginary part lengths in 16 bits each.
struct RunRef {
    uint32_t begin;
    uint32_t lens;
};
template <int W>
__device__ __forceinline__ RunRef run_ref(const GroupRec<W>& gr) {
    return RunRef{static_cast<uint32_t>(gr.begin),
                  static_cast<uint32_t>(gr.mid - gr.begin) | (static_cast<uint32_t>(gr.end - gr.mid) << 16)};
}

// LoopOverTerms: lanes over 64 groups of the chunk per step.  With SIG the
// candidate must have U's single (even-qubit, total) popcount signature.
// Rows past the end of U are clamped copies of the last row; their results
// are discarded by the caller.
// Compaction buffer entries: a candidate that passed the prefilters as row |
// lane << 3 (LoopOverTerms, exact tables) or row | sample << 3
// (LoopOverBatch).
template <bool NW>
using CEntry = uint32_t;

template <int W, int SIG, int NR, bool NW, bool BL, class Sink>
__device__ __forceinline__ void find_terms(const PairArgs& A, const Rows<W, NR>& R, int g0, int g1,
                                           const void* groups_v, const uint64_t* __restrict__ ghash,
                                           const uint64_t* __restrict__ gsplit, Sink& sink, const uint32_t* lfilt,
                                           CEntry<NW>* cb, const uint64_t* rowkey) {
    constexpr int TK = table_kind(W, NW);
    using HT = typename TabT<TK>::hash;
    // wide keys on an exact table need the XY masks only in the prefilter,
    // which then takes rows, masks and reference key in spin-split form
    constexpr bool SPLIT = SIG && !NW && TK != kTabVerify;
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(groups_v);
    const Table& T = A.ktable;
    const SlotReader<TK> slots(T);
    if (g0 >= g1) return;
    const int lane = lane_id();
    const uint32_t lane8 = static_cast<uint32_t>(lane) << 3;
    // U's signature: even-qubit popcount and the other one (odd qubits, or
    // all qubits for narrow keys).  A candidate's mismatch is the OR of its
    // two counts less U's (each popcount's own addend) and of 2^16 on lanes
    // past the bucket; it may be at most sig_tol.  When U has several
    // signatures nothing is subtracted and every valid lane passes.
    const uint32_t sig_a = A.sig_all ? 0u : static_cast<uint32_t>(A.sig_pa);
    const uint32_t sig_b = A.sig_all ? 0u : static_cast<uint32_t>(SPLIT ? A.sig_n - A.sig_pa : A.sig_n);
    const uint32_t sig_tol = A.sig_all ? 0xFFFFu : 0u;
    const uint32_t neg_a = 0u - sig_a, neg_b = 0u - sig_b;
    uint64_t rx[NR][W], ref[W];
#pragma unroll
    for (int w = 0; w < W; ++w) ref[w] = SPLIT ? spin_split(A.rad_ref[w]) : A.rad_ref[w];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int w = 0; w < W; ++w) rx[r][w] = SPLIT ? spin_split(R.x[r][w]) : R.x[r][w];
    // the step's group fields live in plain registers (mask words, term
    // run, hash)
    auto mask_word = [&](int g, int w) -> uint64_t {
        return SPLIT ? gsplit[static_cast<int64_t>(g) * W + w] : groups[g].xy[w];
    };
    uint64_t gxy[W];
    RunRef run;
    uint64_t gh;
    {
        const int g = min(g0 + lane, g1 - 1);
#pragma unroll
        for (int w = 0; w < W; ++w) gxy[w] = mask_word(g, w);
        run = run_ref(groups[g]);
        gh = ghash[g];
    }
    for (int base = g0; base < g1; base += kWave) {
        const int g = base + lane;
        const bool valid = g < g1;
        // the next step's group fields, requested before this step's probes
        // so that they arrive with them (clamped: no branch, whose join would
        // make the compiler wait for them at once)
        uint64_t nxy[W];
        RunRef nrun;
        uint64_t ngh;
        {
            const int ng = min(base + kWave + lane, g1 - 1);
#pragma unroll
            for (int w = 0; w < W; ++w) nxy[w] = mask_word(ng, w);
            nrun = run_ref(groups[ng]);
            ngh = ghash[ng];
        }
        // the exact prefilters of candidate x ^ XY for row r: U's radius
        // around its majority key, U's single popcount signature (unless
        // sig_all; lanes past the bucket carry 2^16 in the mismatch), U's
        // Bloom filter (BL).  Each test is one compare, kept as two lane
        // conditions (a, b) so that their ballots are the compares' own
        // masks, combined in scalar registers.
        const uint32_t vpen = valid ? 0u : 0x10000u;
        auto filter2 = [&](int r, bool& ok_a, bool& ok_b) {
            ok_a = valid;
            ok_b = true;
            if constexpr (SIG) {
                uint32_t pa = 0, pb = 0, d = 0;
                if constexpr (NW) {
                    const uint32_t x32 = static_cast<uint32_t>(rx[r][0]) ^ static_cast<uint32_t>(gxy[0]);
                    pa = popc_plus(x32 & static_cast<uint32_t>(kEven), neg_a);
                    pb = popc_plus(x32, neg_b);
                    d += __popc(x32 ^ static_cast<uint32_t>(ref[0]));
                } else {
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const uint64_t xp = rx[r][w] ^ gxy[w];
                        if constexpr (SPLIT) {
                            if (w == 0) {
                                pa = popc_plus(static_cast<uint32_t>(xp), neg_a);
                                pb = popc_plus(static_cast<uint32_t>(xp >> 32), neg_b);
                            } else {
                                pa += __popc(static_cast<uint32_t>(xp));
                                pb += __popc(static_cast<uint32_t>(xp >> 32));
                            }
                        } else {
                            if (w == 0) {
                                pa = neg_a;
                                pb = neg_b;
                            }
                            pa += popc64(xp & kEven);
                            pb += popc64(xp);
                        }
                        d += popc64(xp ^ ref[w]);
                    }
                }
                const uint32_t t = pa | pb | vpen;
                ok_a = d <= static_cast<uint32_t>(A.rad_max);
                ok_b = t <= sig_tol;
            }
            if constexpr (BL) {
                const uint32_t hf = static_cast<uint32_t>(R.hx[r] >> 32) ^ static_cast<uint32_t>(gh >> 32);
                const uint32_t bits = bloom_bits(hf);
                ok_b = ok_b & ((lfilt[bloom_word(hf, A.bloom_mask)] & bits) == bits);
            }
        };
        auto filter = [&](int r) -> bool {
            bool a, b;
            filter2(r, a, b);
            return a & b;
        };
        auto salted = [&](int r) -> HT { return static_cast<HT>((R.hx[r] ^ T.salt) ^ gh); };
        if constexpr (TK != kTabVerify) {
            // exact tables: the candidates that pass are compacted into dense
            // lanes (LDS, ballot + mbcnt), and only those are probed, 64 at a
            // time; a probe's group fields come from its source lane
            auto probe_round = [&](int n) {
                const bool on = lane < n;
                const uint32_t meta = cb[on ? lane : 0];
                const int r = static_cast<int>(meta & 7u);
                const int src = static_cast<int>(meta >> 3);
                // the candidate's salted hash: the row's (LDS) ^ the group's
                // (source lane)
                const uint64_t hrow = rowkey[NR * W + r] ^ T.salt;
                HT h;
                if constexpr (NW) {
                    h = static_cast<HT>(static_cast<uint32_t>(hrow) ^
                                        static_cast<uint32_t>(__shfl(static_cast<int>(gh), src, kWave)));
                } else {
                    const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(gh), src, kWave));
                    const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(gh >> 32), src, kWave));
                    h = static_cast<HT>(hrow ^ ((static_cast<uint64_t>(hi) << 32) | lo));
                }
                const auto s1 = slots.load(slot1(T, h), on);
                const auto s2 = slots.load(slot2(T, h), need_slot2<TK>(T, s1, h));
                const int jj = table_settle<TK, W>(T, A.keys, s1, s2, h, nullptr, A.kstash, on);
                const RunRef rr{static_cast<uint32_t>(__shfl(static_cast<int>(run.begin), src, kWave)),
                                static_cast<uint32_t>(__shfl(static_cast<int>(run.lens), src, kWave))};
                // low word of x ^ XY, which only the narrow hit queue carries
                // (wide keys hold the masks in spin-split form here)
                const uint32_t gx = NW ? static_cast<uint32_t>(__shfl(static_cast<int>(gxy[0]), src, kWave)) : 0u;
                sink.hit(r, on && jj >= 0, base + src, jj, rr, static_cast<uint32_t>(rowkey[r * W]) ^ gx);
                sink.flush();   // the queue never holds more than two waves of hits
            };
            int cn = 0;   // entries in cb (wave-uniform)
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                bool a, b;
                filter2(r, a, b);
                const uint64_t m = __builtin_amdgcn_ballot_w64(a) & __builtin_amdgcn_ballot_w64(b);
                if (a & b) (cb + cn)[lanes_below(m)] = static_cast<uint32_t>(r) | lane8;
                cn += __popcll(m);
                if (cn >= kWave) {
                    wave_sync();
                    probe_round(kWave);
                    const int rest = cn - kWave;
                    CEntry<NW> t{};
                    if (lane < rest) t = cb[kWave + lane];
                    wave_sync();
                    if (lane < rest) cb[lane] = t;
                    wave_sync();
                    cn = rest;
                }
            }
            if (cn > 0) {
                wave_sync();
                probe_round(cn);
                wave_sync();
            }
        } else {
            uint64_t xp[NR][W];
            typename TabT<TK>::slot v1[NR], v2[NR];
            HT hs[NR];
            bool okr[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                okr[r] = filter(r);
#pragma unroll
                for (int w = 0; w < W; ++w) xp[r][w] = R.x[r][w] ^ gxy[w];
                hs[r] = salted(r);
                v1[r] = slots.load(slot1(T, hs[r]), okr[r]);
            }
            // second slots only where the first leaves the lookup open
#pragma unroll
            for (int r = 0; r < NR; ++r) v2[r] = slots.load(slot2(T, hs[r]), need_slot2<TK>(T, v1[r], hs[r]));
            // all rows settled first: only the indices stay live through the drains
            int jr[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r)
                jr[r] = table_settle<TK, W>(T, A.keys, v1[r], v2[r], hs[r], xp[r], A.kstash, okr[r]);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                sink.hit(r, jr[r] >= 0, g, jr[r], run, static_cast<uint32_t>(R.x[r][0] ^ gxy[0]));
                sink.flush();   // the queue never holds more than two waves of hits
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) gxy[w] = nxy[w];
        run = nrun;
        gh = ngh;
    }
}

// LoopOverBatch: lanes over 64 samples x' of the chunk per step.  A pair
// (x, x') can be coupled only if popcount(x ^ x') is at most the largest XY
// popcount; the few that pass (under 1% at the workloads measured) are
// compacted into an LDS buffer (ballot + mbcnt) across steps and looked up in
// the XY table 64 at a time.  Only the keys are streamed; the hashes are read
// for the pairs that pass.
template <int W, int NR, bool NW, class Sink>
__device__ __forceinline__ void find_batch(const PairArgs& A, const Rows<W, NR>& R, int chunk, Sink& sink,
                                           CEntry<NW>* cb, const uint64_t* rowkey) {
    constexpr int TK = table_kind(W, NW);
    using HT = typename TabT<TK>::hash;
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(A.groups);
    const Table& T = A.gtable;
    const SlotReader<TK> slots(T);
    const int lane = lane_id();
    const int64_t j0 = static_cast<int64_t>(chunk) * A.per_chunk;
    const int64_t j1 = min(A.M, j0 + A.per_chunk);
    // entries [0, n) of cb: row | sample << 3 in the first word
    auto probe_round = [&](int n) {
        const bool on = lane < n;
        const uint32_t meta = cb[on ? lane : 0];
        const int r = static_cast<int>(meta & 7u);
        const int j = static_cast<int>(meta >> 3);
        const int64_t row = min(R.row0 + r, A.rows - 1);
        const HT h = static_cast<HT>((A.khash[row] ^ T.salt) ^ A.khash[j]);
        uint64_t xj[W], m[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            xj[w] = A.keys[static_cast<int64_t>(j) * W + w];
            m[w] = rowkey[r * W + w] ^ xj[w];
        }
        const auto s1 = slots.load(slot1(T, h), on);
        const auto s2 = slots.load(slot2(T, h), need_slot2<TK>(T, s1, h));
        const int g = table_settle<TK, W>(T, A.gkeys, s1, s2, h, m, A.gstash, on);
        RunRef run{};
        if (Sink::kCarry && g >= 0) run = run_ref(groups[g]);
        sink.hit(r, on && g >= 0, g, j, run, static_cast<uint32_t>(xj[0]));
        sink.flush();   // the queue never holds more than two waves of hits
    };
    int cn = 0;   // entries in cb (wave-uniform)
    for (int64_t base = j0; base < j1; base += kWave) {
        const int64_t j = base + lane;
        const bool valid = j < j1;
        const int64_t jj = valid ? j : j0;
        uint64_t xj[W];
#pragma unroll
        for (int w = 0; w < W; ++w) xj[w] = A.keys[jj * W + w];
        // popcount of x ^ x', plus 256 on lanes past the chunk: one compare
        const uint32_t vpen = valid ? 0u : 256u;
        uint32_t pc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if constexpr (NW) {
                pc[r] = vpen + __popc(static_cast<uint32_t>(R.x[r][0]) ^ static_cast<uint32_t>(xj[0]));
            } else {
                pc[r] = vpen;
#pragma unroll
                for (int w = 0; w < W; ++w) pc[r] += popc64(R.x[r][w] ^ xj[w]);
            }
        }
        const uint32_t jm = static_cast<uint32_t>(j) << 3;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const bool ok = pc[r] <= static_cast<uint32_t>(A.maxpop);
            const uint64_t mk = __builtin_amdgcn_ballot_w64(ok);
            if (ok) {
                const uint32_t at = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mk >> 32),
                                                              __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mk),
                                                                                        static_cast<uint32_t>(cn)));
                cb[at] = static_cast<uint32_t>(r) | jm;
            }
            cn += __popcll(mk);
            if (cn >= kWave) {
                wave_sync();
                probe_round(kWave);
                const int rest = cn - kWave;
                CEntry<NW> t{};
                if (lane < rest) t = cb[kWave + lane];
                wave_sync();
                if (lane < rest) cb[lane] = t;
                wave_sync();
                cn = rest;
            }
        }
    }
    if (cn > 0) {
        wave_sync();
        probe_round(cn);
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// Sinks: what happens to the pairs a wave finds.
// ---------------------------------------------------------------------------
constexpr int kAccCols = 32;   // accumulator columns per row

// Hit queue entries.  Narrow keys: (j | r << 24, first term, real / imaginary
// lengths, candidate x'), so that draining needs no group record; otherwise
// (r | g << 4, j) and the group record is read when draining.
template <bool NW>
using QEntry = std::conditional_t<NW, uint4, uint2>;

template <int W, int PREC, bool ADJ, int NR, bool NW>
struct AccSink {
    using P = Prec<PREC>;
    using Acc = typename P::Acc;
    using Vec = typename P::Vec;
    using Term = typename P::template Term<W>;
    using QE = QEntry<NW>;
    static constexpr bool kCarry = NW;

    const GroupRec<W>* groups;
    const Term* terms;
    const Vec* vec;
    QE* q;                  // LDS hit queue [2 * kWave] (flushed after each row's hits)
    Acc* acc;               // LDS accumulators [NR][kAccCols]: lane l adds into column l % kAccCols
    const uint64_t* rowkey; // LDS row keys [NR][W]
    int qn = 0;
    int nrows = 0;          // rows inside U (the rest are clamped copies)
    int64_t hits = 0;       // coupled pairs of those rows

    // a pair as the drain needs it
    struct Pair {
        int r;
        uint32_t j;
        int b, m, e;             // term run: real part [b, m), imaginary part [m, e)
        uint64_t ket[W];
    };

    __device__ __forceinline__ void hit(int r, bool h, int g, int j, RunRef run, uint32_t xp) {
        const uint64_t m = __ballot(h);
        if (h) {
            if constexpr (NW)
                q[qn + lanes_below(m)] = make_uint4(static_cast<uint32_t>(j) | (static_cast<uint32_t>(r) << 24),
                                                    run.begin, run.lens, xp);
            else
                q[qn + lanes_below(m)] = make_uint2(static_cast<uint32_t>(r) | (static_cast<uint32_t>(g) << 4),
                                                    static_cast<uint32_t>(j));
        }
        qn += __popcll(m);
        hits += __popcll(__ballot(h && r < nrows));
    }

    __device__ __forceinline__ int entry_row(const QE& e) const {
        if constexpr (NW)
            return static_cast<int>(e.x >> 24);
        else
            return static_cast<int>(e.x & 15u);
    }

    // decodes entry e (narrow: from the entry alone; else with group record gr)
    __device__ __forceinline__ Pair decode(const QE& e, const GroupRec<W>& gr) const {
        Pair p;
        p.r = entry_row(e);
        if constexpr (NW) {
            p.j = e.x & 0xFFFFFFu;
            p.b = static_cast<int>(e.y);
            p.m = p.b + static_cast<int>(e.z & 0xFFFFu);
            p.e = p.m + static_cast<int>(e.z >> 16);
            p.ket[0] = ADJ ? rowkey[p.r] : static_cast<uint64_t>(e.w);
        } else {
            p.j = e.y;
            p.b = gr.begin;
            p.m = gr.mid;
            p.e = gr.end;
#pragma unroll
            for (int w = 0; w < W; ++w) p.ket[w] = rowkey[p.r * W + w] ^ (ADJ ? 0ull : gr.xy[w]);
        }
        return p;
    }

    // called by the whole wave; lanes 0-31 add first, then lanes 32-63 (the
    // two halves share the columns, so the order of the adds is fixed)
    __device__ __forceinline__ void add(int r, const Acc& v, bool on) {
        Acc* a = acc + r * kAccCols + (lane_id() & (kAccCols - 1));
        if (on && lane_id() < kAccCols) {
            Acc t = *a;
            acc_plus(t, v);
            *a = t;
        }
        wave_sync();
        if (on && lane_id() >= kAccCols) {
            Acc t = *a;
            acc_plus(t, v);
            *a = t;
        }
        wave_sync();
    }

    // the long runs set aside in lq[0, n), kLongPer at a time, each spread
    // over kWave / kLongPer lanes: lane k first holds entry k (and, for wide
    // keys, its group record); a lane group takes its entry from that lane,
    // so that a run waits only for its own terms
    static constexpr int kLongPer = 2;
    static constexpr int kLongLanes = kWave / kLongPer;
    __device__ __forceinline__ void drain_long(const QE* lq, int n) {
        const int lane = lane_id();
        const int part = lane / kLongLanes, sub = lane % kLongLanes;
        const QE le = lq[min(lane, n - 1)];
        GroupRec<W> lgr{};
        if constexpr (!NW) lgr = groups[le.x >> 4];
        for (int k = 0; k < n; k += kLongPer) {
            const bool on = k + part < n;
            const int src = min(k + part, n - 1);
            const Pair p = decode(lane_shfl(le, src), lane_shfl(lgr, src));
            typename P::H hr = strided_first<W, NW, kLongLanes>(terms, p.b, p.m, sub, p.ket);
            typename P::H hi = strided_first<W, NW, kLongLanes>(terms, p.m, p.e, sub, p.ket);
            strided_rest<W, NW, kLongLanes>(terms, p.b, p.m, sub, p.ket, hr);
            strided_rest<W, NW, kLongLanes>(terms, p.m, p.e, sub, p.ket, hi);
            Acc v{};
            if (on) P::madd(v, hr, hi, vec[p.j]);
            add(p.r, v, on);
        }
    }

    // entries [o, o + n) of the queue, one pair per lane; runs longer than
    // kLongRun are set aside (over the entries just read, q + o) and done by
    // the whole wave
    __device__ __forceinline__ void drain(int o, int n) {
        const bool mine = lane_id() < n;
        QE e{};
        GroupRec<W> gr{};
        if (mine) {
            e = q[o + lane_id()];
            if constexpr (!NW) gr = groups[e.x >> 4];
        }
        const Pair p = decode(e, gr);
        const bool lng = mine && p.e - p.b > kLongRun;
        const uint64_t ml = __ballot(lng);
        QE* lq = q + o;
        if (lng) lq[lanes_below(ml)] = e;
        Acc v{};
        if (mine && !lng) {
            typename P::H hr, hi;
            melem<W, NW>(terms, p.b, p.m, p.e, 0, 1, p.ket, hr, hi);
            P::madd(v, hr, hi, vec[p.j]);
        }
        add(p.r, v, mine && !lng);
        if (ml) {
            wave_sync();
            drain_long(lq, __popcll(ml));
            wave_sync();
        }
    }

    __device__ __forceinline__ void flush() {
        if (qn >= kWave) {
            wave_sync();
            int o = 0;
            for (; qn - o >= kWave; o += kWave) drain(o, kWave);
            wave_sync();
            const int rest = qn - o;
            QE t{};
            if (lane_id() < rest) t = q[o + lane_id()];
            wave_sync();
            if (lane_id() < rest) q[lane_id()] = t;
            qn = rest;
        }
    }

    __device__ __forceinline__ void finish() {
        wave_sync();
        if (qn) drain(0, qn);
        qn = 0;
        wave_sync();
    }
};

struct CountSink {
    static constexpr bool kCarry = false;
    int cnt[kRows];
    // r may differ between lanes
    __device__ __forceinline__ void hit(int r, bool h, int, int, RunRef, uint32_t) {
#pragma unroll
        for (int k = 0; k < kRows; ++k) cnt[k] += __popcll(__ballot(h && r == k));
    }
    __device__ __forceinline__ void flush() {}
};

struct FillSink {
    static constexpr bool kCarry = false;
    int64_t pos[kRows];
    int64_t row0;
    int n;          // rows of this wave inside U; the rest are clamped copies
    int jbits;
    uint64_t* pkey;
    uint32_t* pval;
    const int32_t* perm = nullptr;   // row slot k is sample perm[row0 + k] (else row0 + k)
    const int32_t* gmap = nullptr;   // group g is gmap[g] (records in bucket order; else g)
    // r may differ between lanes
    __device__ __forceinline__ void hit(int r, bool h, int g, int j, RunRef, uint32_t) {
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const uint64_t m = __ballot(h && r == k);
            if (h && r == k && k < n) {
                const int64_t p = pos[k] + lanes_below(m);
                const int64_t row = perm ? perm[row0 + k] : row0 + k;
                pkey[p] = (static_cast<uint64_t>(row) << jbits) | static_cast<uint64_t>(j);
                pval[p] = static_cast<uint32_t>(gmap ? gmap[g] : g);
            }
            pos[k] += __popcll(m);
        }
    }
    __device__ __forceinline__ void flush() {}
};

// VARIANT: 0 TERMS without signature filter, 3 TERMS with it, 1 BATCH.
// NW: keys of at most 32 qubits (narrow table, 32-bit bit work).
// BL: the prefiltered LoopOverTerms also tests U's Bloom filter in LDS.
template <int W, int VARIANT, int NR, bool NW, bool BL = false, class Sink>
__device__ __forceinline__ void find(const PairArgs& A, const Rows<W, NR>& R, int chunk, Sink& sink,
                                     CEntry<NW>* cb, const uint64_t* rowkey, const uint32_t* lfilt = nullptr) {
    const int g0 = chunk * A.per_chunk;
    const int g1 = min(A.n_groups, g0 + A.per_chunk);
    if constexpr (VARIANT == 0)
        find_terms<W, 0, NR, NW, false>(A, R, g0, g1, A.groups, A.ghash, A.gsplit, sink, lfilt, cb, rowkey);
    else if constexpr (VARIANT == 3)
        find_terms<W, 1, NR, NW, BL>(A, R, g0, g1, A.groups, A.ghash, A.gsplit, sink, lfilt, cb, rowkey);
    else
        find_batch<W, NR, NW>(A, R, chunk, sink, cb, rowkey);
}

// ---------------------------------------------------------------------------
// Fused forward / adjoint kernel (TERMS, BATCH).
//   forward: acc_x = sum_{x'} H_xx' vec_x'  (ket x', vec = a)
//   adjoint: acc_y = sum_{x}  H_xy vec_x    (ket y,  vec = w / a)
// ---------------------------------------------------------------------------
// WPB waves per workgroup, each owning its own row tile (tile = blockIdx.x *
// WPB + wave); with WPB > 1 the waves share U's Bloom filter, staged in LDS
// (dynamic shared memory) once per workgroup.  LoopOverBatch runs on a 1-D
// grid with chunk = workgroup id mod chunks: workgroups go to the eight XCDs
// in turn, so with a multiple of eight chunks each XCD streams only its own
// chunks of U through its L2.  PART: LoopOverTerms by U's table partitions
// (a separate instantiation, so that the plain kernel keeps its registers).
// The work item of workgroup blockIdx.x in the partitioned LoopOverTerms
// (1-D grid): workgroup w serves XCD w % 8; the rest of w gives the pass p
// (partition k = w % 8 + 8 p), then (tile, sub-chunk); the tile's class c
// gives the group bucket c ^ k ^ part(salt), whose candidates all fall in
// partition k.  Loads the tile's rows and sets the bucket range [g0, g1) of
// the records in bucket order and the chunk index k * part_sub + sub; false
// for a workgroup past the items.
template <int W, int NR>
__device__ __forceinline__ bool part_item(const PairArgs& A, Rows<W, NR>& R, uint64_t* rowkey, int& g0, int& g1,
                                          int& chunk) {
    const int nparts = 1 << A.part_bits;
    const int64_t rest = blockIdx.x / kXcds;
    const int64_t per_pass = A.part_tiles * A.part_sub;
    const int k = static_cast<int>(blockIdx.x % kXcds) + kXcds * static_cast<int>(rest / per_pass);
    const int64_t item = rest % per_pass;
    const int sub = static_cast<int>(item % A.part_sub);
    const int64_t t = item / A.part_sub;
    if (k >= nparts || t >= A.tile_off[nparts]) return false;
    int c = 0;   // the tile's class: the last class starting at or before t
    for (int q = 1; q < nparts; ++q) c += t >= A.tile_off[q] ? 1 : 0;
    const int64_t p0 = A.class_off[c] + (t - A.tile_off[c]) * NR;
    const int n = static_cast<int>(min(static_cast<int64_t>(NR), A.class_off[c + 1] - p0));
    load_rows_perm<W, NR>(A, R, rowkey, p0, n, A.row_perm);
    const int r = rev_bits(c ^ k ^ A.part_salt, A.part_bits);
    const int bs = A.gbucket[r << (kMaxPartBits - A.part_bits)];
    const int be = A.gbucket[(r + 1) << (kMaxPartBits - A.part_bits)];
    const int per = (be - bs + A.part_sub - 1) / A.part_sub;
    g0 = min(be, bs + sub * per);
    g1 = min(be, g0 + per);
    chunk = k * A.part_sub + sub;
    return true;
}

template <int W, int VARIANT, int PREC, bool ADJ, int NR, bool NW, int WPB, bool PART = false>
__global__ __launch_bounds__(kWave * WPB) void k_pairs(PairArgs A, const void* __restrict__ vec,
                                                       void* __restrict__ partial) {
    using P = Prec<PREC>;
    using Acc = typename P::Acc;
    constexpr bool BL = WPB > 1;
    __shared__ uint64_t rowkey_s[WPB][kRowBuf<W, NR>];
    __shared__ QEntry<NW> q_s[WPB][2 * kWave];
    __shared__ CEntry<NW> cb_s[WPB][2 * kWave];
    static_assert(sizeof(Acc) == sizeof(double2), "accumulators are 16 bytes");
    __shared__ double2 acc_s[WPB][NR * kAccCols];
    extern __shared__ uint32_t lfilt[];
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
    if (!read_sample_params(A)) return;   // the same for every thread of the block
    if constexpr (BL) {
        for (uint32_t t = threadIdx.x; t < A.bloom_words; t += kWave * WPB) lfilt[t] = A.bloom[t];
        __syncthreads();
    }
    int64_t tile = static_cast<int64_t>(blockIdx.x) * WPB + wave;
    int chunk = static_cast<int>(blockIdx.y);
    if constexpr (VARIANT == 1) {
        chunk = static_cast<int>(blockIdx.x % static_cast<unsigned>(A.chunks));
        tile = static_cast<int64_t>(blockIdx.x / static_cast<unsigned>(A.chunks));
    }
    uint64_t* rowkey = rowkey_s[wave];
    Acc* acc = reinterpret_cast<Acc*>(acc_s[wave]);
    Rows<W, NR> R;
    int g0 = 0, g1 = 0;
    static_assert(!PART || (VARIANT != 1 && WPB == 1 && NR == kPartRows), "partitioned LoopOverTerms tiles");
    constexpr bool part = PART;
    if constexpr (part) {
        if (!part_item<W, NR>(A, R, rowkey, g0, g1, chunk)) return;
    } else {
        if (tile * NR >= A.rows) return;   // no block-wide barrier follows
        load_rows<W, NR>(A, R, rowkey, tile);
    }
    for (int i = lane_id(); i < NR * kAccCols; i += kWave) acc[i] = Acc{};
    wave_sync();
    AccSink<W, PREC, ADJ, NR, NW> sink;
    sink.groups = static_cast<const GroupRec<W>*>(part ? A.groups_b : A.groups);
    sink.terms = static_cast<const typename P::template Term<W>*>(PREC == 0 ? A.terms : A.terms_f);
    sink.vec = static_cast<const typename P::Vec*>(vec);
    sink.q = q_s[wave];
    sink.acc = acc;
    sink.rowkey = rowkey;
    if constexpr (part)
        find_terms<W, VARIANT == 3 ? 1 : 0, NR, NW, BL>(A, R, g0, g1, A.groups_b, A.ghash_b, A.gsplit_b, sink, lfilt, cb_s[wave],
                                                         rowkey);
    else
        find<W, VARIANT, NR, NW, BL>(A, R, chunk, sink, cb_s[wave], rowkey, lfilt);
    sink.finish();
    // per-row totals: lane r adds the columns of row r in order
    if (lane_id() < R.n) {
        Acc t{};
        for (int l = 0; l < kAccCols; ++l) acc_plus(t, acc[lane_id() * kAccCols + l]);
        int64_t id = R.row0 + lane_id();
        if constexpr (part) {
            id = R.id[0];
#pragma unroll
            for (int r = 1; r < NR; ++r) id = lane_id() == r ? R.id[r] : id;
        }
        store_acc(partial, static_cast<int64_t>(chunk) * A.rows + id, t);
    }
}

// Pair counts per (row, chunk) and the pair list (FillSink), LoopOverTerms
// and LoopOverBatch; PART: LoopOverTerms by U's table partitions (1-D grid,
// as the partitioned pair kernel; rows through the class order, groups in
// bucket order, reported under their own ids).
template <int W, int VARIANT, bool NW, bool PART = false>
__global__ __launch_bounds__(kWave) void k_count(PairArgs A, int chunks, int32_t* __restrict__ counts) {
    __shared__ uint64_t rowkey[kRowBuf<W, kRows>];
    __shared__ CEntry<NW> cb[2 * kWave];
    Rows<W, kRows> R;
    if (!read_sample_params(A)) {   // no pairs while U is invalid (PART: the caller clears the counts)
        const int64_t row = static_cast<int64_t>(blockIdx.x) * kRows + lane_id();
        if (!PART && lane_id() < kRows && row < A.rows) counts[row * chunks + blockIdx.y] = 0;
        return;
    }
    CountSink sink;
#pragma unroll
    for (int r = 0; r < kRows; ++r) sink.cnt[r] = 0;
    int chunk = static_cast<int>(blockIdx.y);
    if constexpr (PART) {
        int g0 = 0, g1 = 0;
        if (!part_item<W, kRows>(A, R, rowkey, g0, g1, chunk)) return;
        wave_sync();
        find_terms<W, VARIANT == 3 ? 1 : 0, kRows, NW, false>(A, R, g0, g1, A.groups_b, A.ghash_b, A.gsplit_b,
                                                              sink, nullptr, cb, rowkey);
    } else {
        load_rows<W, kRows>(A, R, rowkey, blockIdx.x);
        wave_sync();
        find<W, VARIANT, kRows, NW>(A, R, blockIdx.y, sink, cb, rowkey);
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r)
        if (lane_id() == r && r < R.n) counts[R.id[r] * chunks + chunk] = sink.cnt[r];
}

template <int W, int VARIANT, bool NW, bool PART = false>
__global__ __launch_bounds__(kWave) void k_fill(PairArgs A, int chunks, int jbits, const int64_t* __restrict__ offsets,
                                                uint64_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
    __shared__ uint64_t rowkey[kRowBuf<W, kRows>];
    __shared__ CEntry<NW> cb[2 * kWave];
    if (!read_sample_params(A)) return;
    Rows<W, kRows> R;
    int chunk = static_cast<int>(blockIdx.y);
    int g0 = 0, g1 = 0;
    if constexpr (PART) {
        if (!part_item<W, kRows>(A, R, rowkey, g0, g1, chunk)) return;
    } else {
        load_rows<W, kRows>(A, R, rowkey, blockIdx.x);
    }
    wave_sync();
    FillSink sink;
    sink.row0 = R.row0;
    sink.n = R.n;
    sink.jbits = jbits;
    sink.pkey = pkey;
    sink.pval = pval;
    if constexpr (PART) {
        sink.perm = A.row_perm;
        sink.gmap = A.gid_b;
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) sink.pos[r] = r < R.n ? offsets[R.id[r] * chunks + chunk] : 0;
    if constexpr (PART)
        find_terms<W, VARIANT == 3 ? 1 : 0, kRows, NW, false>(A, R, g0, g1, A.groups_b, A.ghash_b, A.gsplit_b,
                                                              sink, nullptr, cb, rowkey);
    else
        find<W, VARIANT, kRows, NW>(A, R, blockIdx.y, sink, cb, rowkey);
}

// ---------------------------------------------------------------------------
// Batched pair kernel.  Workgroup w (one wave) takes work items w, w + grid,
// ... of its key format's range (one item per workgroup unless the schedule
// asks for a few workgroups per compute unit; the hardware hands workgroups
// to free slots in order, which balances uneven items as a work counter
// would, without its round trip); item t belongs to the problem whose
// [item0, item0 + items) holds it (found by a ballot over the item starts,
// kept in four lane registers), and is the (row tile, chunk) pair
// u / chunks, u % chunks of that problem.  The item body is the forward row
// kernel above with the problem's own tables, variant and signature filter;
// a row's chunk partials land at the problem's partial offset.
// ---------------------------------------------------------------------------
// Wave-uniform copies of values read from memory at a uniform address: the
// first lane's, so that they live in scalar registers (the compiler cannot
// tell that a descriptor read through a pointer is the same in every lane).
__device__ __forceinline__ uint32_t rfl32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int32_t rfl32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
    return (static_cast<uint64_t>(rfl32(static_cast<uint32_t>(v >> 32))) << 32) | rfl32(static_cast<uint32_t>(v));
}
__device__ __forceinline__ int64_t rfl64(int64_t v) { return static_cast<int64_t>(rfl64(static_cast<uint64_t>(v))); }
template <class T>
__device__ __forceinline__ T* rflp(T* p) {
    return reinterpret_cast<T*>(rfl64(reinterpret_cast<uint64_t>(p)));
}
__device__ __forceinline__ Table rfl_table(const Table& t) {
    Table u;
    u.slots = rflp(t.slots);
    u.mask = rfl32(t.mask);
    u.ibits = rfl32(t.ibits);
    u.imask = rfl32(t.imask);
    u.fpshift = rfl32(t.fpshift);
    u.capbits = rfl32(t.capbits);
    u.pmask = rfl32(t.pmask);
    u.salt = rfl64(t.salt);
    u.stash = rflp(t.stash);
    return u;
}

// One work item of the batched kernel: the forward row kernel over a row
// tile and chunk of problem D, with the problem's own tables, variant and
// signature filter (NW: the problem's narrow format).  Returns the coupled
// pairs of the tile's rows inside U.
template <int W, int PREC, int NR, bool NW>
__device__ __forceinline__ int64_t batch_item(const PairArgs& A, const Rows<W, NR>& R, int variant, int64_t s0,
                                              int chunk, const void* vec_all, typename Prec<PREC>::Acc* acc,
                                              QEntry<NW>* q, CEntry<NW>* cb, const uint64_t* rowkey) {
    using P = Prec<PREC>;
    AccSink<W, PREC, false, NR, NW> sink;
    sink.groups = static_cast<const GroupRec<W>*>(A.groups);
    sink.terms = static_cast<const typename P::template Term<W>*>(PREC == 0 ? A.terms : A.terms_f);
    sink.vec = static_cast<const typename P::Vec*>(vec_all) + s0;
    sink.q = q;
    sink.acc = acc;
    sink.rowkey = rowkey;
    sink.nrows = R.n;
    // one LoopOverTerms body: without a usable prefilter the problem has
    // sig_all set and rad_max 128, which every candidate passes
    if (variant == 1)
        find_batch<W, NR, NW>(A, R, chunk, sink, cb, rowkey);
    else
        find_terms<W, 1, NR, NW, false>(A, R, chunk * A.per_chunk, min(A.n_groups, (chunk + 1) * A.per_chunk),
                                        A.groups, A.ghash, A.gsplit, sink, nullptr, cb, rowkey);
    sink.finish();
    return sink.hits;
}

// NW: the kernel takes the items of the narrow problems, [0, narrow_items),
// from counter 0; else the rest from counter 1.
template <int W, int PREC, int NR, bool NW>
__global__ __launch_bounds__(kWave) void k_pairs_batched(BatchDev B, const void* __restrict__ vec_all,
                                                         void* __restrict__ partial_all) {
    using P = Prec<PREC>;
    using Acc = typename P::Acc;
    __shared__ uint64_t rowkey[kRowBuf<W, NR>];
    __shared__ QEntry<NW> q[2 * kWave];
    __shared__ CEntry<NW> cb[2 * kWave];
    static_assert(sizeof(Acc) == sizeof(double2), "accumulators are 16 bytes");
    __shared__ double2 acc_raw[NR * kAccCols];
    Acc* acc = reinterpret_cast<Acc*>(acc_raw);
    const int lane = lane_id();
    constexpr int kSlices = kMaxBatch / kWave;
    int64_t istart[kSlices];
#pragma unroll
    for (int c = 0; c < kSlices; ++c) {
        const int p = c * kWave + lane;
        istart[c] = p < B.n ? B.probs[B.sched[p]].item0 : INT64_MAX;
    }
    const int64_t first = NW ? 0 : B.narrow_items;
    const int64_t last = NW ? B.narrow_items : B.total_items;
    for (int64_t t = first + blockIdx.x; t < last; t += gridDim.x) {
        int pos = -1;
#pragma unroll
        for (int c = 0; c < kSlices; ++c) pos += __popcll(__ballot(istart[c] <= t));
        // the problem's descriptor, every field wave-uniform
        const int k = rfl32(B.sched[pos]);
        const BatchProb& D = B.probs[k];
        const int64_t s0 = rfl64(D.s0), M = rfl64(D.M), item0 = rfl64(D.item0), pbase = rfl64(D.pbase);
        const int chunks = rfl32(D.chunks), variant = rfl32(D.variant);
        PairArgs A;
        A.groups = rflp(D.groups);
        A.ghash = rflp(D.ghash);
        A.gsplit = rflp(D.gsplit);
        A.terms = rflp(D.terms);
        A.terms_f = rflp(D.terms_f);
        A.gkeys = rflp(D.gkeys);
        A.gtable = rfl_table(D.gtable);
        A.n_groups = rfl32(D.n_groups);
        A.maxpop = rfl32(D.maxpop);
        A.keys = B.keys + s0 * W;
        A.khash = B.khash + s0;
        A.ktable = rfl_table(D.ktable);
        A.M = M;
        A.rows = M;
        A.per_chunk = rfl32(D.per_chunk);
        const uint32_t smin = rfl32(B.sigmin[k]), smax = rfl32(B.sigmax[k]);
        A.sig_pa = static_cast<int>(smin >> 8);
        A.sig_n = static_cast<int>(smin & 255u);
        A.sig_all = smin != smax;
        A.rad_ref[0] = rfl64(static_cast<uint64_t>(B.rad[3 * k]));
        A.rad_ref[1] = rfl64(static_cast<uint64_t>(B.rad[3 * k + 1]));
        const int rmax = static_cast<int>(rfl64(static_cast<uint64_t>(B.rad[3 * k + 2])));
        A.rad_max = 2 * rmax < rfl32(D.n_qubits) ? rmax : 128;
        read_stash_counts(A);
        const int64_t u = t - item0;
        const int64_t tile = u / chunks;
        const int chunk = static_cast<int>(u - tile * chunks);
        Rows<W, NR> R;
        load_rows<W, NR>(A, R, rowkey, tile);
        for (int i = lane; i < NR * kAccCols; i += kWave) acc[i] = Acc{};
        wave_sync();
        const int64_t hits = batch_item<W, PREC, NR, NW>(A, R, variant, s0, chunk, vec_all, acc, q, cb, rowkey);
        if (lane < R.n) {
            Acc s{};
            for (int l = 0; l < kAccCols; ++l) acc_plus(s, acc[lane * kAccCols + l]);
            auto* part = static_cast<double2*>(partial_all) + pbase;
            store_acc(part, static_cast<int64_t>(chunk) * M + R.row0 + lane, s);
        }
        if (lane == 0) atomicAdd(B.pairs + k, static_cast<unsigned long long>(hits));
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// LoopOverTrie: one lane per row, walk U tree x XY chunk tree.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void trie_views(const PairArgs& A, int chunk, TrieView& U, TrieView& V, int64_t& vbase) {
    U.keys = A.u_keys;
    U.nodes = A.u_nodes;
    U.nkeys = A.u_nkeys;
    U.n = A.M;
    vbase = static_cast<int64_t>(chunk) * A.xy_chunk;
    V.keys = A.xy_keys + vbase * W;
    V.nodes = A.xy_nodes + static_cast<int64_t>(chunk) * (A.xy_chunk - 1);
    V.nkeys = A.xy_nkeys + static_cast<int64_t>(chunk) * (A.xy_chunk - 1) * W;
    V.n = min(static_cast<int64_t>(A.xy_chunk), static_cast<int64_t>(A.n_groups) - vbase);
}

// Bytes of LDS that hold one XY chunk tree (nodes, node keys, keys).
template <int W>
__host__ __device__ inline size_t trie_chunk_bytes(int64_t chunk) {
    const int64_t nn = chunk > 1 ? chunk - 1 : 0;
    return static_cast<size_t>(nn) * sizeof(TNode) + static_cast<size_t>(nn + chunk) * W * sizeof(uint64_t);
}
constexpr size_t kTrieLdsMax = 48 * 1024;

// STAGE: the workgroup first copies its XY chunk tree into LDS (when it fits
// in kTrieLdsMax), so that the XY side of every walk step is an LDS read.
template <int W, int PREC, bool ADJ, bool STAGE>
__global__ __launch_bounds__(kTrieBlock) void k_pairs_trie(PairArgs A, const void* __restrict__ vec,
                                                           void* __restrict__ partial) {
    using P = Prec<PREC>;
    extern __shared__ uint64_t tsm[];
    // no walk over an invalid U (the trees assume unique keys); uniform per block
    if (__builtin_amdgcn_readfirstlane(static_cast<int>(*A.prep_err)) != 0) return;
    TrieView U, V;
    int64_t vbase;
    trie_views<W>(A, blockIdx.y, U, V, vbase);
    if constexpr (STAGE) {
        const int64_t nn = V.n > 1 ? V.n - 1 : 0;
        TNode* ln = reinterpret_cast<TNode*>(tsm);
        uint64_t* lnk = reinterpret_cast<uint64_t*>(ln + nn);
        uint64_t* lk = lnk + nn * W;
        for (int64_t t = threadIdx.x; t < nn; t += kTrieBlock) ln[t] = V.nodes[t];
        for (int64_t t = threadIdx.x; t < nn * W; t += kTrieBlock) lnk[t] = V.nkeys[t];
        for (int64_t t = threadIdx.x; t < V.n * W; t += kTrieBlock) lk[t] = V.keys[t];
        __syncthreads();
        V.nodes = ln;
        V.nkeys = lnk;
        V.keys = lk;
    }
    // lanes take the rows in sorted key order: neighbouring lanes then walk
    // similar paths (less divergence, shared cache lines)
    const int64_t srow = static_cast<int64_t>(blockIdx.x) * kTrieBlock + threadIdx.x;
    if (srow >= A.M) return;   // no barrier follows
    const int64_t row = A.u_perm[srow];
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = A.u_keys[srow * W + w];
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(A.groups);
    const auto* __restrict__ terms =
        static_cast<const typename P::template Term<W>*>(PREC == 0 ? A.terms : A.terms_f);
    const auto* __restrict__ v = static_cast<const typename P::Vec*>(vec);
    typename P::Acc acc;
    trie_walk<W>(x, U, V, [&](int32_t ul, int32_t vl) {
        const GroupRec<W> gr = groups[A.xy_gid[vbase + vl]];
        const uint64_t* ket = ADJ ? x : (U.keys + static_cast<int64_t>(ul) * W);
        typename P::H hr, hi;
        melem<W>(terms, gr.begin, gr.mid, gr.end, 0, 1, ket, hr, hi);
        P::madd(acc, hr, hi, v[A.u_perm[ul]]);
    });
    store_acc(partial, static_cast<int64_t>(blockIdx.y) * A.M + row, acc);
}

template <int W>
__global__ __launch_bounds__(kTrieBlock) void k_count_trie(PairArgs A, int chunks, int32_t* __restrict__ counts) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kTrieBlock + threadIdx.x;
    if (row >= A.M) return;
    if (*A.prep_err != 0u) {   // no pairs while U is invalid
        counts[row * chunks + blockIdx.y] = 0;
        return;
    }
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = A.keys[row * W + w];
    TrieView U, V;
    int64_t vbase;
    trie_views<W>(A, blockIdx.y, U, V, vbase);
    int n = 0;
    trie_walk<W>(x, U, V, [&](int32_t, int32_t) { ++n; });
    counts[row * chunks + blockIdx.y] = n;
}

template <int W>
__global__ __launch_bounds__(kTrieBlock) void k_fill_trie(PairArgs A, int chunks, int jbits,
                                                          const int64_t* __restrict__ offsets,
                                                          uint64_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kTrieBlock + threadIdx.x;
    if (row >= A.M || *A.prep_err != 0u) return;
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = A.keys[row * W + w];
    TrieView U, V;
    int64_t vbase;
    trie_views<W>(A, blockIdx.y, U, V, vbase);
    int64_t pos = offsets[row * chunks + blockIdx.y];
    trie_walk<W>(x, U, V, [&](int32_t ul, int32_t vl) {
        pkey[pos] = (static_cast<uint64_t>(row) << jbits) | static_cast<uint64_t>(A.u_perm[ul]);
        pval[pos] = static_cast<uint32_t>(A.xy_gid[vbase + vl]);
        ++pos;
    });
}

// ---------------------------------------------------------------------------
// LoopOverTrie, wave-cooperative walk.  A workgroup of kTW waves shares one
// XY chunk tree (staged in LDS when it is small); each wave owns kTRows rows
// of U taken in sorted key order and walks U's tree against the chunk tree
// for all of them at once.  The frontier of (row, U node, XY node, bit down
// to which the pair is verified) entries is a stack in LDS: every step the
// wave takes up to 64 entries from its top, one per lane, checks the bits
// between the entry's verified bit and the next branch bit with one masked
// XOR, and compacts the surviving children back onto the stack with
// ballot + mbcnt; a pair of leaves is a coupled pair and goes to the sink.
// Close to a full stack the wave takes one entry per step (a depth-first
// walk grows the stack by at most one entry per bit), so the stack never
// overflows.
// ---------------------------------------------------------------------------
constexpr int kTW = 4;          // waves per workgroup
constexpr int kTRows = kRows;   // rows per wave
constexpr int kTStack = 512;    // stack entries per wave
constexpr size_t kTrieStageMax = 16 * 1024;
constexpr int kTrieWaveMaxChunk = 32767;   // XY nodes coded in 16 bits

// entry: x = U node (>= 0 internal, < 0 leaf ~i); y = XY node code (16 bits:
// leaf i -> i, internal n -> chunk size + n) | verified bit d << 16 | row << 24
__device__ __forceinline__ uint32_t tenc(int32_t v, int chunk_n, int d, int r) {
    const uint32_t vc = v >= 0 ? static_cast<uint32_t>(chunk_n + v) : static_cast<uint32_t>(~v);
    return vc | (static_cast<uint32_t>(d) << 16) | (static_cast<uint32_t>(r) << 24);
}

template <int W, class Sink>
__device__ __forceinline__ int64_t trie_wave_walk(const PairArgs& A, const TrieView& U, const TrieView& V,
                                                  int64_t vbase, const uint64_t* rowkey, int nrows, uint2* stk,
                                                  Sink& sink) {
    const int lane = lane_id();
    const int chunk_n = static_cast<int>(V.n);
    const int32_t u0 = U.n > 1 ? 0 : ~0;
    const int32_t v0 = V.n > 1 ? 0 : ~0;
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(A.groups);
    if (lane < nrows) stk[lane] = make_uint2(static_cast<uint32_t>(u0), tenc(v0, chunk_n, 64 * W, lane));
    int sp = nrows;   // wave-uniform
    int64_t visits = 0;
    constexpr int kSlack = 64 * W + 2;
    wave_sync();
    while (sp > 0) {
        const int n = (sp + kWave <= kTStack - kSlack) ? min(kWave, sp) : 1;
        const bool on = lane < n;
        // idle lanes decode the roots (valid indices; their results are discarded)
        const uint2 e = on ? stk[sp - n + lane] : make_uint2(static_cast<uint32_t>(u0), tenc(v0, chunk_n, 0, 0));
        sp -= n;
        visits += n;
        wave_sync();   // the popped entries are read before the pushes overwrite them
        const int32_t u = static_cast<int32_t>(e.x);
        const int vc = static_cast<int>(e.y & 0xFFFFu);
        const int d = static_cast<int>((e.y >> 16) & 0xFFu);
        const int r = static_cast<int>(e.y >> 24);
        const int32_t v = vc >= chunk_n ? vc - chunk_n : ~vc;
        const uint64_t* x = rowkey + r * W;
        const TNode nu = u >= 0 ? U.nodes[u] : TNode{0, 0, ~u, -1};
        const TNode nv = v >= 0 ? V.nodes[v] : TNode{0, 0, ~v, -1};
        const uint64_t* ku = u >= 0 ? U.nkeys + static_cast<int64_t>(u) * W : U.keys + static_cast<int64_t>(~u) * W;
        const uint64_t* kv = v >= 0 ? V.nkeys + static_cast<int64_t>(v) * W : V.keys + static_cast<int64_t>(~v) * W;
        const int b = nu.bit > nv.bit ? nu.bit : nv.bit;
        const bool agree = on && trie_agree<W>(x, ku, kv, b + 1, d);
        const bool leaf = agree && b < 0;
        int32_t a_u = kNoNode, a_v = kNoNode, c_u = kNoNode, c_v = kNoNode;
        if (agree && b >= 0) {
            const int xb = trie_bit<W>(x, b);
            int32_t u_0, u_1, v_0, v_1;
            if (nu.bit == b) {
                u_0 = nu.left;
                u_1 = nu.right;
            } else {
                const int ub = trie_bit<W>(ku, b);
                u_0 = ub ? kNoNode : u;
                u_1 = ub ? u : kNoNode;
            }
            if (nv.bit == b) {
                v_0 = nv.left;
                v_1 = nv.right;
            } else {
                const int vb = trie_bit<W>(kv, b);
                v_0 = vb ? kNoNode : v;
                v_1 = vb ? v : kNoNode;
            }
            // x'_b = 0: U child 0 with XY child x_b; x'_b = 1: U child 1 with XY child 1 - x_b
            a_u = u_0;
            a_v = xb ? v_1 : v_0;
            c_u = u_1;
            c_v = xb ? v_0 : v_1;
        }
        const bool a_ok = a_u != kNoNode && a_v != kNoNode;
        const bool c_ok = c_u != kNoNode && c_v != kNoNode;
        const uint64_t ma = __ballot(a_ok), mc = __ballot(c_ok);
        if (a_ok) stk[sp + lanes_below(ma)] = make_uint2(static_cast<uint32_t>(a_u), tenc(a_v, chunk_n, b, r));
        if (c_ok)
            stk[sp + __popcll(ma) + lanes_below(mc)] = make_uint2(static_cast<uint32_t>(c_u), tenc(c_v, chunk_n, b, r));
        sp += __popcll(ma) + __popcll(mc);
        // a pair of leaves: sample j = U's leaf in caller order, group of XY's leaf
        int g = 0, j = 0;
        RunRef run{};
        uint32_t xp = 0;
        if (leaf) {
            g = A.xy_gid[vbase + nv.rep];
            j = A.u_perm[nu.rep];
            xp = static_cast<uint32_t>(U.keys[static_cast<int64_t>(nu.rep) * W]);
            if (Sink::kCarry) run = run_ref(groups[g]);
        }
        sink.hit(r, leaf, g, j, run, xp);
        sink.flush();
        wave_sync();
    }
    return visits;
}

template <int W>
__device__ __forceinline__ void stage_chunk_tree(TrieView& V, uint64_t* tsm, int nthreads) {
    const int64_t nn = V.n > 1 ? V.n - 1 : 0;
    TNode* ln = reinterpret_cast<TNode*>(tsm);
    uint64_t* lnk = reinterpret_cast<uint64_t*>(ln + nn);
    uint64_t* lk = lnk + nn * W;
    for (int64_t t = threadIdx.x; t < nn; t += nthreads) ln[t] = V.nodes[t];
    for (int64_t t = threadIdx.x; t < nn * W; t += nthreads) lnk[t] = V.nkeys[t];
    for (int64_t t = threadIdx.x; t < V.n * W; t += nthreads) lk[t] = V.keys[t];
    __syncthreads();
    V.nodes = ln;
    V.nkeys = lnk;
    V.keys = lk;
}

template <int W, int PREC, bool ADJ, bool NW, bool STAGE>
__global__ __launch_bounds__(kWave * kTW) void k_pairs_trie_w(PairArgs A, const void* __restrict__ vec,
                                                              void* __restrict__ partial) {
    using P = Prec<PREC>;
    using Acc = typename P::Acc;
    extern __shared__ uint64_t tsm[];
    __shared__ uint64_t rowkey_s[kTW][kTRows * W];
    __shared__ QEntry<NW> q_s[kTW][2 * kWave];
    __shared__ double2 acc_s[kTW][kTRows * kAccCols];
    __shared__ uint2 stk_s[kTW][kTStack];
    // no walk over an invalid U (the trees assume unique keys); uniform per block
    if (__builtin_amdgcn_readfirstlane(static_cast<int>(*A.prep_err)) != 0) return;
    TrieView U, V;
    int64_t vbase;
    trie_views<W>(A, blockIdx.y, U, V, vbase);
    if constexpr (STAGE) stage_chunk_tree<W>(V, tsm, kWave * kTW);
    const int wave = static_cast<int>(threadIdx.x) / kWave;
    const int lane = lane_id();
    const int64_t srow0 = (static_cast<int64_t>(blockIdx.x) * kTW + wave) * kTRows;
    if (srow0 >= A.M) return;   // no block-wide barrier follows
    const int nrows = static_cast<int>(min(static_cast<int64_t>(kTRows), A.M - srow0));
    uint64_t* rowkey = rowkey_s[wave];
    if (lane < kTRows * W) rowkey[lane] = A.u_keys[min(srow0 + lane / W, A.M - 1) * W + lane % W];
    Acc* acc = reinterpret_cast<Acc*>(acc_s[wave]);
    for (int i = lane; i < kTRows * kAccCols; i += kWave) acc[i] = Acc{};
    wave_sync();
    AccSink<W, PREC, ADJ, kTRows, NW> sink;
    sink.groups = static_cast<const GroupRec<W>*>(A.groups);
    sink.terms = static_cast<const typename P::template Term<W>*>(PREC == 0 ? A.terms : A.terms_f);
    sink.vec = static_cast<const typename P::Vec*>(vec);
    sink.q = q_s[wave];
    sink.acc = acc;
    sink.rowkey = rowkey;
    trie_wave_walk<W>(A, U, V, vbase, rowkey, nrows, stk_s[wave], sink);
    sink.finish();
    if (lane < nrows) {
        Acc t{};
        for (int l = 0; l < kAccCols; ++l) acc_plus(t, acc[lane * kAccCols + l]);
        store_acc(partial, static_cast<int64_t>(blockIdx.y) * A.M + A.u_perm[srow0 + lane], t);
    }
}

// Pair counts (MODE 0), pair emission (MODE 1) or node-pair visits (MODE 2)
// of the wave-cooperative walk.
struct NullSink {
    static constexpr bool kCarry = false;
    __device__ __forceinline__ void hit(int, bool, int, int, RunRef, uint32_t) {}
    __device__ __forceinline__ void flush() {}
};

template <int W, int MODE>
__global__ __launch_bounds__(kWave) void k_trie_w_list(PairArgs A, int chunks, int jbits,
                                                       int32_t* __restrict__ counts,
                                                       const int64_t* __restrict__ offsets,
                                                       uint64_t* __restrict__ pkey, uint32_t* __restrict__ pval,
                                                       unsigned long long* __restrict__ visits) {
    __shared__ uint64_t rowkey[kTRows * W];
    __shared__ uint2 stk[kTStack];
    const int lane = lane_id();
    const int64_t srow0 = static_cast<int64_t>(blockIdx.x) * kTRows;
    if (srow0 >= A.M) return;
    const int nrows = static_cast<int>(min(static_cast<int64_t>(kTRows), A.M - srow0));
    if (*A.prep_err != 0u) {   // no pairs while U is invalid
        if (MODE == 0 && lane < nrows) counts[static_cast<int64_t>(A.u_perm[srow0 + lane]) * chunks + blockIdx.y] = 0;
        return;
    }
    TrieView U, V;
    int64_t vbase;
    trie_views<W>(A, blockIdx.y, U, V, vbase);
    if (lane < kTRows * W) rowkey[lane] = A.u_keys[min(srow0 + lane / W, A.M - 1) * W + lane % W];
    wave_sync();
    if constexpr (MODE == 0) {
        CountSink sink;
#pragma unroll
        for (int r = 0; r < kRows; ++r) sink.cnt[r] = 0;
        trie_wave_walk<W>(A, U, V, vbase, rowkey, nrows, stk, sink);
#pragma unroll
        for (int r = 0; r < kRows; ++r)
            if (lane == r && r < nrows) counts[static_cast<int64_t>(A.u_perm[srow0 + r]) * chunks + blockIdx.y] = sink.cnt[r];
    } else if constexpr (MODE == 1) {
        FillSink sink;
        sink.row0 = srow0;
        sink.n = nrows;
        sink.jbits = jbits;
        sink.pkey = pkey;
        sink.pval = pval;
        sink.perm = A.u_perm;
#pragma unroll
        for (int r = 0; r < kRows; ++r)
            sink.pos[r] = r < nrows ? offsets[static_cast<int64_t>(A.u_perm[srow0 + r]) * chunks + blockIdx.y] : 0;
        trie_wave_walk<W>(A, U, V, vbase, rowkey, nrows, stk, sink);
    } else {
        NullSink sink;
        const int64_t n = trie_wave_walk<W>(A, U, V, vbase, rowkey, nrows, stk, sink);
        if (lane == 0) atomicAdd(visits, static_cast<unsigned long long>(n));
    }
}

// MatrixElement for given sample pairs (ket x_j); with cnt / grp also the
// pair's group and its term count.
template <int W, bool NW>
__global__ __launch_bounds__(256) void k_pair_elements(PairArgs A, int64_t n, const int32_t* __restrict__ pi,
                                                       const int32_t* __restrict__ pj, double2* __restrict__ out,
                                                       int32_t* __restrict__ cnt, int32_t* __restrict__ grp,
                                                       uint32_t* __restrict__ err) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t >= n) return;
    const int64_t i = pi[t], j = pj[t];
    if (i < 0 || j < 0 || i >= A.M || j >= A.M) {
        atomicOr(err, static_cast<uint32_t>(kErrIndex));
        out[t] = make_double2(0.0, 0.0);
        if (cnt) {
            cnt[t] = 0;
            grp[t] = -1;
        }
        return;
    }
    uint64_t xj[W], m[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        xj[w] = A.keys[j * W + w];
        m[w] = A.keys[i * W + w] ^ xj[w];
    }
    const int g = table_find<table_kind(W, NW), W>(A.gtable, A.gkeys, A.khash[i] ^ A.khash[j], m);
    double hr = 0.0, hi = 0.0;
    int32_t nt = 0;
    if (g >= 0) {
        const GroupRec<W> gr = static_cast<const GroupRec<W>*>(A.groups)[g];
        melem<W, NW>(static_cast<const TermRec<W>*>(A.terms), gr.begin, gr.mid, gr.end, 0, 1, xj, hr, hi);
        nt = gr.end - gr.begin;
    }
    out[t] = make_double2(hr, hi);
    if (cnt) {
        cnt[t] = nt;
        grp[t] = g;
    }
}

// Per-term phase exponents of pair t (ket x_j): the group's terms are
// stored as two runs, even |Y| then odd |Y|, each in caller order; they are
// merged back into caller order by their caller index.
template <int W>
__global__ __launch_bounds__(256) void k_pair_phases(PairArgs A, int64_t n, const int32_t* __restrict__ pj,
                                                     const int32_t* __restrict__ grp,
                                                     const int64_t* __restrict__ offsets, uint8_t* __restrict__ kout,
                                                     int64_t capacity, const int32_t* __restrict__ src,
                                                     const uint8_t* __restrict__ ny, uint32_t* __restrict__ err) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t >= n) return;
    if (offsets[n] > capacity) {
        if (t == 0) atomicOr(err, static_cast<uint32_t>(kErrCapacity));
        return;
    }
    const int g = grp[t];
    if (g < 0) return;
    const int64_t j = pj[t];
    uint64_t xj[W];
#pragma unroll
    for (int w = 0; w < W; ++w) xj[w] = A.keys[j * W + w];
    const GroupRec<W> gr = static_cast<const GroupRec<W>*>(A.groups)[g];
    const TermRec<W>* __restrict__ terms = static_cast<const TermRec<W>*>(A.terms);
    int a = gr.begin, b = gr.mid;
    int64_t o = offsets[t];
    while (a < gr.mid || b < gr.end) {
        const bool take_a = b >= gr.end || (a < gr.mid && src[a] < src[b]);
        const int p = take_a ? a : b;
        int pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) pc += popc64(xj[w] & terms[p].yz[w]);
        kout[o++] = static_cast<uint8_t>((ny[p] + 2 * pc) & 3);
        if (take_a)
            ++a;
        else
            ++b;
    }
}

inline unsigned div_up(int64_t n, int64_t d) { return static_cast<unsigned>((n + d - 1) / d); }

// ---------------------------------------------------------------------------
// Stored pair lists.  k_pairs_to_csr turns the emitted pairs (row-major by
// construction: each (row, chunk) writes a contiguous range) into a CSR of
// (column j, H_ij with the ket x_j); k_spmv then sums a row with one wave,
// lanes striding over its pairs and a fixed-order butterfly at the end:
//   forward: acc_i = sum_p H_p vec[j_p]
//   adjoint: acc_y = sum_p conj(H_p) vec[j_p]  (H_xy = conj(H_yx), H Hermitian)
// ---------------------------------------------------------------------------
template <int W, bool NW>
__global__ __launch_bounds__(256) void k_pairs_to_csr(PairArgs A, int64_t n, const uint64_t* __restrict__ pkey,
                                                      const uint32_t* __restrict__ pval, int jbits,
                                                      int32_t* __restrict__ col, double2* __restrict__ h) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t >= n) return;
    const int64_t j = static_cast<int64_t>(pkey[t] & ((1ull << jbits) - 1ull));
    const GroupRec<W> gr = static_cast<const GroupRec<W>*>(A.groups)[pval[t]];
    uint64_t xj[W];
#pragma unroll
    for (int w = 0; w < W; ++w) xj[w] = A.keys[j * W + w];
    double hr, hi;
    melem<W, NW>(static_cast<const TermRec<W>*>(A.terms), gr.begin, gr.mid, gr.end, 0, 1, xj, hr, hi);
    col[t] = static_cast<int32_t>(j);
    h[t] = make_double2(hr, hi);
}

__global__ __launch_bounds__(256) void k_rowptr(const int64_t* __restrict__ offsets, int64_t M, int chunks,
                                                int64_t* __restrict__ rowptr) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i <= M) rowptr[i] = offsets[i * chunks];
}

template <int PREC, bool ADJ>
__global__ __launch_bounds__(kWave) void k_spmv(int64_t M, const int64_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col, const double2* __restrict__ h,
                                                const void* __restrict__ vec, void* __restrict__ partial) {
    using P = Prec<PREC>;
    const int64_t i = blockIdx.x;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    typename P::Acc acc;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kWave) {
        double2 hv = h[p];
        if (ADJ) hv.y = -hv.y;
        const int32_t j = col[p];
        if constexpr (PREC == 0) {
            mac(acc, hv.x, hv.y, static_cast<const double2*>(vec)[j]);
        } else {
            const float4 s = split_c(hv.x, hv.y);
            mac(acc, F2{s.x, s.y}, F2{s.z, s.w}, static_cast<const float4*>(vec)[j]);
        }
    }
    wave_sum(acc);
    if (threadIdx.x == 0) store_acc(partial, i, acc);
}



template <int W, int VARIANT, int PREC, bool ADJ, bool NW>
hipError_t launch_pairs_t(const PairArgs& A, const Plan& P, const void* vec, void* partial, hipStream_t st) {
    if constexpr (VARIANT == 2) {
        const size_t lds = trie_chunk_bytes<W>(A.xy_chunk);
        if (A.xy_chunk <= kTrieWaveMaxChunk) {
            dim3 grid(div_up(A.M, kTRows * kTW), static_cast<unsigned>(P.chunks));
            if (lds <= kTrieStageMax)
                hipLaunchKernelGGL((k_pairs_trie_w<W, PREC, ADJ, NW, true>), grid, dim3(kWave * kTW), lds, st, A, vec,
                                   partial);
            else
                hipLaunchKernelGGL((k_pairs_trie_w<W, PREC, ADJ, NW, false>), grid, dim3(kWave * kTW), 0, st, A, vec,
                                   partial);
        } else {
            dim3 grid(div_up(A.M, kTrieBlock), static_cast<unsigned>(P.chunks));
            if (lds <= kTrieLdsMax)
                hipLaunchKernelGGL((k_pairs_trie<W, PREC, ADJ, true>), grid, dim3(kTrieBlock), lds, st, A, vec, partial);
            else
                hipLaunchKernelGGL((k_pairs_trie<W, PREC, ADJ, false>), grid, dim3(kTrieBlock), 0, st, A, vec, partial);
        }
    } else if (VARIANT == 3 && P.bloom_words > 0 && P.waves_per_block == 4) {
        constexpr int kW = 4;
        const size_t lds = sizeof(uint32_t) * P.bloom_words;
        if (P.rows_per_block == 4) {
            dim3 grid(div_up(div_up(A.rows, 4), kW), static_cast<unsigned>(P.chunks));
            hipLaunchKernelGGL((k_pairs<W, VARIANT, PREC, ADJ, 4, NW, kW>), grid, dim3(kWave * kW), lds, st, A, vec,
                               partial);
        } else {
            dim3 grid(div_up(div_up(A.rows, kRows), kW), static_cast<unsigned>(P.chunks));
            hipLaunchKernelGGL((k_pairs<W, VARIANT, PREC, ADJ, kRows, NW, kW>), grid, dim3(kWave * kW), lds, st, A,
                               vec, partial);
        }
    } else if (P.rows_per_block == 4) {
        dim3 grid(div_up(A.rows, 4), static_cast<unsigned>(P.chunks));
        if (VARIANT == 1) grid = dim3(div_up(A.rows, 4) * static_cast<unsigned>(P.chunks));
        hipLaunchKernelGGL((k_pairs<W, VARIANT, PREC, ADJ, 4, NW, 1>), grid, dim3(kWave), 0, st, A, vec, partial);
    } else {
        dim3 grid(div_up(A.rows, kRows), static_cast<unsigned>(P.chunks));
        if (VARIANT == 1) grid = dim3(div_up(A.rows, kRows) * static_cast<unsigned>(P.chunks));
        if constexpr (VARIANT != 1) {
            if (A.part) {
                // partitioned LoopOverTerms: at most rows / 8 + 2^bits tiles
                // (classes padded to whole tiles) per partition, part_sub
                // chunks each; 8 partitions per pass
                grid = dim3(static_cast<unsigned>(A.part_tiles * A.part_sub * (int64_t(1) << A.part_bits)));
                hipLaunchKernelGGL((k_pairs<W, VARIANT, PREC, ADJ, kRows, NW, 1, true>), grid, dim3(kWave), 0, st, A,
                                   vec, partial);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_pairs<W, VARIANT, PREC, ADJ, kRows, NW, 1>), grid, dim3(kWave), 0, st, A, vec, partial);
    }
    return hipGetLastError();
}

template <int W, int VARIANT, bool ADJ, bool NW>
hipError_t dispatch_prec(int precision, const PairArgs& A, const Plan& P, const void* vec, void* partial,
                         hipStream_t st) {
    return precision == 0 ? launch_pairs_t<W, VARIANT, 0, ADJ, NW>(A, P, vec, partial, st)
                          : launch_pairs_t<W, VARIANT, 1, ADJ, NW>(A, P, vec, partial, st);
}

template <int W, bool ADJ, bool NW>
hipError_t dispatch_variant(int variant, int precision, const PairArgs& A, const Plan& P, const void* vec,
                            void* partial, hipStream_t st) {
    if (variant == 0 && P.sig_filter) return dispatch_prec<W, 3, ADJ, NW>(precision, A, P, vec, partial, st);
    if (variant == 0) return dispatch_prec<W, 0, ADJ, NW>(precision, A, P, vec, partial, st);
    if (variant == 1) return dispatch_prec<W, 1, ADJ, NW>(precision, A, P, vec, partial, st);
    return dispatch_prec<W, 2, ADJ, NW>(precision, A, P, vec, partial, st);
}

template <bool ADJ>
hipError_t dispatch_width(const HamDev& H, int variant, int precision, const PairArgs& A, const Plan& P,
                          const void* v, void* partial, hipStream_t st) {
    if (H.W == 2) return dispatch_variant<2, ADJ, false>(variant, precision, A, P, v, partial, st);
    if (H.narrow) return dispatch_variant<1, ADJ, true>(variant, precision, A, P, v, partial, st);
    return dispatch_variant<1, ADJ, false>(variant, precision, A, P, v, partial, st);
}

}  // namespace

int rows_per_block(int variant, int requested) {
    if (variant == 2) return kTrieBlock;
    return requested == 4 ? 4 : kRows;
}

hipError_t launch_trie_visits(const HamDev& H, const SampleDev& S, const Plan& P, unsigned long long* visits,
                              hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    if (A.xy_chunk > kTrieWaveMaxChunk) return hipErrorInvalidValue;
    dim3 grid(div_up(A.M, kTRows), static_cast<unsigned>(P.chunks));
    if (H.W == 2)
        hipLaunchKernelGGL((k_trie_w_list<2, 2>), grid, dim3(kWave), 0, st, A, P.chunks, 0, nullptr, nullptr, nullptr,
                           nullptr, visits);
    else
        hipLaunchKernelGGL((k_trie_w_list<1, 2>), grid, dim3(kWave), 0, st, A, P.chunks, 0, nullptr, nullptr, nullptr,
                           nullptr, visits);
    return hipGetLastError();
}

hipError_t launch_pairs(bool adjoint, int variant, int precision, const HamDev& H, const SampleDev& S, const Plan& P,
                        const double2* vec, const float4* vecf, void* partial, hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    const void* v = precision == 0 ? static_cast<const void*>(vec) : static_cast<const void*>(vecf);
    return adjoint ? dispatch_width<true>(H, variant, precision, A, P, v, partial, st)
                   : dispatch_width<false>(H, variant, precision, A, P, v, partial, st);
}

template <int W, int PREC, int NR, bool NW>
static const void* batch_kernel_ptr() {
    return reinterpret_cast<const void*>(&k_pairs_batched<W, PREC, NR, NW>);
}

template <int W, bool NW>
static const void* batch_kernel_w(int precision, int rows) {
    if (precision == 0) return rows == 4 ? batch_kernel_ptr<W, 0, 4, NW>() : batch_kernel_ptr<W, 0, 8, NW>();
    return rows == 4 ? batch_kernel_ptr<W, 1, 4, NW>() : batch_kernel_ptr<W, 1, 8, NW>();
}

static const void* batch_kernel(int W, bool narrow, int precision, int rows) {
    if (W == 2) return batch_kernel_w<2, false>(precision, rows);
    return narrow ? batch_kernel_w<1, true>(precision, rows) : batch_kernel_w<1, false>(precision, rows);
}

int batch_blocks_per_cu(int W, bool narrow, int precision, int rows) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel(W, W == 1 && narrow, precision, rows), kWave,
                                                     0) !=
        hipSuccess)
        return 0;
    return n;
}

hipError_t launch_batch_pairs(const BatchDev& B, int precision, int rows, int narrow_blocks, int wide_blocks,
                              hipStream_t st) {
    const void* vec = precision == 0 ? static_cast<const void*>(B.a) : static_cast<const void*>(B.af);
    void* part = B.partial;
    void* args[] = {const_cast<BatchDev*>(&B), &vec, &part};
    if (B.narrow_items > 0) {
        const hipError_t e = hipLaunchKernel(batch_kernel(B.W, true, precision, rows),
                                             dim3(static_cast<unsigned>(narrow_blocks)), dim3(kWave), args, 0, st);
        if (e != hipSuccess) return e;
    }
    if (B.total_items > B.narrow_items)
        return hipLaunchKernel(batch_kernel(B.W, false, precision, rows), dim3(static_cast<unsigned>(wide_blocks)),
                               dim3(kWave), args, 0, st);
    return hipSuccess;
}

template <int W, bool NW>
static hipError_t count_w(int variant, const PairArgs& A, const Plan& P, int32_t* counts, hipStream_t st) {
    if (variant == 2 && A.xy_chunk <= kTrieWaveMaxChunk) {
        dim3 grid(div_up(A.M, kTRows), static_cast<unsigned>(P.chunks));
        hipLaunchKernelGGL((k_trie_w_list<W, 0>), grid, dim3(kWave), 0, st, A, P.chunks, 0, counts, nullptr, nullptr,
                           nullptr, nullptr);
    } else if (variant == 2) {
        dim3 grid(div_up(A.M, kTrieBlock), static_cast<unsigned>(P.chunks));
        hipLaunchKernelGGL(k_count_trie<W>, grid, dim3(kTrieBlock), 0, st, A, P.chunks, counts);
    } else if (variant == 0 && A.part) {
        const dim3 grid(static_cast<unsigned>(A.part_tiles * A.part_sub * (int64_t(1) << A.part_bits)));
        if (P.sig_filter)
            hipLaunchKernelGGL((k_count<W, 3, NW, true>), grid, dim3(kWave), 0, st, A, P.chunks, counts);
        else
            hipLaunchKernelGGL((k_count<W, 0, NW, true>), grid, dim3(kWave), 0, st, A, P.chunks, counts);
    } else {
        dim3 grid(div_up(A.M, kRows), static_cast<unsigned>(P.chunks));
        if (variant == 0 && P.sig_filter)
            hipLaunchKernelGGL((k_count<W, 3, NW>), grid, dim3(kWave), 0, st, A, P.chunks, counts);
        else if (variant == 0)
            hipLaunchKernelGGL((k_count<W, 0, NW>), grid, dim3(kWave), 0, st, A, P.chunks, counts);
        else
            hipLaunchKernelGGL((k_count<W, 1, NW>), grid, dim3(kWave), 0, st, A, P.chunks, counts);
    }
    return hipGetLastError();
}

template <int W, bool NW>
static hipError_t fill_w(int variant, const PairArgs& A, const Plan& P, int jbits, const int64_t* offsets,
                         uint64_t* pkey, uint32_t* pval, hipStream_t st) {
    if (variant == 2 && A.xy_chunk <= kTrieWaveMaxChunk) {
        dim3 grid(div_up(A.M, kTRows), static_cast<unsigned>(P.chunks));
        hipLaunchKernelGGL((k_trie_w_list<W, 1>), grid, dim3(kWave), 0, st, A, P.chunks, jbits, nullptr, offsets, pkey,
                           pval, nullptr);
    } else if (variant == 2) {
        dim3 grid(div_up(A.M, kTrieBlock), static_cast<unsigned>(P.chunks));
        hipLaunchKernelGGL(k_fill_trie<W>, grid, dim3(kTrieBlock), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
    } else if (variant == 0 && A.part) {
        const dim3 grid(static_cast<unsigned>(A.part_tiles * A.part_sub * (int64_t(1) << A.part_bits)));
        if (P.sig_filter)
            hipLaunchKernelGGL((k_fill<W, 3, NW, true>), grid, dim3(kWave), 0, st, A, P.chunks, jbits, offsets, pkey,
                               pval);
        else
            hipLaunchKernelGGL((k_fill<W, 0, NW, true>), grid, dim3(kWave), 0, st, A, P.chunks, jbits, offsets, pkey,
                               pval);
    } else {
        dim3 grid(div_up(A.M, kRows), static_cast<unsigned>(P.chunks));
        if (variant == 0 && P.sig_filter)
            hipLaunchKernelGGL((k_fill<W, 3, NW>), grid, dim3(kWave), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
        else if (variant == 0)
            hipLaunchKernelGGL((k_fill<W, 0, NW>), grid, dim3(kWave), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
        else
            hipLaunchKernelGGL((k_fill<W, 1, NW>), grid, dim3(kWave), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
    }
    return hipGetLastError();
}

hipError_t launch_pairs_count(int variant, const HamDev& H, const SampleDev& S, const Plan& P, int32_t* counts,
                              hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    if (H.W == 2) return count_w<2, false>(variant, A, P, counts, st);
    return H.narrow ? count_w<1, true>(variant, A, P, counts, st) : count_w<1, false>(variant, A, P, counts, st);
}

hipError_t launch_pairs_fill(int variant, const HamDev& H, const SampleDev& S, const Plan& P, int jbits,
                             const int64_t* offsets, uint64_t* pkey, uint32_t* pval, hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    if (H.W == 2) return fill_w<2, false>(variant, A, P, jbits, offsets, pkey, pval, st);
    return H.narrow ? fill_w<1, true>(variant, A, P, jbits, offsets, pkey, pval, st)
                    : fill_w<1, false>(variant, A, P, jbits, offsets, pkey, pval, st);
}

hipError_t launch_pairs_to_csr(const HamDev& H, const SampleDev& S, int64_t n, const uint64_t* pkey,
                               const uint32_t* pval, int jbits, int32_t* col, double2* h, hipStream_t st) {
    Plan P;
    const PairArgs A = make_args(H, S, P);
    const dim3 grid(div_up(n, 256)), block(256);
    if (H.W == 2)
        hipLaunchKernelGGL((k_pairs_to_csr<2, false>), grid, block, 0, st, A, n, pkey, pval, jbits, col, h);
    else if (H.narrow)
        hipLaunchKernelGGL((k_pairs_to_csr<1, true>), grid, block, 0, st, A, n, pkey, pval, jbits, col, h);
    else
        hipLaunchKernelGGL((k_pairs_to_csr<1, false>), grid, block, 0, st, A, n, pkey, pval, jbits, col, h);
    return hipGetLastError();
}

hipError_t launch_rowptr(const int64_t* offsets, int64_t M, int chunks, int64_t* rowptr, hipStream_t st) {
    hipLaunchKernelGGL(k_rowptr, dim3(div_up(M + 1, 256)), dim3(256), 0, st, offsets, M, chunks, rowptr);
    return hipGetLastError();
}

hipError_t launch_spmv(bool adjoint, int precision, int64_t M, const int64_t* rowptr, const int32_t* col,
                       const double2* h, const void* vec, void* partial, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>(M)), block(kWave);
    if (precision == 0) {
        if (adjoint)
            hipLaunchKernelGGL((k_spmv<0, true>), grid, block, 0, st, M, rowptr, col, h, vec, partial);
        else
            hipLaunchKernelGGL((k_spmv<0, false>), grid, block, 0, st, M, rowptr, col, h, vec, partial);
    } else {
        if (adjoint)
            hipLaunchKernelGGL((k_spmv<1, true>), grid, block, 0, st, M, rowptr, col, h, vec, partial);
        else
            hipLaunchKernelGGL((k_spmv<1, false>), grid, block, 0, st, M, rowptr, col, h, vec, partial);
    }
    return hipGetLastError();
}

hipError_t launch_pair_elements(const HamDev& H, const SampleDev& S, int64_t n, const int32_t* pi, const int32_t* pj,
                                double2* out, int32_t* cnt, int32_t* grp, uint32_t* err, hipStream_t st) {
    Plan P;
    const PairArgs A = make_args(H, S, P);
    const dim3 grid(div_up(n, 256)), block(256);
    if (H.W == 2)
        hipLaunchKernelGGL((k_pair_elements<2, false>), grid, block, 0, st, A, n, pi, pj, out, cnt, grp, err);
    else if (H.narrow)
        hipLaunchKernelGGL((k_pair_elements<1, true>), grid, block, 0, st, A, n, pi, pj, out, cnt, grp, err);
    else
        hipLaunchKernelGGL((k_pair_elements<1, false>), grid, block, 0, st, A, n, pi, pj, out, cnt, grp, err);
    return hipGetLastError();
}

hipError_t launch_pair_phases(const HamDev& H, const SampleDev& S, int64_t n, const int32_t* pj, const int32_t* grp,
                              const int64_t* offsets, uint8_t* kout, int64_t capacity, uint32_t* err,
                              hipStream_t st) {
    Plan P;
    const PairArgs A = make_args(H, S, P);
    const dim3 grid(div_up(n, 256)), block(256);
    if (H.W == 2)
        hipLaunchKernelGGL(k_pair_phases<2>, grid, block, 0, st, A, n, pj, grp, offsets, kout, capacity, H.term_src,
                           H.term_ny, err);
    else
        hipLaunchKernelGGL(k_pair_phases<1>, grid, block, 0, st, A, n, pj, grp, offsets, kout, capacity, H.term_src,
                           H.term_ny, err);
    return hipGetLastError();
}

}  // namespace eloc
