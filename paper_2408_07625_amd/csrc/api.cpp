// C ABI of the engine (include/eloc.h): context, Hamiltonian ingest, sample
// preparation and the entry points.  Device work is enqueued through the
// launchers of kernels.hip on the context's stream.
#include "eloc.h"
#include "ham.h"
#include "host.h"
#include "internal.h"
#include "trie.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>


using namespace eloc;

namespace {

// U tables of at least this many bytes are probed by partition (an XCD's L2
// is 4 MB), in as many partitions (8, 16 or 32) as it takes to bring one
// partition down to kPartTargetBytes
constexpr uint64_t kPartAutoBytes = uint64_t(8) << 20;
constexpr uint64_t kPartTargetBytes = uint64_t(1) << 20;

}  // namespace

struct eloc_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    uint64_t R[128];
    DevBuf R_dev;

    bool ham_set = false;
    HamDev H;
    DevBuf groups, terms, terms_f, term_src, term_ny, ghash, gkeys, gslots, gstash;
    DevBuf groups_b, ghash_b, gsplit_b, gid_b;   // group records bucketed by the partition of their hash
    DevBuf gsplit;              // spin_split of every group's XY mask
    DevBuf gbucket;             // their bucket starts [kMaxParts + 1] (int32)
    DevBuf pe_cnt, pe_grp;   // pair_elements: term counts and groups of the pairs
    DevBuf xyt_keys, xyt_gid, xyt_nodes, xyt_nkeys;

    bool samples_set = false;
    SampleDev S;
    DevBuf keys, khash, kslots, kstash, sig, bitcounts, rad, sparams, bloom;
    uint32_t bloom_words = 0;   // Bloom filter of U (0: none)
    bool bloom_built = false;   // built on first use by a kernel that reads it
    DevBuf ut_keys, ut_perm, ut_nodes, ut_nkeys;
    bool ut_valid = false;
    DevBuf part_perm, part_class, part_tile;   // U's rows by partition class
    bool part_ok = false;                      // U's table is partitioned and its rows classed
    int part_bits = 0;                         // 2^part_bits partitions of U's table (0: none)
    DevBuf s_key, s_val, s_key2, s_val2;   // sort scratch

    DevBuf a, b, af, bf, v, vf, shift, amp_scratch;
    DevBuf partial, energy_scratch, err_run, err_prep;
    uint32_t* err_host = nullptr;    // pinned words for synchronous read-backs
    void* ws = nullptr;              // this device's fixed workspace (eloc_local_energy_noalloc)

    DevBuf counts, offsets, scan_scratch, pkey, pval, pkey2, pval2, hist, hist_off, hist_scratch;

    // conventional local energy: the extra states' list (raw, sorted, run
    // flags and positions) and the set X = U followed by the extra states
    DevBuf m_raw, m_sorted, m_perm, m_flags, m_pos, m_count;
    // the last eloc_find_misses result (m_sorted / m_flags / m_pos), valid
    // for these samples, this Hamiltonian and tolerance
    bool miss_valid = false;
    double miss_tol = 0.0;
    int64_t miss_total = 0, miss_uniq = 0;
    DevBuf x_keys, x_hash, x_slots, x_stash, x_sig, x_bitcounts, x_rad, x_params, x_err, x_logpsi;
    DevBuf x_a, x_b, x_af, x_bf, x_shift;
    DevBuf x_part_perm, x_part_class, x_part_tile;   // U's rows by partition class of the U-and-extra table
    // stochastic reconfiguration scratch
    DevBuf sr_w, sr_mean, sr_part, sr_T, sr_L, sr_y;
    // sampler: two prefix beams, the candidates of a level, the allowed count
    DevBuf ar_keys[2], ar_l[2], ar_T[2], ar_cl, ar_cT, ar_ck, ar_ci, ar_ck2, ar_ci2, ar_cnt;
    DevBuf ar_hist, ar_sel, ar_keep, ar_off;   // top-K selection scratch

    // stored pair list (CSR by row of (column, H_ij)), valid until the
    // samples or the Hamiltonian change
    DevBuf st_rowptr, st_col, st_h;
    bool st_valid = false;
    int64_t st_pairs = 0;

    int tune_chunks = 0;     // 0 = automatic
    int tune_sig = 1;
    int tune_rows = 0;       // 0 = automatic
    int tune_bloom = 0;      // the LDS Bloom filter is slower on MI355X (occupancy); opt-in
    int tune_waves = 0;      // 0 = automatic
    int tune_part = 0;       // 0 automatic, 1 on where possible, -1 off
    int tune_part_count = 0; // partitions: 0 automatic, 8, 16 or 32
    int tune_trie_chunk = 0; // XY masks per LoopOverTrie chunk tree (0: automatic)
    uint64_t kslots_n = 0;   // slots of U's membership table
    uint64_t salt_state = 0x5EED2408ull;

    // stage profiling: HIP events around each stage, read (and reset) by
    // eloc_profile_read
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    struct Mark {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
};

namespace {

int fail(eloc_ctx c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(eloc_ctx c, hipError_t e, const char* where) {
    return fail(c, e == hipErrorOutOfMemory ? ELOC_ENOMEM : ELOC_EHIP,
                std::string(where) + ": " + hipGetErrorString(e));
}

#define ELOC_HIP(ctx, expr)                                 \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

int valid_variant(int v) { return v == ELOC_TERMS || v == ELOC_BATCH || v == ELOC_TRIE || v == ELOC_AUTO; }

// ELOC_AUTO: LoopOverBatch when U is no larger than the unique XY set (its
// M^2 candidates, most rejected by a popcount test, are then fewer than
// LoopOverTerms' M x |XY| lookups), else LoopOverTerms.
int resolve_variant(const eloc_ctx c, int v) {
    if (v != ELOC_AUTO) return v;
    return c->S.n <= c->H.n_groups ? ELOC_BATCH : ELOC_TERMS;
}

// Launch geometry.  TERMS / BATCH: one wave per rows_per_block rows, the
// inner loop (groups / samples) split into chunks of whole 64-lane steps so
// that the grid has about `target` waves.  TRIE: one lane per row, one chunk
// per XY tree.
// LoopOverTerms by the 2^bits partitions of the membership table, over M
// rows, where the launch shape allows it (one wave of kPartRows rows per
// workgroup): each XCD probes its own partitions, one at a time, so that
// the XCD's L2 holds the partition it works on (the partition of a
// candidate is linear in the row's and the group's hashes).
void set_part_plan(Plan& P, int64_t M, int bits) {
    if (bits <= 0 || P.rows_per_block != kPartRows || P.waves_per_block != 1) return;
    const int64_t target = 65536;   // (row tile, chunk) waves, as the unpartitioned plan
    const int64_t nparts = int64_t(1) << bits;
    const int64_t items = ((M + kPartRows - 1) / kPartRows + nparts) * nparts;
    P.part = true;
    P.part_sub = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(64, (target + items - 1) / items)));
    P.chunks = static_cast<int>(nparts) * P.part_sub;
    P.bloom_words = 0;
}

Plan make_plan(const eloc_ctx c, int variant, int64_t n_rows = -1, bool allow_part = false) {
    Plan P;
    const int64_t M = n_rows >= 0 ? n_rows : c->S.n;
    // LoopOverTerms with the prefilters reads U's Bloom filter from LDS when
    // U has one: 4 waves of 4 rows share it; else one wave of 8 rows
    // (the shared filter needs 4-row waves to keep the workgroup's LDS under 64 KB)
    const bool bloom = variant == ELOC_TERMS && c->tune_bloom != 0 && c->bloom_words > 0 && c->tune_rows != 8 &&
                       c->tune_waves != 1;
    const int rows = c->tune_rows ? c->tune_rows : (bloom ? 4 : 8);
    P.rows_per_block = rows_per_block(variant, rows);
    P.waves_per_block = bloom ? 4 : 1;
    // the exact prefilters of LoopOverTerms (U's single popcount signature,
    // U's radius around its majority key): the kernel reads their parameters
    // from the device, and a prefilter that U does not allow passes everything
    P.sig_filter = c->tune_sig != 0;
    P.bloom_words = (bloom && P.sig_filter) ? c->bloom_words : 0;
    P.bloom = c->bloom.as<uint32_t>();
    if (variant == ELOC_TRIE) {
        P.chunks = c->H.xyt.chunks;
        P.per_chunk = c->H.xyt.chunk;
        return P;
    }
    const int64_t waves = (M + P.rows_per_block - 1) / P.rows_per_block;   // row tiles
    // about 65 536 (row tile, chunk) waves: at the medium workload 8 chunks of
    // LoopOverTerms run 1.17 ms against 1.25 ms with 2 (a shorter tail)
    const int64_t target = 65536;
    const int64_t span = (variant == ELOC_TERMS) ? c->H.n_groups : M;
    const int64_t steps = (span + 63) / 64;
    int64_t chunks = c->tune_chunks > 0 ? c->tune_chunks : (target + waves - 1) / waves;
    // LoopOverBatch: a multiple of eight chunks, one set per XCD (the kernel
    // maps workgroup id mod chunks to the chunk)
    if (variant == ELOC_BATCH && c->tune_chunks <= 0) chunks = (std::max<int64_t>(chunks, 8) + 7) / 8 * 8;
    chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, steps));
    const int64_t per_steps = (steps + chunks - 1) / chunks;
    const int64_t per = per_steps * 64;
    P.chunks = static_cast<int>((span + per - 1) / per);
    P.per_chunk = static_cast<int>(per);
    // LoopOverTerms over a large U table: by its partitions
    if (allow_part && variant == ELOC_TERMS && c->part_ok && n_rows < 0) set_part_plan(P, M, c->part_bits);
    return P;
}

// Partition bits of U's table of `bytes` bytes and `cap` slots (0: not
// partitioned): automatic for tables of kPartAutoBytes or more, enough
// partitions (8 to 32) to bring one down to kPartTargetBytes; a tuned count
// otherwise.  Never more than the table's slots allow.
int part_bits_for(const eloc_ctx c, uint64_t bytes, uint64_t cap) {
    if (c->tune_part < 0 || (c->tune_part == 0 && bytes < kPartAutoBytes)) return 0;
    int bits = 3;
    if (c->tune_part_count >= 8) {
        while ((1 << bits) < c->tune_part_count) ++bits;
    } else {
        while (bits < kMaxPartBits && (bytes >> bits) > kPartTargetBytes) ++bits;
    }
    while (bits >= 3 && cap < part_min_slots(c->H.part.shift, bits)) --bits;
    return bits >= 3 ? bits : 0;
}

// One cuckoo table of U with a fresh salt, its verification (duplicates,
// signature bitmap) and the prefilter parameters; asynchronous.
int build_sample_table(eloc_ctx c) {
    const int64_t n = c->S.n;
    const int tk = table_kind(c->H.W, c->H.narrow);
    c->S.table = make_table(c->kslots.p, c->kstash.as<Stash>(), c->kslots_n, n, splitmix64(c->salt_state),
                            c->H.part.shift, c->part_bits);
    ELOC_HIP(c, hipMemsetAsync(c->kslots.p, 0, slot_bytes(tk) * c->kslots_n, c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->kstash.p, 0, sizeof(Stash), c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->sig.p, 0, sizeof(uint64_t) * kSigWords, c->stream));
    ELOC_HIP(c, launch_table_insert(tk, c->khash.as<uint64_t>(), n, c->kslots.p, c->kstash.as<Stash>(), c->S.table,
                                    c->err_prep.as<uint32_t>(), c->stream));
    ELOC_HIP(c, launch_sample_verify(c->H.W, c->H.narrow, c->S, c->sig.as<uint64_t>(), c->err_prep.as<uint32_t>(),
                                     c->stream));
    ELOC_HIP(c, launch_sample_params(c->sig.as<uint64_t>(), c->rad.as<unsigned long long>(), c->H.n_qubits,
                                     c->sparams.as<SampleParams>(), c->stream));
    return ELOC_OK;
}

int read_err(eloc_ctx c, DevBuf& word) {
    hipError_t e = hipMemcpyAsync(c->err_host, word.p, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read error word");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    return static_cast<int>(*c->err_host);
}

int map_err(eloc_ctx c, uint32_t bits) {
    if (bits & kErrBits) return fail(c, ELOC_EINVAL, "a sample key has bits set at or above n_qubits");
    if (bits & kErrDup) return fail(c, ELOC_EDUP, "duplicate keys in the sample batch");
    if (bits & kErrBits) return fail(c, ELOC_EINVAL, "a sample key has bits set at or above n_qubits");
    if (bits & kErrWeights) return fail(c, ELOC_EINVAL, "weights must be finite, >= 0, with a positive sum");
    if (bits & kErrRange)
        return fail(c, ELOC_ERANGE, "log-amplitudes not finite, or Re log psi spread above 60 (FP32 form) or 700 (FP64 form)");
    if (bits & kErrIndex) return fail(c, ELOC_EINVAL, "pair index outside the sample batch");
    if (bits & kErrCapacity) return fail(c, ELOC_ECAPACITY, "an output buffer of the last call was too small");
    return ELOC_OK;
}

// Synchronous verdict on the current samples (the errors eloc_set_samples
// latched on the device).  A membership table whose cuckoo insertion did not
// settle (which also fails the key's own lookup, so it reads as a duplicate)
// is rebuilt here with new salts; *rebuilt tells the caller that work
// enqueued before this call saw the broken table.
int samples_verdict(eloc_ctx c, bool* rebuilt) {
    if (rebuilt) *rebuilt = false;
    int bits = read_err(c, c->err_prep);
    if (bits < 0) return bits;
    for (int attempt = 0; (bits & kErrTable) && !(bits & kErrBits); ++attempt) {
        if (attempt == 8) return fail(c, ELOC_EHIP, "membership table could not be built");
        ELOC_HIP(c, hipMemsetAsync(c->err_prep.p, 0, sizeof(uint32_t), c->stream));
        const int rc = build_sample_table(c);
        if (rc) return rc;
        bits = read_err(c, c->err_prep);
        if (bits < 0) return bits;
        if (rebuilt) *rebuilt = true;
    }
    return map_err(c, static_cast<uint32_t>(bits));
}

// Fill a cuckoo table with keys 0..n-1 (hashes `hash`); a new salt is drawn
// if an insertion does not settle.
int build_table(eloc_ctx c, int tk, const uint64_t* hash, int64_t n, void* slots, Stash* stash, uint64_t cap,
                Table* out) {
    for (int attempt = 0; attempt < 8; ++attempt) {
        const uint64_t salt = splitmix64(c->salt_state);
        Table T = make_table(slots, stash, cap, n, salt);
        ELOC_HIP(c, hipMemsetAsync(slots, 0, slot_bytes(tk) * cap, c->stream));
        ELOC_HIP(c, hipMemsetAsync(stash, 0, sizeof(Stash), c->stream));
        ELOC_HIP(c, hipMemsetAsync(c->err_prep.p, 0, sizeof(uint32_t), c->stream));
        ELOC_HIP(c, launch_table_insert(tk, hash, n, slots, stash, T, c->err_prep.as<uint32_t>(), c->stream));
        const int bits = read_err(c, c->err_prep);
        if (bits < 0) return bits;
        if (!(static_cast<uint32_t>(bits) & kErrTable)) {
            *out = T;
            return ELOC_OK;
        }
    }
    return fail(c, ELOC_EHIP, "membership table could not be built");
}

template <int W>
int ingest(eloc_ctx c, int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
           const uint64_t* yz) {
    HostHam<W> hh;
    const std::string why = build_host_ham<W>(c->R, n_terms, coeff, xy, yz, hh);
    if (!why.empty()) return fail(c, ELOC_EINVAL, why);
    const int64_t G = hh.G;
    const std::vector<GroupRec<W>>& groups = hh.groups;
    const std::vector<TermRec<W>>& terms = hh.terms;
    const std::vector<TermRecF<W>>& terms_f = hh.terms_f;
    const std::vector<uint64_t>& ghash = hh.ghash;
    const std::vector<uint64_t>& gkeys = hh.gkeys;
    const std::vector<int32_t>& order = hh.order;
    const std::vector<uint64_t>& xsorted = hh.xsorted;
    const int maxpop = hh.maxpop, diag = hh.diag;
    // the sorted XY masks and their group ids; LoopOverTrie's chunk trees
    // over them are built at its first use on a sample set (their size
    // depends on the number of rows)
    ELOC_HIP(c, c->xyt_keys.ensure(sizeof(uint64_t) * G * W));
    ELOC_HIP(c, c->xyt_gid.ensure(sizeof(int32_t) * G));
    ELOC_HIP(c, hipMemcpy(c->xyt_keys.p, xsorted.data(), sizeof(uint64_t) * G * W, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->xyt_gid.p, order.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice));
    ELOC_HIP(c, c->groups.ensure(sizeof(GroupRec<W>) * G));
    ELOC_HIP(c, c->terms.ensure(sizeof(TermRec<W>) * n_terms));
    ELOC_HIP(c, c->terms_f.ensure(sizeof(TermRecF<W>) * n_terms));
    ELOC_HIP(c, c->term_src.ensure(sizeof(int32_t) * n_terms));
    ELOC_HIP(c, c->term_ny.ensure(sizeof(uint8_t) * n_terms));
    ELOC_HIP(c, c->ghash.ensure(sizeof(uint64_t) * G));
    ELOC_HIP(c, c->gkeys.ensure(sizeof(uint64_t) * G * W));
    const uint64_t cap = table_capacity(G);
    // narrow keys (one 32-bit word) also carry a run's real and imaginary
    // lengths in 16 bits each through the hit queue
    const bool narrow = n_qubits <= 32 && hh.maxpart < kNarrowMaxPart;
    const int tk = table_kind(W, narrow);
    ELOC_HIP(c, c->gslots.ensure(slot_bytes(tk) * cap));
    ELOC_HIP(c, hipMemcpy(c->groups.p, groups.data(), sizeof(GroupRec<W>) * G, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->terms.p, terms.data(), sizeof(TermRec<W>) * n_terms, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->terms_f.p, terms_f.data(), sizeof(TermRecF<W>) * n_terms, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->term_src.p, hh.term_src.data(), sizeof(int32_t) * n_terms, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->term_ny.p, hh.term_ny.data(), sizeof(uint8_t) * n_terms, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->ghash.p, ghash.data(), sizeof(uint64_t) * G, hipMemcpyHostToDevice));
    ELOC_HIP(c, hipMemcpy(c->gkeys.p, gkeys.data(), sizeof(uint64_t) * G * W, hipMemcpyHostToDevice));
    // the XY masks in spin-split form, for the LoopOverTerms prefilter
    std::vector<uint64_t> gsplit(gkeys.size());
    for (size_t i = 0; i < gkeys.size(); ++i) gsplit[i] = spin_split(gkeys[i]);
    ELOC_HIP(c, c->gsplit.ensure(sizeof(uint64_t) * G * W));
    ELOC_HIP(c, hipMemcpy(c->gsplit.p, gsplit.data(), sizeof(uint64_t) * G * W, hipMemcpyHostToDevice));
    // the group records bucketed by the partition of their hash (stable)
    {
        std::vector<GroupRec<W>> gb;
        std::vector<uint64_t> hb, sb;
        std::vector<int32_t> ib;
        ib.reserve(static_cast<size_t>(G));
        gb.reserve(static_cast<size_t>(G));
        hb.reserve(static_cast<size_t>(G));
        sb.reserve(static_cast<size_t>(G * W));
        int bucket[kMaxParts + 1] = {};
        // a context tuned to partition every table partitions small ones by
        // runs of 32 slots, else by blocks of 64K slots
        c->H.part.shift = c->tune_part > 0 ? kPartShiftSmall : kPartShiftLarge;
        for (int b = 0; b < kMaxParts; ++b) {
            bucket[b] = static_cast<int>(gb.size());
            for (int64_t g = 0; g < G; ++g)
                if (rev_bits(hash_part(ghash[static_cast<size_t>(g)], c->H.part.shift, kMaxPartBits), kMaxPartBits) ==
                    b) {
                    gb.push_back(groups[static_cast<size_t>(g)]);
                    hb.push_back(ghash[static_cast<size_t>(g)]);
                    ib.push_back(static_cast<int32_t>(g));
                    for (int w = 0; w < W; ++w) sb.push_back(gsplit[static_cast<size_t>(g * W + w)]);
                }
        }
        bucket[kMaxParts] = static_cast<int>(G);
        ELOC_HIP(c, c->groups_b.ensure(sizeof(GroupRec<W>) * G));
        ELOC_HIP(c, c->ghash_b.ensure(sizeof(uint64_t) * G));
        ELOC_HIP(c, hipMemcpy(c->groups_b.p, gb.data(), sizeof(GroupRec<W>) * G, hipMemcpyHostToDevice));
        ELOC_HIP(c, hipMemcpy(c->ghash_b.p, hb.data(), sizeof(uint64_t) * G, hipMemcpyHostToDevice));
        ELOC_HIP(c, c->gid_b.ensure(sizeof(int32_t) * G));
        ELOC_HIP(c, hipMemcpy(c->gid_b.p, ib.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice));
        ELOC_HIP(c, c->gsplit_b.ensure(sizeof(uint64_t) * G * W));
        ELOC_HIP(c, hipMemcpy(c->gsplit_b.p, sb.data(), sizeof(uint64_t) * G * W, hipMemcpyHostToDevice));
        for (int b = 0; b <= kMaxParts; ++b) c->H.part.bucket[b] = bucket[b];
        ELOC_HIP(c, c->gbucket.ensure(sizeof(int32_t) * (kMaxParts + 1)));
        ELOC_HIP(c, hipMemcpy(c->gbucket.p, bucket, sizeof(int32_t) * (kMaxParts + 1), hipMemcpyHostToDevice));
    }
    ELOC_HIP(c, c->gstash.ensure(sizeof(Stash)));
    Table T;
    int rc = build_table(c, tk, c->ghash.as<uint64_t>(), G, c->gslots.p, c->gstash.as<Stash>(), cap, &T);
    if (rc) return rc;

    HamDev H;
    H.n_qubits = n_qubits;
    H.W = W;
    H.narrow = narrow;
    H.n_terms = n_terms;
    H.n_groups = G;
    H.maxpop = maxpop;
    H.diag_group = diag;
    H.groups = c->groups.p;
    H.terms = c->terms.p;
    H.terms_f = c->terms_f.p;
    H.term_src = c->term_src.as<int32_t>();
    H.term_ny = c->term_ny.as<uint8_t>();
    H.group_hash = c->ghash.as<uint64_t>();
    H.group_keys = c->gkeys.as<uint64_t>();
    H.group_split = c->gsplit.as<uint64_t>();
    H.group_table = T;
    H.part.groups = c->groups_b.p;
    H.part.shift = c->H.part.shift;
    H.part.ghash = c->ghash_b.as<uint64_t>();
    H.part.gsplit = c->gsplit_b.as<uint64_t>();
    H.part.gid = c->gid_b.as<int32_t>();
    for (int b = 0; b <= kMaxParts; ++b) H.part.bucket[b] = c->H.part.bucket[b];
    H.part.bucket_dev = c->gbucket.as<int32_t>();
    H.xyt.keys = c->xyt_keys.as<uint64_t>();
    H.xyt.gid = c->xyt_gid.as<int32_t>();
    H.xyt.nodes = nullptr;   // chunk trees not built yet
    H.xyt.nkeys = nullptr;
    H.xyt.chunk = 0;
    H.xyt.chunks = 0;
    c->H = H;
    c->ham_set = true;
    return ELOC_OK;
}

hipEvent_t pool_event(eloc_ctx c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records a start event for `stage` when profiling; returns the mark index or -1.
int prof_begin(eloc_ctx c, int stage) {
    if (!c->prof) return -1;
    hipEvent_t a = pool_event(c), b = pool_event(c);
    if (!a || !b) return -1;
    if (hipEventRecord(a, c->stream) != hipSuccess) return -1;
    c->marks.push_back({stage, a, b});
    return static_cast<int>(c->marks.size()) - 1;
}

void prof_end(eloc_ctx c, int mark) {
    if (mark < 0) return;
    (void)hipEventRecord(c->marks[static_cast<size_t>(mark)].b, c->stream);
}

int check_ready(eloc_ctx c) {
    if (!c) return ELOC_EINVAL;
    if (!c->ham_set) return fail(c, ELOC_ESTATE, "no Hamiltonian set");
    if (!c->samples_set) return fail(c, ELOC_ESTATE, "no samples set");
    // U's Bloom filter is built only when the tuning asks for it
    if (c->tune_bloom && c->bloom_words && !c->bloom_built) {
        ELOC_HIP(c, c->bloom.ensure(sizeof(uint32_t) * c->bloom_words));
        ELOC_HIP(c, hipMemsetAsync(c->bloom.p, 0, sizeof(uint32_t) * c->bloom_words, c->stream));
        ELOC_HIP(c, launch_bloom_build(c->khash.as<uint64_t>(), c->S.n, c->bloom.as<uint32_t>(), c->bloom_words,
                                       c->stream));
        c->bloom_built = true;
    }
    return ELOC_OK;
}

// Sorted copy of U with its radix tree, built on first use by LoopOverTrie
// after every eloc_set_samples.
// XY masks per chunk tree of LoopOverTrie for M rows: about 2^25 (row,
// chunk) walks (measured: 2^16 rows fastest with about 128 chunks, 2^20
// rows with 32: 382 ms against 425 with 128 and 406 with 16), at least 64
// masks a chunk and at most what the walk's 16-bit node codes allow; or the
// tuned size.
int64_t trie_chunk_for(const eloc_ctx c, int64_t M) {
    const int64_t G = c->H.n_groups;
    if (c->tune_trie_chunk > 0) return std::max<int64_t>(2, std::min<int64_t>(c->tune_trie_chunk, std::max<int64_t>(G, 2)));
    const int64_t chunks = std::max<int64_t>(1, ((int64_t(1) << 25) + M - 1) / std::max<int64_t>(M, 1));
    int64_t chunk = (G + chunks - 1) / chunks;
    chunk = std::max<int64_t>(chunk, std::min<int64_t>(G, 64));
    return std::max<int64_t>(2, std::min<int64_t>(chunk, 32767));
}

// The XY chunk trees for chunks of `chunk` masks (synchronous with respect
// to the stream: later work on it sees them).
int build_xy_trie(eloc_ctx c, int64_t chunk) {
    const int64_t G = c->H.n_groups;
    const int W = c->H.W;
    const int64_t chunks = (G + chunk - 1) / chunk;
    ELOC_HIP(c, c->xyt_nodes.ensure(sizeof(TNode) * std::max<int64_t>(1, chunks * (chunk - 1))));
    ELOC_HIP(c, c->xyt_nkeys.ensure(sizeof(uint64_t) * W * std::max<int64_t>(1, chunks * (chunk - 1))));
    ELOC_HIP(c, launch_trie_build(W, c->xyt_keys.as<uint64_t>(), G, chunk, c->xyt_nodes.as<TNode>(),
                                  c->xyt_nkeys.as<uint64_t>(), c->stream));
    c->H.xyt.nodes = c->xyt_nodes.as<TNode>();
    c->H.xyt.nkeys = c->xyt_nkeys.as<uint64_t>();
    c->H.xyt.chunk = static_cast<int>(chunk);
    c->H.xyt.chunks = static_cast<int>(chunks);
    return ELOC_OK;
}

int ensure_utrie(eloc_ctx c) {
    if (c->ut_valid) return ELOC_OK;
    const int64_t M = c->S.n;
    const int W = c->H.W;
    {
        const int64_t chunk = trie_chunk_for(c, M);
        if (chunk != c->H.xyt.chunk) {
            const int rc = build_xy_trie(c, chunk);
            if (rc) return rc;
        }
    }
    const int64_t tiles = radix_tiles(M);
    ELOC_HIP(c, c->ut_keys.ensure(sizeof(uint64_t) * M * W));
    ELOC_HIP(c, c->ut_perm.ensure(sizeof(int32_t) * M));
    ELOC_HIP(c, c->ut_nodes.ensure(sizeof(TNode) * std::max<int64_t>(1, M - 1)));
    ELOC_HIP(c, c->ut_nkeys.ensure(sizeof(uint64_t) * W * std::max<int64_t>(1, M - 1)));
    ELOC_HIP(c, c->s_key.ensure(sizeof(uint64_t) * M));
    ELOC_HIP(c, c->s_key2.ensure(sizeof(uint64_t) * M));
    ELOC_HIP(c, c->s_val.ensure(sizeof(uint32_t) * M));
    ELOC_HIP(c, c->s_val2.ensure(sizeof(uint32_t) * M));
    ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
    ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
    ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * scan_scratch_len(256 * tiles)));
    SortScratch ss{c->s_key.as<uint64_t>(), c->s_val.as<uint32_t>(), c->s_key2.as<uint64_t>(),
                   c->s_val2.as<uint32_t>(), c->hist.as<uint32_t>(), c->hist_off.as<int64_t>(),
                   c->hist_scratch.as<int64_t>()};
    const int pm = prof_begin(c, ELOC_STAGE_SAMPLES);
    ELOC_HIP(c, launch_sort_keys(W, c->H.n_qubits, c->keys.as<uint64_t>(), M, ss, c->ut_keys.as<uint64_t>(),
                                 c->ut_perm.as<int32_t>(), c->stream));
    ELOC_HIP(c, launch_trie_build(W, c->ut_keys.as<uint64_t>(), M, M, c->ut_nodes.as<TNode>(),
                                  c->ut_nkeys.as<uint64_t>(), c->stream));
    prof_end(c, pm);
    c->S.ut.keys = c->ut_keys.as<uint64_t>();
    c->S.ut.perm = c->ut_perm.as<int32_t>();
    c->S.ut.nodes = c->ut_nodes.as<TNode>();
    c->S.ut.nkeys = c->ut_nkeys.as<uint64_t>();
    c->ut_valid = true;
    return ELOC_OK;
}

int prepare_variant(eloc_ctx c, int variant) {
    return variant == ELOC_TRIE ? ensure_utrie(c) : ELOC_OK;
}

int amp_prep(eloc_ctx c, const eloc_c64* logpsi, bool fp32) {
    const int64_t M = c->S.n;
    ELOC_HIP(c, c->a.ensure(sizeof(double2) * M));
    ELOC_HIP(c, c->b.ensure(sizeof(double2) * M));
    ELOC_HIP(c, c->af.ensure(sizeof(float4) * (fp32 ? M : 1)));
    ELOC_HIP(c, c->bf.ensure(sizeof(float4) * (fp32 ? M : 1)));
    ELOC_HIP(c, c->shift.ensure(sizeof(double) * 2));
    ELOC_HIP(c, c->amp_scratch.ensure(sizeof(double) * amp_scratch_len()));
    const int pm = prof_begin(c, ELOC_STAGE_AMPLITUDES);
    ELOC_HIP(c, launch_amp_prep(reinterpret_cast<const double2*>(logpsi), M, fp32, c->a.as<double2>(),
                                c->b.as<double2>(), c->af.as<float4>(), c->bf.as<float4>(),
                                c->shift.as<double>(), c->amp_scratch.as<double>(), c->err_run.as<uint32_t>(),
                                c->stream));
    prof_end(c, pm);
    return ELOC_OK;
}

// The row sums of the forward (vec = a) or adjoint (vec = v) pass into
// c->partial: the fused pair kernel for a variant, or one pass over the
// stored pair list (one partial per row).
int row_sums(eloc_ctx c, bool adjoint, int variant, int precision, const double2* vec, const float4* vecf, Plan* plan) {
    const int64_t M = c->S.n;
    const bool fp32 = precision == ELOC_FP32C;
    const Plan P = variant == ELOC_STORED ? Plan{} : make_plan(c, variant, -1, true);
    ELOC_HIP(c, c->partial.ensure((fp32 ? sizeof(float4) : sizeof(double2)) * P.chunks * M));
    const int pm = prof_begin(c, adjoint ? ELOC_STAGE_ADJOINT_PAIRS : ELOC_STAGE_PAIRS);
    if (variant == ELOC_STORED) {
        const void* v = fp32 ? static_cast<const void*>(vecf) : static_cast<const void*>(vec);
        ELOC_HIP(c, launch_spmv(adjoint, precision, M, c->st_rowptr.as<int64_t>(), c->st_col.as<int32_t>(),
                                c->st_h.as<double2>(), v, c->partial.p, c->stream));
    } else {
        ELOC_HIP(c, launch_pairs(adjoint, variant, precision, c->H, c->S, P, vec, vecf, c->partial.p, c->stream));
    }
    prof_end(c, pm);
    *plan = P;
    return ELOC_OK;
}

// Variant checks shared by the forward and adjoint entry points.
int forward_variant(eloc_ctx c, int* variant) {
    if (*variant == ELOC_STORED) {
        if (!c->st_valid) return fail(c, ELOC_ESTATE, "no stored pair list for these samples (eloc_store_pairs)");
        return ELOC_OK;
    }
    if (!valid_variant(*variant)) return fail(c, ELOC_EINVAL, "unknown or unavailable variant");
    *variant = resolve_variant(c, *variant);
    return prepare_variant(c, *variant);
}

int count_into_offsets(eloc_ctx c, int variant, const Plan& P, int64_t* total) {
    const int rc = samples_verdict(c, nullptr);   // synchronising anyway
    if (rc) return rc;
    const int64_t n = c->S.n * P.chunks;
    ELOC_HIP(c, c->counts.ensure(sizeof(int32_t) * n));
    ELOC_HIP(c, c->offsets.ensure(sizeof(int64_t) * (n + 1)));
    ELOC_HIP(c, c->scan_scratch.ensure(sizeof(int64_t) * scan_scratch_len(n)));
    // the partitioned count skips its writes while U is invalid
    if (P.part) ELOC_HIP(c, hipMemsetAsync(c->counts.p, 0, sizeof(int32_t) * n, c->stream));
    ELOC_HIP(c, launch_pairs_count(variant, c->H, c->S, P, c->counts.as<int32_t>(), c->stream));
    ELOC_HIP(c, launch_scan_i32(c->counts.as<int32_t>(), n, c->offsets.as<int64_t>(),
                                c->scan_scratch.as<int64_t>(), c->stream));
    int64_t t = 0;
    ELOC_HIP(c, hipMemcpyAsync(&t, c->offsets.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    *total = t;
    return ELOC_OK;
}

}  // namespace

// ===========================================================================
// exported
// ===========================================================================
extern "C" {

int eloc_create(eloc_ctx* out, int device, void* hip_stream) {
    if (!out) return ELOC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ELOC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ELOC_EHIP;
    eloc_ctx c = new eloc_ctx_s();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    make_hash_words(c->R);
    if (c->R_dev.ensure(sizeof(c->R)) != hipSuccess ||
        hipMemcpy(c->R_dev.p, c->R, sizeof(c->R), hipMemcpyHostToDevice) != hipSuccess ||
        c->err_run.ensure(sizeof(uint32_t)) != hipSuccess || c->err_prep.ensure(sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->err_run.p, 0, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->err_prep.p, 0, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->err_host), sizeof(uint32_t) * 4, hipHostMallocDefault) != hipSuccess ||
        noalloc_workspace(device, &c->ws) != hipSuccess) {
        eloc_destroy(c);
        return ELOC_EHIP;
    }
    *out = c;
    return ELOC_OK;
}

void eloc_destroy(eloc_ctx c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    DevBuf* bufs[] = {&c->R_dev, &c->groups, &c->terms, &c->terms_f, &c->term_src, &c->term_ny, &c->pe_cnt, &c->pe_grp, &c->ghash, &c->gkeys, &c->gslots,
                      &c->keys, &c->khash, &c->kslots, &c->sig, &c->bitcounts, &c->rad, &c->sparams, &c->bloom, &c->a, &c->b, &c->af, &c->bf, &c->v, &c->vf,
                      &c->shift, &c->amp_scratch, &c->partial, &c->energy_scratch, &c->err_run, &c->err_prep,
                      &c->counts, &c->offsets, &c->scan_scratch, &c->pkey, &c->pval, &c->pkey2, &c->pval2,
                      &c->hist, &c->hist_off, &c->hist_scratch, &c->gstash, &c->kstash, &c->xyt_keys, &c->xyt_gid, &c->xyt_nodes, &c->xyt_nkeys,
                      &c->ut_keys, &c->ut_perm, &c->ut_nodes, &c->ut_nkeys, &c->s_key, &c->s_val, &c->s_key2, &c->s_val2,
                      &c->m_raw, &c->m_sorted, &c->m_perm, &c->m_flags, &c->m_pos, &c->m_count, &c->x_keys, &c->x_hash, &c->x_slots,
                      &c->x_stash, &c->x_sig, &c->x_bitcounts, &c->x_rad, &c->x_params, &c->x_err, &c->x_logpsi,
                      &c->x_a, &c->x_b, &c->x_af, &c->x_bf, &c->x_shift, &c->x_part_perm, &c->x_part_class, &c->x_part_tile, &c->st_rowptr, &c->st_col, &c->st_h,
                      &c->sr_w, &c->sr_mean, &c->sr_part, &c->sr_T, &c->sr_L, &c->sr_y,
                      &c->groups_b, &c->ghash_b, &c->gsplit_b, &c->gid_b, &c->gsplit, &c->gbucket, &c->part_perm, &c->part_class, &c->part_tile,
                      &c->ar_keys[0], &c->ar_keys[1], &c->ar_l[0], &c->ar_l[1], &c->ar_T[0], &c->ar_T[1],
                      &c->ar_cl, &c->ar_cT, &c->ar_ck, &c->ar_ci, &c->ar_ck2, &c->ar_ci2, &c->ar_cnt,
                      &c->ar_hist, &c->ar_sel, &c->ar_keep, &c->ar_off};
    for (DevBuf* b : bufs) b->release();
    for (auto& m : c->marks) {
        c->ev_pool.push_back(m.a);
        c->ev_pool.push_back(m.b);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->err_host) (void)hipHostFree(c->err_host);
    delete c;
}

const char* eloc_last_error(eloc_ctx c) { return c ? c->err.c_str() : "null context"; }

int eloc_set_stream(eloc_ctx c, void* hip_stream) {
    if (!c) return ELOC_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return ELOC_OK;
}

int eloc_set_hamiltonian(eloc_ctx c, int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                         const uint64_t* yz) {
    if (!c) return ELOC_EINVAL;
    if (n_qubits < 1 || n_qubits > 128) return fail(c, ELOC_EINVAL, "n_qubits must be in 1..128");
    if (n_terms < 1 || !coeff || !xy || !yz) return fail(c, ELOC_EINVAL, "empty Hamiltonian or null pointer");
    const int W = (n_qubits + 63) / 64;
    for (int64_t l = 0; l < n_terms; ++l) {
        for (int w = 0; w < W; ++w) {
            const int valid = n_qubits - 64 * w;
            if (valid < 64) {
                const uint64_t allowed = (1ull << valid) - 1ull;
                if ((xy[l * W + w] | yz[l * W + w]) & ~allowed)
                    return fail(c, ELOC_EINVAL, "a term mask has bits set at or above n_qubits");
            }
        }
        if (!std::isfinite(coeff[l])) return fail(c, ELOC_EINVAL, "non-finite coefficient");
    }
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, ELOC_EHIP, "hipSetDevice");
    c->ham_set = false;
    c->samples_set = false;    // sample tables depend on the qubit count
    c->miss_valid = false;
    c->st_valid = false;
    return W == 1 ? ingest<1>(c, n_qubits, n_terms, coeff, xy, yz) : ingest<2>(c, n_qubits, n_terms, coeff, xy, yz);
}

int eloc_hamiltonian_info(eloc_ctx c, int64_t* n_groups, int64_t* n_terms, int* n_qubits) {
    if (!c) return ELOC_EINVAL;
    if (!c->ham_set) return fail(c, ELOC_ESTATE, "no Hamiltonian set");
    if (n_groups) *n_groups = c->H.n_groups;
    if (n_terms) *n_terms = c->H.n_terms;
    if (n_qubits) *n_qubits = c->H.n_qubits;
    return ELOC_OK;
}

int eloc_samples_info(eloc_ctx c, int64_t* n_unique, int64_t* table_slots, int* table_stash) {
    if (!c) return ELOC_EINVAL;
    if (!c->samples_set) return fail(c, ELOC_ESTATE, "no samples set");
    if (n_unique) *n_unique = c->S.n;
    if (table_slots) *table_slots = static_cast<int64_t>(c->kslots_n);
    if (table_stash) {
        // the stash count is the first word of the stash
        const int bits = read_err(c, c->kstash);
        if (bits < 0) return bits;
        *table_stash = bits;
    }
    return ELOC_OK;
}

int eloc_set_samples(eloc_ctx c, int64_t n_unique, const uint64_t* keys_dev) {
    if (!c) return ELOC_EINVAL;
    if (!c->ham_set) return fail(c, ELOC_ESTATE, "set the Hamiltonian first");
    if (n_unique < 1 || n_unique >= (int64_t(1) << 24) || !keys_dev)
        return fail(c, ELOC_EINVAL, "n_unique must be in 1..2^24-1 with a key pointer");
    const int W = c->H.W;
    c->samples_set = false;
    c->miss_valid = false;
    ELOC_HIP(c, c->keys.ensure(sizeof(uint64_t) * n_unique * W));
    ELOC_HIP(c, c->khash.ensure(sizeof(uint64_t) * n_unique));
    const uint64_t cap = table_capacity(n_unique);
    const int tk = table_kind(W, c->H.narrow);
    ELOC_HIP(c, c->kslots.ensure(slot_bytes(tk) * cap));
    ELOC_HIP(c, c->kstash.ensure(sizeof(Stash)));
    ELOC_HIP(c, c->sig.ensure(sizeof(uint64_t) * kSigWords));
    ELOC_HIP(c, c->bitcounts.ensure(sizeof(uint32_t) * 64 * W));
    ELOC_HIP(c, c->rad.ensure(sizeof(unsigned long long) * 3));
    ELOC_HIP(c, c->sparams.ensure(sizeof(SampleParams)));
    const int pm = prof_begin(c, ELOC_STAGE_SAMPLES);
    ELOC_HIP(c, hipMemcpyAsync(c->keys.p, keys_dev, sizeof(uint64_t) * n_unique * W, hipMemcpyDeviceToDevice,
                               c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->err_prep.p, 0, sizeof(uint32_t), c->stream));
    // errors of calls on the previous samples are not carried over
    ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->bitcounts.p, 0, sizeof(uint32_t) * 64 * W, c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->rad.p, 0, sizeof(unsigned long long) * 3, c->stream));
    ELOC_HIP(c, launch_sample_hash(W, c->keys.as<uint64_t>(), n_unique, c->R_dev.as<uint64_t>(), c->H.n_qubits,
                                   c->khash.as<uint64_t>(), c->bitcounts.as<uint32_t>(), c->err_prep.as<uint32_t>(),
                                   c->stream));
    ELOC_HIP(c, launch_sample_radius(W, c->keys.as<uint64_t>(), n_unique, c->bitcounts.as<uint32_t>(),
                                     c->rad.as<unsigned long long>(), c->stream));
    // Bloom filter of U: about 4 bits per key, at most 32 KB (it is staged in
    // LDS); none for batches too large for it to reject much
    c->bloom_words = n_unique <= (int64_t(1) << 17)
                         ? static_cast<uint32_t>(std::min<uint64_t>(kBloomMaxWords,
                                                                    std::max<uint64_t>(256, pow2_at_least(n_unique / 8))))
                         : 0u;
    c->bloom_built = false;
    SampleDev S;
    S.n = n_unique;
    S.keys = c->keys.as<uint64_t>();
    S.hash = c->khash.as<uint64_t>();
    S.sig = c->sig.as<uint64_t>();
    S.params = c->sparams.as<SampleParams>();
    S.prep_err = c->err_prep.as<uint32_t>();
    c->S = S;
    c->kslots_n = cap;
    c->part_bits = part_bits_for(c, slot_bytes(tk) * cap, cap);
    // table insert, verification and prefilter parameters, all on the
    // device: errors (duplicates, bits >= N, a table that did not settle)
    // stay latched in the preparation error word until a synchronising call
    const int rc = build_sample_table(c);
    if (rc) return rc;
    c->part_ok = false;
    c->S.part.bits = 0;
    if (c->part_bits > 0) {
        const int64_t tiles = radix_tiles(n_unique);
        ELOC_HIP(c, c->s_key.ensure(sizeof(uint64_t) * n_unique));
        ELOC_HIP(c, c->s_key2.ensure(sizeof(uint64_t) * n_unique));
        ELOC_HIP(c, c->s_val.ensure(sizeof(uint32_t) * n_unique));
        ELOC_HIP(c, c->s_val2.ensure(sizeof(uint32_t) * n_unique));
        ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
        ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
        ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * scan_scratch_len(256 * tiles)));
        ELOC_HIP(c, c->part_perm.ensure(sizeof(int32_t) * n_unique));
        ELOC_HIP(c, c->part_class.ensure(sizeof(int64_t) * (kMaxParts + 1)));
        ELOC_HIP(c, c->part_tile.ensure(sizeof(int64_t) * (kMaxParts + 1)));
        ELOC_HIP(c, launch_row_classes(c->khash.as<uint64_t>(), n_unique, c->H.part.shift, c->part_bits,
                                       c->s_key.as<uint64_t>(),
                                       c->s_val.as<uint32_t>(),
                                       c->s_key2.as<uint64_t>(), c->s_val2.as<uint32_t>(), c->hist.as<uint32_t>(),
                                       c->hist_off.as<int64_t>(), c->hist_scratch.as<int64_t>(),
                                       c->part_perm.as<int32_t>(), c->part_class.as<int64_t>(),
                                       c->part_tile.as<int64_t>(), c->stream));
        c->S.part.row_perm = c->part_perm.as<int32_t>();
        c->S.part.class_off = c->part_class.as<int64_t>();
        c->S.part.tile_off = c->part_tile.as<int64_t>();
        c->S.part.bits = c->part_bits;
        c->part_ok = true;
    }
    prof_end(c, pm);
    c->ut_valid = false;
    c->st_valid = false;
    c->samples_set = true;
    return ELOC_OK;
}

int eloc_local_energy(eloc_ctx c, int variant, int precision, const eloc_c64* logpsi_dev,
                      const double* weights_dev, eloc_c64* eloc_dev, double* stats_dev) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (precision != ELOC_FP64 && precision != ELOC_FP32C) return fail(c, ELOC_EINVAL, "unknown precision");
    if (!logpsi_dev || !eloc_dev || !stats_dev) return fail(c, ELOC_EINVAL, "null pointer");
    rc = forward_variant(c, &variant);
    if (rc) return rc;
    const int64_t M = c->S.n;
    const bool fp32 = precision == ELOC_FP32C;
    ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    rc = amp_prep(c, logpsi_dev, fp32);
    if (rc) return rc;
    Plan P;
    rc = row_sums(c, false, variant, precision, c->a.as<double2>(), c->af.as<float4>(), &P);
    if (rc) return rc;
    int pm = prof_begin(c, ELOC_STAGE_FINISH);
    ELOC_HIP(c, launch_finish(precision, M, P, c->partial.p, c->b.as<double2>(), c->bf.as<float4>(),
                              reinterpret_cast<double2*>(eloc_dev), c->stream));
    prof_end(c, pm);
    ELOC_HIP(c, c->energy_scratch.ensure(sizeof(double) * energy_scratch_len()));
    pm = prof_begin(c, ELOC_STAGE_ENERGY);
    ELOC_HIP(c, launch_energy(reinterpret_cast<const double2*>(eloc_dev), reinterpret_cast<const double2*>(logpsi_dev),
                              weights_dev, c->shift.as<double>(), M, stats_dev, c->energy_scratch.as<double>(),
                              c->err_run.as<uint32_t>(), c->stream));
    prof_end(c, pm);
    return ELOC_OK;
}

int eloc_local_energy_noalloc(eloc_ctx c, int variant, int precision, const eloc_c64* logpsi_dev,
                              const double* weights_dev, eloc_c64* eloc_dev, double* stats_dev) {
    if (!c) return ELOC_EINVAL;
    if (!c->ham_set) return fail(c, ELOC_ESTATE, "no Hamiltonian set");
    if (!c->samples_set) return fail(c, ELOC_ESTATE, "no samples set");
    if (precision != ELOC_FP64 && precision != ELOC_FP32C) return fail(c, ELOC_EINVAL, "unknown precision");
    if (!logpsi_dev || !eloc_dev || !stats_dev) return fail(c, ELOC_EINVAL, "null pointer");
    if (variant == ELOC_TRIE)
        return fail(c, ELOC_EINVAL, "LoopOverTrie builds U's sorted copy on first use, which allocates; "
                                    "use ELOC_TERMS, ELOC_BATCH, ELOC_AUTO or ELOC_STORED");
    if (variant == ELOC_STORED) {
        if (!c->st_valid) return fail(c, ELOC_ESTATE, "no stored pair list for these samples (eloc_store_pairs)");
    } else {
        if (!valid_variant(variant)) return fail(c, ELOC_EINVAL, "unknown variant");
        variant = resolve_variant(c, variant);
    }
    if (!c->ws) return fail(c, ELOC_EHIP, "no fixed workspace on this device");
    const int64_t M = c->S.n;
    const bool fp32 = precision == ELOC_FP32C;
    Plan P = variant == ELOC_STORED ? Plan{} : make_plan(c, variant, -1, true);
    // the partitioned LoopOverTerms keeps one partial sum per partition and
    // row: where that outgrows the workspace, the plain loop serves
    const size_t acc_bytes = fp32 ? sizeof(float4) : sizeof(double2);
    if (P.part && acc_bytes * static_cast<size_t>(P.chunks) * M > kNoAllocBytes / 2)
        P = make_plan(c, variant, -1, false);
    P.bloom_words = 0;   // U's Bloom filter is built on first use (it allocates)
    // workspace layout, every part 256-byte aligned
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t o_a = take(sizeof(double2) * M), o_b = take(sizeof(double2) * M);
    const size_t o_af = take(fp32 ? sizeof(float4) * M : 0), o_bf = take(fp32 ? sizeof(float4) * M : 0);
    const size_t o_shift = take(sizeof(double) * 2);
    const size_t o_amp = take(sizeof(double) * amp_scratch_len());
    const size_t o_part = take(acc_bytes * static_cast<size_t>(P.chunks) * M);
    const size_t o_en = take(sizeof(double) * energy_scratch_len());
    if (off > kNoAllocBytes)
        return fail(c, ELOC_ECAPACITY,
                    "the allocation-free forward pass needs " + std::to_string(off) + " bytes of workspace for " +
                        std::to_string(M) + " samples; the fixed workspace holds " + std::to_string(kNoAllocBytes));
    unsigned char* ws = static_cast<unsigned char*>(c->ws);
    double2* a = reinterpret_cast<double2*>(ws + o_a);
    double2* b = reinterpret_cast<double2*>(ws + o_b);
    float4* af = fp32 ? reinterpret_cast<float4*>(ws + o_af) : nullptr;
    float4* bf = fp32 ? reinterpret_cast<float4*>(ws + o_bf) : nullptr;
    double* shift = reinterpret_cast<double*>(ws + o_shift);
    void* partial = ws + o_part;
    ELOC_HIP(c, launch_fill_u32(c->err_run.as<uint32_t>(), 1, 0u, c->stream));
    ELOC_HIP(c, launch_amp_prep(reinterpret_cast<const double2*>(logpsi_dev), M, fp32, a, b, af, bf, shift,
                                reinterpret_cast<double*>(ws + o_amp), c->err_run.as<uint32_t>(), c->stream));
    if (variant == ELOC_STORED) {
        const void* v = fp32 ? static_cast<const void*>(af) : static_cast<const void*>(a);
        ELOC_HIP(c, launch_spmv(false, precision, M, c->st_rowptr.as<int64_t>(), c->st_col.as<int32_t>(),
                                c->st_h.as<double2>(), v, partial, c->stream));
    } else {
        ELOC_HIP(c, launch_pairs(false, variant, precision, c->H, c->S, P, a, af, partial, c->stream));
    }
    ELOC_HIP(c, launch_finish(precision, M, P, partial, b, bf, reinterpret_cast<double2*>(eloc_dev), c->stream));
    ELOC_HIP(c, launch_energy(reinterpret_cast<const double2*>(eloc_dev), reinterpret_cast<const double2*>(logpsi_dev),
                              weights_dev, shift, M, stats_dev, reinterpret_cast<double*>(ws + o_en),
                              c->err_run.as<uint32_t>(), c->stream));
    return ELOC_OK;
}

int eloc_find_misses(eloc_ctx c, double tol, int64_t capacity, uint64_t* keys_dev, int64_t* n_misses_host) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!n_misses_host) return fail(c, ELOC_EINVAL, "null pointer");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, ELOC_EINVAL, "tol must be finite and >= 0");
    if (capacity < 0) return fail(c, ELOC_EINVAL, "negative capacity");
    rc = samples_verdict(c, nullptr);
    if (rc) return rc;
    const int W = c->H.W;
    int64_t total = c->miss_total, uniq = c->miss_uniq;
    // one-word keys of at most kMissBitmapQubits qubits: the states are
    // marked in a bitmap over the key space, whose set bits are the unique
    // states in ascending order (no list, no sort)
    const bool bitmap = W == 1 && c->H.n_qubits <= kMissBitmapQubits;
    const int64_t nwords = int64_t(1) << std::max(0, c->H.n_qubits - 5);
    if (bitmap && !(c->miss_valid && c->miss_tol == tol)) {
        c->miss_valid = false;
        const Plan P = make_plan(c, ELOC_TERMS);
        ELOC_HIP(c, c->m_raw.ensure(sizeof(uint32_t) * nwords));
        ELOC_HIP(c, c->m_flags.ensure(sizeof(int32_t) * nwords));
        ELOC_HIP(c, c->m_pos.ensure(sizeof(int64_t) * (nwords + 1)));
        ELOC_HIP(c, c->scan_scratch.ensure(sizeof(int64_t) * scan_scratch_len(nwords)));
        uint32_t* bits = static_cast<uint32_t*>(c->m_raw.p);
        ELOC_HIP(c, hipMemsetAsync(bits, 0, sizeof(uint32_t) * nwords, c->stream));
        ELOC_HIP(c, launch_misses_bitmap(c->H, c->S, P.chunks, P.per_chunk, tol, bits, c->stream));
        ELOC_HIP(c, launch_bitmap_counts(bits, nwords, c->m_flags.as<int32_t>(), c->stream));
        ELOC_HIP(c, launch_scan_i32(c->m_flags.as<int32_t>(), nwords, c->m_pos.as<int64_t>(),
                                    c->scan_scratch.as<int64_t>(), c->stream));
        ELOC_HIP(c, hipMemcpyAsync(&uniq, c->m_pos.as<int64_t>() + nwords, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   c->stream));
        ELOC_HIP(c, hipStreamSynchronize(c->stream));
        total = uniq;
    } else if (!(c->miss_valid && c->miss_tol == tol)) {
        c->miss_valid = false;
        const Plan P = make_plan(c, ELOC_TERMS);
        // one append pass into the buffer as it stands; when the states
        // outnumber it, a second pass into one of the counted size
        ELOC_HIP(c, c->m_count.ensure(sizeof(unsigned long long)));
        total = 0;
        for (int pass = 0; pass < 2; ++pass) {
            const int64_t room = static_cast<int64_t>(c->m_raw.p ? c->m_raw.bytes / (sizeof(uint64_t) * W) : 0);
            ELOC_HIP(c, hipMemsetAsync(c->m_count.p, 0, sizeof(unsigned long long), c->stream));
            ELOC_HIP(c, launch_misses(c->H, c->S, P.chunks, P.per_chunk, tol, c->m_count.as<unsigned long long>(),
                                      room, c->m_raw.as<uint64_t>(), c->stream));
            unsigned long long cnt = 0;
            ELOC_HIP(c, hipMemcpyAsync(&cnt, c->m_count.p, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
            ELOC_HIP(c, hipStreamSynchronize(c->stream));
            total = static_cast<int64_t>(cnt);
            if (total >= (int64_t(1) << 31))
                return fail(c, ELOC_ECAPACITY, "more than 2^31 coupled states outside U before deduplication");
            if (total <= room) break;
            if (pass == 1) return fail(c, ELOC_EHIP, "the coupled states outside U changed between two passes");
            ELOC_HIP(c, c->m_raw.ensure(sizeof(uint64_t) * (total + total / 4) * W));
        }
        uniq = 0;
    }
    if (!bitmap && !c->miss_valid && total > 0) {
        // sort (W-word keys, most significant word last) and keep the first of every run
        const int64_t tiles = radix_tiles(total);
        ELOC_HIP(c, c->s_key.ensure(sizeof(uint64_t) * total));
        ELOC_HIP(c, c->s_key2.ensure(sizeof(uint64_t) * total));
        ELOC_HIP(c, c->s_val.ensure(sizeof(uint32_t) * total));
        ELOC_HIP(c, c->s_val2.ensure(sizeof(uint32_t) * total));
        ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
        ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
        ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * scan_scratch_len(256 * tiles)));
        ELOC_HIP(c, c->m_sorted.ensure(sizeof(uint64_t) * total * W));
        ELOC_HIP(c, c->m_perm.ensure(sizeof(int32_t) * total));
        ELOC_HIP(c, c->m_flags.ensure(sizeof(int32_t) * total));
        ELOC_HIP(c, c->m_pos.ensure(sizeof(int64_t) * (total + 1)));
        ELOC_HIP(c, c->scan_scratch.ensure(sizeof(int64_t) * scan_scratch_len(total)));
        SortScratch ss{c->s_key.as<uint64_t>(), c->s_val.as<uint32_t>(), c->s_key2.as<uint64_t>(),
                       c->s_val2.as<uint32_t>(), c->hist.as<uint32_t>(), c->hist_off.as<int64_t>(),
                       c->hist_scratch.as<int64_t>()};
        ELOC_HIP(c, launch_sort_keys(W, c->H.n_qubits, c->m_raw.as<uint64_t>(), total, ss, c->m_sorted.as<uint64_t>(),
                                     c->m_perm.as<int32_t>(), c->stream));
        ELOC_HIP(c, launch_unique_flags(W, c->m_sorted.as<uint64_t>(), total, c->m_flags.as<int32_t>(), c->stream));
        ELOC_HIP(c, launch_scan_i32(c->m_flags.as<int32_t>(), total, c->m_pos.as<int64_t>(),
                                    c->scan_scratch.as<int64_t>(), c->stream));
        ELOC_HIP(c, hipMemcpyAsync(&uniq, c->m_pos.as<int64_t>() + total, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   c->stream));
        ELOC_HIP(c, hipStreamSynchronize(c->stream));
    }
    c->miss_valid = true;
    c->miss_tol = tol;
    c->miss_total = total;
    c->miss_uniq = uniq;
    *n_misses_host = uniq;
    if (uniq > capacity) return fail(c, ELOC_ECAPACITY, "capacity too small for the coupled states outside U");
    if (uniq > 0) {
        if (!keys_dev) return fail(c, ELOC_EINVAL, "null pointer");
        if (bitmap)
            ELOC_HIP(c, launch_bitmap_keys(static_cast<const uint32_t*>(c->m_raw.p), nwords, c->m_pos.as<int64_t>(),
                                           keys_dev, c->stream));
        else
            ELOC_HIP(c, launch_unique_scatter(W, c->m_sorted.as<uint64_t>(), total, c->m_flags.as<int32_t>(),
                                              c->m_pos.as<int64_t>(), keys_dev, c->stream));
    }
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    return ELOC_OK;
}

int eloc_local_energy_full(eloc_ctx c, int precision, const eloc_c64* logpsi_dev, const double* weights_dev,
                           int64_t n_extra, const uint64_t* extra_keys_dev, const eloc_c64* extra_logpsi_dev,
                           eloc_c64* eloc_dev, double* stats_dev) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (precision != ELOC_FP64 && precision != ELOC_FP32C) return fail(c, ELOC_EINVAL, "unknown precision");
    if (!logpsi_dev || !eloc_dev || !stats_dev || n_extra < 0 || (n_extra > 0 && (!extra_keys_dev || !extra_logpsi_dev)))
        return fail(c, ELOC_EINVAL, "null pointer or negative count");
    rc = samples_verdict(c, nullptr);
    if (rc) return rc;
    const int64_t M = c->S.n;
    const int64_t X = M + n_extra;
    if (X >= (int64_t(1) << 24)) return fail(c, ELOC_EINVAL, "U and the extra states must number under 2^24");
    const int W = c->H.W;
    const bool fp32 = precision == ELOC_FP32C;
    const int tk = table_kind(W, c->H.narrow);
    const uint64_t cap = table_capacity(X);
    ELOC_HIP(c, c->x_keys.ensure(sizeof(uint64_t) * X * W));
    ELOC_HIP(c, c->x_hash.ensure(sizeof(uint64_t) * X));
    ELOC_HIP(c, c->x_slots.ensure(slot_bytes(tk) * cap));
    ELOC_HIP(c, c->x_stash.ensure(sizeof(Stash)));
    ELOC_HIP(c, c->x_sig.ensure(sizeof(uint64_t) * kSigWords));
    ELOC_HIP(c, c->x_bitcounts.ensure(sizeof(uint32_t) * 64 * W));
    ELOC_HIP(c, c->x_rad.ensure(sizeof(unsigned long long) * 3));
    ELOC_HIP(c, c->x_params.ensure(sizeof(SampleParams)));
    ELOC_HIP(c, c->x_err.ensure(sizeof(uint32_t)));
    ELOC_HIP(c, c->x_logpsi.ensure(sizeof(double2) * X));
    // X = U's keys and log-amplitudes, then the extra states'
    ELOC_HIP(c, hipMemcpyAsync(c->x_keys.p, c->keys.p, sizeof(uint64_t) * M * W, hipMemcpyDeviceToDevice, c->stream));
    ELOC_HIP(c, hipMemcpyAsync(c->x_logpsi.p, logpsi_dev, sizeof(double2) * M, hipMemcpyDeviceToDevice, c->stream));
    if (n_extra > 0) {
        ELOC_HIP(c, hipMemcpyAsync(c->x_keys.as<uint64_t>() + M * W, extra_keys_dev, sizeof(uint64_t) * n_extra * W,
                                   hipMemcpyDeviceToDevice, c->stream));
        ELOC_HIP(c, hipMemcpyAsync(c->x_logpsi.as<double2>() + M, extra_logpsi_dev, sizeof(double2) * n_extra,
                                   hipMemcpyDeviceToDevice, c->stream));
    }
    ELOC_HIP(c, hipMemsetAsync(c->x_err.p, 0, sizeof(uint32_t), c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->x_bitcounts.p, 0, sizeof(uint32_t) * 64 * W, c->stream));
    ELOC_HIP(c, hipMemsetAsync(c->x_rad.p, 0, sizeof(unsigned long long) * 3, c->stream));
    ELOC_HIP(c, launch_sample_hash(W, c->x_keys.as<uint64_t>(), X, c->R_dev.as<uint64_t>(), c->H.n_qubits,
                                   c->x_hash.as<uint64_t>(), c->x_bitcounts.as<uint32_t>(), c->x_err.as<uint32_t>(),
                                   c->stream));
    ELOC_HIP(c, launch_sample_radius(W, c->x_keys.as<uint64_t>(), X, c->x_bitcounts.as<uint32_t>(),
                                     c->x_rad.as<unsigned long long>(), c->stream));
    SampleDev S;
    S.n = X;
    S.rows = M;
    S.keys = c->x_keys.as<uint64_t>();
    S.hash = c->x_hash.as<uint64_t>();
    S.sig = c->x_sig.as<uint64_t>();
    S.params = c->x_params.as<SampleParams>();
    S.prep_err = c->x_err.as<uint32_t>();
    // membership table of X (a new salt if an insertion does not settle),
    // duplicate and bit checks, prefilter parameters; verdict before use
    // a large table is split into partitions as U's is (the group records are
    // bucketed for the same partition shift at ingest)
    const int xbits = part_bits_for(c, slot_bytes(tk) * cap, cap);
    uint32_t bits = kErrTable;
    for (int attempt = 0; attempt < 8 && (bits & kErrTable) && !(bits & kErrBits); ++attempt) {
        S.table = make_table(c->x_slots.p, c->x_stash.as<Stash>(), cap, X, splitmix64(c->salt_state),
                             c->H.part.shift, xbits);
        ELOC_HIP(c, hipMemsetAsync(c->x_slots.p, 0, slot_bytes(tk) * cap, c->stream));
        ELOC_HIP(c, hipMemsetAsync(c->x_stash.p, 0, sizeof(Stash), c->stream));
        ELOC_HIP(c, hipMemsetAsync(c->x_sig.p, 0, sizeof(uint64_t) * kSigWords, c->stream));
        if (attempt > 0) ELOC_HIP(c, hipMemsetAsync(c->x_err.p, 0, sizeof(uint32_t), c->stream));
        ELOC_HIP(c, launch_table_insert(tk, c->x_hash.as<uint64_t>(), X, c->x_slots.p, c->x_stash.as<Stash>(), S.table,
                                        c->x_err.as<uint32_t>(), c->stream));
        ELOC_HIP(c, launch_sample_verify(W, c->H.narrow, S, c->x_sig.as<uint64_t>(), c->x_err.as<uint32_t>(),
                                         c->stream));
        ELOC_HIP(c, launch_sample_params(c->x_sig.as<uint64_t>(), c->x_rad.as<unsigned long long>(), c->H.n_qubits,
                                         c->x_params.as<SampleParams>(), c->stream));
        const int b = read_err(c, c->x_err);
        if (b < 0) return b;
        bits = static_cast<uint32_t>(b);
    }
    if (bits & kErrBits) return fail(c, ELOC_EINVAL, "an extra state has bits set at or above n_qubits");
    if (bits & kErrTable) return fail(c, ELOC_EHIP, "membership table could not be built");
    if (bits & kErrDup) return fail(c, ELOC_EDUP, "an extra state repeats or is in U");
    // amplitudes over X, LoopOverTerms over U's rows, row combination
    ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    ELOC_HIP(c, c->x_a.ensure(sizeof(double2) * X));
    ELOC_HIP(c, c->x_b.ensure(sizeof(double2) * X));
    ELOC_HIP(c, c->x_af.ensure(sizeof(float4) * (fp32 ? X : 1)));
    ELOC_HIP(c, c->x_bf.ensure(sizeof(float4) * (fp32 ? X : 1)));
    ELOC_HIP(c, c->x_shift.ensure(sizeof(double) * 2));
    ELOC_HIP(c, c->amp_scratch.ensure(sizeof(double) * amp_scratch_len()));
    ELOC_HIP(c, launch_amp_prep(c->x_logpsi.as<double2>(), X, fp32, c->x_a.as<double2>(), c->x_b.as<double2>(),
                                c->x_af.as<float4>(), c->x_bf.as<float4>(), c->x_shift.as<double>(),
                                c->amp_scratch.as<double>(), c->err_run.as<uint32_t>(), c->stream));
    Plan P = make_plan(c, ELOC_TERMS, M);
    P.bloom_words = 0;
    S.part.bits = 0;
    if (xbits > 0) {
        // U's rows (the first M of X) in classes by their hashes' partition
        // field, as eloc_set_samples orders them for U's own table
        const int64_t tiles = radix_tiles(M);
        ELOC_HIP(c, c->s_key.ensure(sizeof(uint64_t) * M));
        ELOC_HIP(c, c->s_key2.ensure(sizeof(uint64_t) * M));
        ELOC_HIP(c, c->s_val.ensure(sizeof(uint32_t) * M));
        ELOC_HIP(c, c->s_val2.ensure(sizeof(uint32_t) * M));
        ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
        ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
        ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * scan_scratch_len(256 * tiles)));
        ELOC_HIP(c, c->x_part_perm.ensure(sizeof(int32_t) * M));
        ELOC_HIP(c, c->x_part_class.ensure(sizeof(int64_t) * (kMaxParts + 1)));
        ELOC_HIP(c, c->x_part_tile.ensure(sizeof(int64_t) * (kMaxParts + 1)));
        ELOC_HIP(c, launch_row_classes(c->x_hash.as<uint64_t>(), M, c->H.part.shift, xbits, c->s_key.as<uint64_t>(),
                                       c->s_val.as<uint32_t>(), c->s_key2.as<uint64_t>(), c->s_val2.as<uint32_t>(),
                                       c->hist.as<uint32_t>(), c->hist_off.as<int64_t>(),
                                       c->hist_scratch.as<int64_t>(), c->x_part_perm.as<int32_t>(),
                                       c->x_part_class.as<int64_t>(), c->x_part_tile.as<int64_t>(), c->stream));
        S.part.row_perm = c->x_part_perm.as<int32_t>();
        S.part.class_off = c->x_part_class.as<int64_t>();
        S.part.tile_off = c->x_part_tile.as<int64_t>();
        S.part.bits = xbits;
        set_part_plan(P, M, xbits);
    }
    ELOC_HIP(c, c->partial.ensure((fp32 ? sizeof(float4) : sizeof(double2)) * P.chunks * M));
    ELOC_HIP(c, launch_pairs(false, ELOC_TERMS, precision, c->H, S, P, c->x_a.as<double2>(), c->x_af.as<float4>(),
                             c->partial.p, c->stream));
    ELOC_HIP(c, launch_finish(precision, M, P, c->partial.p, c->x_b.as<double2>(), c->x_bf.as<float4>(),
                              reinterpret_cast<double2*>(eloc_dev), c->stream));
    // weighted energy over U (its own amplitude shift for the |psi|^2 weights)
    rc = amp_prep(c, logpsi_dev, fp32);
    if (rc) return rc;
    ELOC_HIP(c, c->energy_scratch.ensure(sizeof(double) * energy_scratch_len()));
    ELOC_HIP(c, launch_energy(reinterpret_cast<const double2*>(eloc_dev), reinterpret_cast<const double2*>(logpsi_dev),
                              weights_dev, c->shift.as<double>(), M, stats_dev, c->energy_scratch.as<double>(),
                              c->err_run.as<uint32_t>(), c->stream));
    const int b = read_err(c, c->err_run);
    if (b < 0) return b;
    if (b) ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    return map_err(c, static_cast<uint32_t>(b));
}

int eloc_sr_select(eloc_ctx c, int64_t n, const eloc_c64* logpsi_dev, int n_sr, int32_t* idx_dev) {
    if (!c) return ELOC_EINVAL;
    if (n < 1 || n >= (int64_t(1) << 31) || n_sr < 1 || n_sr > n || !logpsi_dev || !idx_dev)
        return fail(c, ELOC_EINVAL, "need 1 <= n_sr <= n < 2^31 and device pointers");
    const int64_t tiles = radix_tiles(n);
    ELOC_HIP(c, c->s_key.ensure(sizeof(uint64_t) * n));
    ELOC_HIP(c, c->s_key2.ensure(sizeof(uint64_t) * n));
    ELOC_HIP(c, c->s_val.ensure(sizeof(uint32_t) * n));
    ELOC_HIP(c, c->s_val2.ensure(sizeof(uint32_t) * n));
    ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
    ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
    ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * scan_scratch_len(256 * tiles)));
    c->ut_valid = false;   // the sort scratch is shared with U's sorted copy
    ELOC_HIP(c, launch_sr_select(reinterpret_cast<const double2*>(logpsi_dev), n, n_sr, c->s_key.as<uint64_t>(),
                                 c->s_val.as<uint32_t>(), c->s_key2.as<uint64_t>(), c->s_val2.as<uint32_t>(),
                                 c->hist.as<uint32_t>(), c->hist_off.as<int64_t>(), c->hist_scratch.as<int64_t>(),
                                 idx_dev, c->stream));
    return ELOC_OK;
}

int eloc_sr_solve(eloc_ctx c, int n_sr, int64_t n_params, const double* o_re_dev, const double* o_im_dev,
                  const eloc_c64* logpsi_set_dev, const double* grad_dev, double lambda, double* d_dev) {
    if (!c) return ELOC_EINVAL;
    if (n_sr < 1 || n_sr > 256 || n_params < 1 || !(lambda > 0.0) || !std::isfinite(lambda))
        return fail(c, ELOC_EINVAL, "need 1 <= n_sr <= 256, n_params >= 1, finite lambda > 0");
    if (!o_re_dev || !o_im_dev || !logpsi_set_dev || !grad_dev || !d_dev) return fail(c, ELOC_EINVAL, "null pointer");
    const int R = 2 * n_sr + 1;
    const int64_t R16 = (R + 15) / 16 * 16;
    const int64_t n = 2 * n_sr;
    ELOC_HIP(c, c->sr_w.ensure(sizeof(double) * 2 * n_sr));
    ELOC_HIP(c, c->sr_mean.ensure(sizeof(double) * 2 * n_params));
    ELOC_HIP(c, c->sr_part.ensure(sizeof(double) * sr_partial_len(n_params, static_cast<int>(R16), R)));
    ELOC_HIP(c, c->sr_T.ensure(sizeof(double) * R * R));
    ELOC_HIP(c, c->sr_L.ensure(sizeof(double) * n * n));
    ELOC_HIP(c, c->sr_y.ensure(sizeof(double) * n));
    ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    ELOC_HIP(c, launch_sr_solve(n_sr, n_params, o_re_dev, o_im_dev, reinterpret_cast<const double2*>(logpsi_set_dev),
                                grad_dev, lambda, c->sr_w.as<double>(), c->sr_mean.as<double>(), c->sr_part.as<double>(),
                                c->sr_T.as<double>(), c->sr_L.as<double>(), c->sr_y.as<double>(), d_dev,
                                c->err_run.as<uint32_t>(), c->stream));
    return ELOC_OK;
}

int eloc_sample(eloc_ctx c, const eloc_ar_model* m, int64_t k, uint64_t seed, uint64_t* keys_dev, double* logp_dev,
                double* pert_dev, int64_t* n_out_host) {
    if (!c) return ELOC_EINVAL;
    if (!m || !keys_dev || !logp_dev || !n_out_host) return fail(c, ELOC_EINVAL, "null pointer");
    if (m->n_qubits < 1 || m->n_qubits > 128 || m->qudit < 1 || m->qudit > 6 || m->hidden != 64)
        return fail(c, ELOC_EINVAL, "need 1 <= n_qubits <= 128, 1 <= qudit <= 6, hidden == 64");
    if (k < 1 || k >= (int64_t(1) << 24)) return fail(c, ELOC_EINVAL, "need 1 <= k < 2^24");
    if (!m->W1 || !m->b1 || !m->W2 || !m->b2 || !m->W3 || !m->b3) return fail(c, ELOC_EINVAL, "null weights");
    *n_out_host = 0;
    ArModelDev M{m->n_qubits, m->qudit, m->n_up, m->n_down, m->W1, m->b1, m->W2, m->b2, m->W3, m->b3};
    if (M.n_up < 0 || M.n_down < 0) M.n_up = M.n_down = -1;
    const int N = m->n_qubits, W = (N + 63) / 64, D = m->qudit;
    const int Q = (N + D - 1) / D;
    const int64_t maxc = k * (int64_t(1) << D);
    for (int s = 0; s < 2; ++s) {
        ELOC_HIP(c, c->ar_keys[s].ensure(sizeof(uint64_t) * W * k));
        ELOC_HIP(c, c->ar_l[s].ensure(sizeof(double) * k));
        ELOC_HIP(c, c->ar_T[s].ensure(sizeof(double) * k));
    }
    ELOC_HIP(c, c->ar_cl.ensure(sizeof(double) * maxc));
    ELOC_HIP(c, c->ar_cT.ensure(sizeof(double) * maxc));
    ELOC_HIP(c, c->ar_ck.ensure(sizeof(uint64_t) * maxc));
    ELOC_HIP(c, c->ar_ci.ensure(sizeof(uint32_t) * maxc));
    ELOC_HIP(c, c->ar_ck2.ensure(sizeof(uint64_t) * maxc));
    ELOC_HIP(c, c->ar_ci2.ensure(sizeof(uint32_t) * maxc));
    ELOC_HIP(c, c->ar_cnt.ensure(sizeof(unsigned long long)));
    const int64_t tiles = radix_tiles(maxc);
    ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
    ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
    ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * std::max(scan_scratch_len(256 * tiles), scan_scratch_len(maxc))));
    ELOC_HIP(c, c->ar_hist.ensure(sizeof(uint32_t) * 4096));
    ELOC_HIP(c, c->ar_sel.ensure(sizeof(int64_t) * 4));
    ELOC_HIP(c, c->ar_keep.ensure(sizeof(int32_t) * maxc));
    ELOC_HIP(c, c->ar_off.ensure(sizeof(int64_t) * (maxc + 1)));
    ELOC_HIP(c, launch_ar_root(c->ar_keys[0].as<uint64_t>(), W, c->ar_l[0].as<double>(), c->ar_T[0].as<double>(),
                               c->stream));
    int cur = 0;
    int64_t B = 1;
    for (int level = 0; level < Q; ++level) {
        const int Dk = std::min(D, N - level * D);
        const int O = 1 << Dk;
        const int64_t n = B * O;
        ELOC_HIP(c, hipMemsetAsync(c->ar_cnt.p, 0, sizeof(unsigned long long), c->stream));
        ELOC_HIP(c, launch_ar_level(M, level, B, seed, c->ar_keys[cur].as<uint64_t>(), c->ar_l[cur].as<double>(),
                                    c->ar_T[cur].as<double>(), c->ar_cl.as<double>(), c->ar_cT.as<double>(),
                                    c->ar_ck.as<uint64_t>(), c->ar_ci.as<uint32_t>(),
                                    c->ar_cnt.as<unsigned long long>(), c->stream));
        unsigned long long allowed = 0;
        ELOC_HIP(c, hipMemcpyAsync(&allowed, c->ar_cnt.p, sizeof(allowed), hipMemcpyDeviceToHost, c->stream));
        ELOC_HIP(c, hipStreamSynchronize(c->stream));
        const int64_t Bn = std::min<int64_t>(k, static_cast<int64_t>(allowed));
        if (Bn == 0) return ELOC_OK;   // no allowed state
        // the first Bn candidates in (key, index) order: large levels sort
        // only the candidates a two-digit selection keeps, small ones all
        uint32_t* sorted = nullptr;
        if (n >= (int64_t(1) << 16) && n > 4 * Bn) {
            ELOC_HIP(c, launch_ar_select(c->ar_ck.as<uint64_t>(), n, Bn, c->ar_hist.as<uint32_t>(),
                                         c->ar_sel.as<int64_t>(), c->ar_keep.as<int32_t>(), c->ar_off.as<int64_t>(),
                                         c->hist_scratch.as<int64_t>(), c->ar_ck2.as<uint64_t>(),
                                         c->ar_ci2.as<uint32_t>(), c->stream));
            int64_t m = 0;
            ELOC_HIP(c, hipMemcpyAsync(&m, c->ar_off.as<int64_t>() + n, sizeof(m), hipMemcpyDeviceToHost, c->stream));
            ELOC_HIP(c, hipStreamSynchronize(c->stream));
            if (m < Bn || m > n) return fail(c, ELOC_EHIP, "top-K selection kept " + std::to_string(m) + " candidates");
            int alt = 0;
            ELOC_HIP(c, launch_radix_sort_pairs(c->ar_ck2.as<uint64_t>(), c->ar_ci2.as<uint32_t>(),
                                                c->ar_ck.as<uint64_t>(), c->ar_ci.as<uint32_t>(), m, 64,
                                                c->hist.as<uint32_t>(), c->hist_off.as<int64_t>(),
                                                c->hist_scratch.as<int64_t>(), &alt, c->stream));
            sorted = alt ? c->ar_ci.as<uint32_t>() : c->ar_ci2.as<uint32_t>();
        } else {
            int alt = 0;
            ELOC_HIP(c, launch_radix_sort_pairs(c->ar_ck.as<uint64_t>(), c->ar_ci.as<uint32_t>(),
                                                c->ar_ck2.as<uint64_t>(), c->ar_ci2.as<uint32_t>(), n, 64,
                                                c->hist.as<uint32_t>(), c->hist_off.as<int64_t>(),
                                                c->hist_scratch.as<int64_t>(), &alt, c->stream));
            sorted = alt ? c->ar_ci2.as<uint32_t>() : c->ar_ci.as<uint32_t>();
        }
        const int nxt = cur ^ 1;
        ELOC_HIP(c, launch_ar_gather(c->ar_keys[cur].as<uint64_t>(), sorted,
                                     Bn, O, W, level * D, c->ar_cl.as<double>(), c->ar_cT.as<double>(),
                                     c->ar_keys[nxt].as<uint64_t>(), c->ar_l[nxt].as<double>(),
                                     c->ar_T[nxt].as<double>(), c->stream));
        cur = nxt;
        B = Bn;
    }
    ELOC_HIP(c, hipMemcpyAsync(keys_dev, c->ar_keys[cur].p, sizeof(uint64_t) * W * B, hipMemcpyDeviceToDevice, c->stream));
    ELOC_HIP(c, hipMemcpyAsync(logp_dev, c->ar_l[cur].p, sizeof(double) * B, hipMemcpyDeviceToDevice, c->stream));
    if (pert_dev)
        ELOC_HIP(c, hipMemcpyAsync(pert_dev, c->ar_T[cur].p, sizeof(double) * B, hipMemcpyDeviceToDevice, c->stream));
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    *n_out_host = B;
    return ELOC_OK;
}

int eloc_trie_visits(eloc_ctx c, int64_t* visits_host) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!visits_host) return fail(c, ELOC_EINVAL, "null pointer");
    rc = samples_verdict(c, nullptr);
    if (rc) return rc;
    rc = ensure_utrie(c);
    if (rc) return rc;
    const Plan P = make_plan(c, ELOC_TRIE);
    ELOC_HIP(c, c->ar_cnt.ensure(sizeof(unsigned long long)));
    ELOC_HIP(c, hipMemsetAsync(c->ar_cnt.p, 0, sizeof(unsigned long long), c->stream));
    ELOC_HIP(c, launch_trie_visits(c->H, c->S, P, c->ar_cnt.as<unsigned long long>(), c->stream));
    unsigned long long v = 0;
    ELOC_HIP(c, hipMemcpyAsync(&v, c->ar_cnt.p, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    *visits_host = static_cast<int64_t>(v);
    return ELOC_OK;
}

int eloc_check(eloc_ctx c) {
    if (!c) return ELOC_EINVAL;
    if (c->samples_set) {
        bool rebuilt = false;
        const int rc = samples_verdict(c, &rebuilt);
        if (rc) return rc;
        if (rebuilt)
            return fail(c, ELOC_EAGAIN, "U's membership table was rebuilt with a new salt; repeat the last call");
    }
    const int bits = read_err(c, c->err_run);
    if (bits < 0) return bits;
    // a run error is reported once: the word is cleared for the calls after it
    if (bits) ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    return map_err(c, static_cast<uint32_t>(bits));
}

int eloc_count_pairs(eloc_ctx c, int variant, int64_t* n_pairs_host) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!valid_variant(variant)) return fail(c, ELOC_EINVAL, "unknown or unavailable variant");
    variant = resolve_variant(c, variant);
    if (!n_pairs_host) return fail(c, ELOC_EINVAL, "null pointer");
    rc = prepare_variant(c, variant);
    if (rc) return rc;
    const Plan P = make_plan(c, variant, -1, true);
    return count_into_offsets(c, variant, P, n_pairs_host);
}

int eloc_find_pairs(eloc_ctx c, int variant, int64_t capacity, int32_t* i_dev, int32_t* j_dev, int32_t* g_dev,
                    int64_t* n_pairs_host) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!valid_variant(variant)) return fail(c, ELOC_EINVAL, "unknown or unavailable variant");
    variant = resolve_variant(c, variant);
    if (!n_pairs_host) return fail(c, ELOC_EINVAL, "null pointer");
    rc = prepare_variant(c, variant);
    if (rc) return rc;
    const Plan P = make_plan(c, variant, -1, true);
    int64_t total = 0;
    rc = count_into_offsets(c, variant, P, &total);
    if (rc) return rc;
    *n_pairs_host = total;
    if (total > capacity) return fail(c, ELOC_ECAPACITY, "pair capacity too small");
    if (total == 0) return ELOC_OK;
    if (!i_dev || !j_dev || !g_dev) return fail(c, ELOC_EINVAL, "null pointer");
    const int64_t M = c->S.n;
    const int jbits = std::max(1, bits_for(static_cast<uint64_t>(M - 1)));
    const int end_bit = 2 * jbits;
    ELOC_HIP(c, c->pkey.ensure(sizeof(uint64_t) * total));
    ELOC_HIP(c, c->pval.ensure(sizeof(uint32_t) * total));
    ELOC_HIP(c, c->pkey2.ensure(sizeof(uint64_t) * total));
    ELOC_HIP(c, c->pval2.ensure(sizeof(uint32_t) * total));
    ELOC_HIP(c, launch_pairs_fill(variant, c->H, c->S, P, jbits, c->offsets.as<int64_t>(), c->pkey.as<uint64_t>(),
                                  c->pval.as<uint32_t>(), c->stream));
    const int64_t tiles = radix_tiles(total);
    ELOC_HIP(c, c->hist.ensure(sizeof(uint32_t) * 256 * tiles));
    ELOC_HIP(c, c->hist_off.ensure(sizeof(int64_t) * (256 * tiles + 1)));
    ELOC_HIP(c, c->hist_scratch.ensure(sizeof(int64_t) * scan_scratch_len(256 * tiles)));
    int in_alt = 0;
    ELOC_HIP(c, launch_radix_sort_pairs(c->pkey.as<uint64_t>(), c->pval.as<uint32_t>(), c->pkey2.as<uint64_t>(),
                                        c->pval2.as<uint32_t>(), total, end_bit, c->hist.as<uint32_t>(),
                                        c->hist_off.as<int64_t>(), c->hist_scratch.as<int64_t>(), &in_alt,
                                        c->stream));
    const uint64_t* ks = in_alt ? c->pkey2.as<uint64_t>() : c->pkey.as<uint64_t>();
    const uint32_t* vs = in_alt ? c->pval2.as<uint32_t>() : c->pval.as<uint32_t>();
    ELOC_HIP(c, launch_split_pairs(ks, vs, total, jbits, i_dev, j_dev, g_dev, c->stream));
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    return ELOC_OK;
}

int eloc_pair_elements(eloc_ctx c, int64_t n, const int32_t* i_dev, const int32_t* j_dev, eloc_c64* h_dev,
                       int64_t* term_offsets_dev, uint8_t* k_dev, int64_t k_capacity) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(c, ELOC_EINVAL, "pair count must be in 0..2^31-1");
    if (!h_dev || (k_dev && !term_offsets_dev) || (n > 0 && (!i_dev || !j_dev)))
        return fail(c, ELOC_EINVAL, "null pointer");
    if (k_capacity < 0) return fail(c, ELOC_EINVAL, "negative capacity");
    ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    if (n == 0) {
        if (term_offsets_dev) ELOC_HIP(c, hipMemsetAsync(term_offsets_dev, 0, sizeof(int64_t), c->stream));
        return ELOC_OK;
    }
    const bool phases = term_offsets_dev != nullptr;
    if (phases) {
        ELOC_HIP(c, c->pe_cnt.ensure(sizeof(int32_t) * n));
        ELOC_HIP(c, c->pe_grp.ensure(sizeof(int32_t) * n));
        ELOC_HIP(c, c->scan_scratch.ensure(sizeof(int64_t) * scan_scratch_len(n)));
    }
    ELOC_HIP(c, launch_pair_elements(c->H, c->S, n, i_dev, j_dev, reinterpret_cast<double2*>(h_dev),
                                     phases ? c->pe_cnt.as<int32_t>() : nullptr,
                                     phases ? c->pe_grp.as<int32_t>() : nullptr, c->err_run.as<uint32_t>(),
                                     c->stream));
    if (phases) {
        ELOC_HIP(c, launch_scan_i32(c->pe_cnt.as<int32_t>(), n, term_offsets_dev, c->scan_scratch.as<int64_t>(),
                                    c->stream));
        if (k_dev)
            ELOC_HIP(c, launch_pair_phases(c->H, c->S, n, j_dev, c->pe_grp.as<int32_t>(), term_offsets_dev, k_dev,
                                           k_capacity, c->err_run.as<uint32_t>(), c->stream));
    }
    return ELOC_OK;
}

int eloc_local_energy_adjoint(eloc_ctx c, int variant, int precision, const eloc_c64* logpsi_dev,
                              const double* weights_dev, const eloc_c64* eloc_dev, const double* stats_dev,
                              eloc_c64 grad_e, eloc_c64* grad_logpsi_dev) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (precision != ELOC_FP64 && precision != ELOC_FP32C) return fail(c, ELOC_EINVAL, "unknown precision");
    if (!logpsi_dev || !eloc_dev || !stats_dev || !grad_logpsi_dev) return fail(c, ELOC_EINVAL, "null pointer");
    rc = forward_variant(c, &variant);
    if (rc) return rc;
    const int64_t M = c->S.n;
    const bool fp32 = precision == ELOC_FP32C;
    ELOC_HIP(c, hipMemsetAsync(c->err_run.p, 0, sizeof(uint32_t), c->stream));
    rc = amp_prep(c, logpsi_dev, fp32);
    if (rc) return rc;
    ELOC_HIP(c, c->v.ensure(sizeof(double2) * M));
    ELOC_HIP(c, c->vf.ensure(sizeof(float4) * (fp32 ? M : 1)));
    ELOC_HIP(c, launch_adj_vec(c->a.as<double2>(), c->b.as<double2>(), weights_dev, M, fp32, c->v.as<double2>(),
                               c->vf.as<float4>(), c->stream));
    Plan P;
    rc = row_sums(c, true, variant, precision, c->v.as<double2>(), c->vf.as<float4>(), &P);
    if (rc) return rc;
    ELOC_HIP(c, c->amp_scratch.ensure(sizeof(double) * amp_scratch_len()));
    const int pm = prof_begin(c, ELOC_STAGE_ADJOINT_FINISH);
    ELOC_HIP(c, launch_adj_finish(precision, M, P, c->partial.p, c->a.as<double2>(), c->af.as<float4>(),
                                  reinterpret_cast<const double2*>(eloc_dev), weights_dev, stats_dev,
                                  c->amp_scratch.as<double>(), make_double2(grad_e.re, grad_e.im),
                                  reinterpret_cast<double2*>(grad_logpsi_dev), c->stream));
    prof_end(c, pm);
    return ELOC_OK;
}

int eloc_store_pairs(eloc_ctx c, int variant, size_t budget_bytes, int64_t* n_pairs_host) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!n_pairs_host) return fail(c, ELOC_EINVAL, "null pointer");
    if (!valid_variant(variant)) return fail(c, ELOC_EINVAL, "unknown or unavailable variant");
    variant = resolve_variant(c, variant);
    rc = prepare_variant(c, variant);
    if (rc) return rc;
    c->st_valid = false;
    const Plan P = make_plan(c, variant, -1, true);
    int64_t total = 0;
    rc = count_into_offsets(c, variant, P, &total);
    if (rc) return rc;
    *n_pairs_host = total;
    const int64_t M = c->S.n;
    // kept: row pointers, columns, H; transient: the emitted (key, group) pairs
    const double need = static_cast<double>(total) * (sizeof(int32_t) + sizeof(double2) + sizeof(uint64_t) +
                                                      sizeof(uint32_t)) +
                        static_cast<double>(M + 1) * sizeof(int64_t);
    if (need > static_cast<double>(budget_bytes))
        return fail(c, ELOC_ECAPACITY, "the pair list needs " + std::to_string(static_cast<long long>(need)) +
                                           " bytes, more than the budget");
    const int jbits = std::max(1, bits_for(static_cast<uint64_t>(M - 1)));
    ELOC_HIP(c, c->pkey.ensure(sizeof(uint64_t) * std::max<int64_t>(total, 1)));
    ELOC_HIP(c, c->pval.ensure(sizeof(uint32_t) * std::max<int64_t>(total, 1)));
    ELOC_HIP(c, c->st_col.ensure(sizeof(int32_t) * std::max<int64_t>(total, 1)));
    ELOC_HIP(c, c->st_h.ensure(sizeof(double2) * std::max<int64_t>(total, 1)));
    ELOC_HIP(c, c->st_rowptr.ensure(sizeof(int64_t) * (M + 1)));
    if (total > 0) {
        ELOC_HIP(c, launch_pairs_fill(variant, c->H, c->S, P, jbits, c->offsets.as<int64_t>(), c->pkey.as<uint64_t>(),
                                      c->pval.as<uint32_t>(), c->stream));
        ELOC_HIP(c, launch_pairs_to_csr(c->H, c->S, total, c->pkey.as<uint64_t>(), c->pval.as<uint32_t>(), jbits,
                                        c->st_col.as<int32_t>(), c->st_h.as<double2>(), c->stream));
    }
    ELOC_HIP(c, launch_rowptr(c->offsets.as<int64_t>(), M, P.chunks, c->st_rowptr.as<int64_t>(), c->stream));
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    c->st_pairs = total;
    c->st_valid = true;
    return ELOC_OK;
}

int eloc_set_tuning(eloc_ctx c, const eloc_tuning* t) {
    const int tp = t ? t->partition : 0, tc = t ? t->partition_count : 0;
    if (!c || !t || t->chunks < 0 || (t->rows_per_wave != 0 && t->rows_per_wave != 4 && t->rows_per_wave != 8) ||
        (t->waves_per_block != 0 && t->waves_per_block != 1 && t->waves_per_block != 4) || tp < -1 || tp > 1 ||
        !(tc == 0 || tc == 8 || tc == 16 || tc == 32) || t->trie_chunk < 0 || t->trie_chunk > 32767)
        return c ? fail(c, ELOC_EINVAL, "bad tuning") : ELOC_EINVAL;
    c->tune_chunks = t->chunks;
    c->tune_sig = t->sig_filter;
    c->tune_rows = t->rows_per_wave;
    c->tune_bloom = t->bloom;
    c->tune_waves = t->waves_per_block;
    c->tune_part = t->partition;
    c->tune_part_count = t->partition_count;
    c->tune_trie_chunk = t->trie_chunk;
    return ELOC_OK;
}

int eloc_get_tuning(eloc_ctx c, eloc_tuning* t) {
    if (!c || !t) return ELOC_EINVAL;
    t->chunks = c->tune_chunks;
    t->sig_filter = c->tune_sig;
    t->rows_per_wave = c->tune_rows;
    t->bloom = c->tune_bloom;
    t->waves_per_block = c->tune_waves;
    t->partition = c->tune_part;
    t->partition_count = c->tune_part_count;
    t->trie_chunk = c->tune_trie_chunk;
    return ELOC_OK;
}

int eloc_profile_enable(eloc_ctx c, int on) {
    if (!c) return ELOC_EINVAL;
    c->prof = on != 0;
    return ELOC_OK;
}

int eloc_profile_read(eloc_ctx c, double* ms_total, int64_t* count) {
    if (!c || !ms_total || !count) return ELOC_EINVAL;
    for (int k = 0; k < ELOC_NSTAGES; ++k) {
        ms_total[k] = 0.0;
        count[k] = 0;
    }
    ELOC_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& m : c->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess && m.stage >= 0 && m.stage < ELOC_NSTAGES) {
            ms_total[m.stage] += ms;
            count[m.stage] += 1;
        }
        c->ev_pool.push_back(m.a);
        c->ev_pool.push_back(m.b);
    }
    c->marks.clear();
    return ELOC_OK;
}

}  // extern "C"
