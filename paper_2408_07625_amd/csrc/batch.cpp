// Batched launch (C ABI eloc_batch_*): many (Hamiltonian, U) problems of
// uneven size evaluated by one pipeline whose pair stage is one kernel per
// key format over all problems' work items.  The pipeline is captured once
// per precision into a HIP graph and replayed; the schedule (rows per wave,
// workgroups per compute unit, candidates per work item, problem order, and
// the LoopOverTerms / LoopOverBatch choice per problem) is set directly or
// picked by the timing autotuner, whose choice can be kept in a cache file.
#include "eloc.h"
#include "ham.h"
#include "host.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

using namespace eloc;

namespace {

struct ProbInfo {
    int n_qubits;
    int64_t n_terms;
    int64_t G;
    int64_t M;
    int maxpop;
};

}  // namespace

struct eloc_batch_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;
    int n = 0;
    int W = 1;
    int64_t kslot_bytes = 0;   // bytes of all key tables (each problem in its own format)
    int n_cu = 0;
    int64_t S = 0;
    uint64_t salt_state = 0xBA7C4ED5ull;
    uint64_t R[128];
    std::vector<ProbInfo> info;
    std::vector<BatchProb> desc;     // host copy of the descriptors
    std::vector<RTile> tiles;
    std::vector<uint64_t> kcap;      // key-table capacity per problem

    DevBuf R_dev, groups, terms, terms_f, ghash, gkeys, gsplit, gslots, gstash;
    DevBuf probs, pid, tiles_dev, sched, keys, khash, kslots, kstash;
    DevBuf err_dev, sigmin, sigmax, bitcounts, rad, shift, scal, part, pairs, a, b, af, bf, partial;
    uint32_t* err_host = nullptr;

    eloc_batch_schedule schedule{};
    int64_t total_items = 0;
    int64_t narrow_items = 0;   // items of the narrow problems, scheduled first
    bool use_graph = true;
    hipGraphExec_t exec[2] = {nullptr, nullptr};

    // stage timing of eager runs: events around prepare, pairs and finish
    bool prof = false;
    std::vector<hipEvent_t> prof_ev;   // 4 per timed run
    std::vector<hipEvent_t> ev_pool;
};

namespace {

int bfail(eloc_batch b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

int bhip(eloc_batch b, hipError_t e, const char* where) {
    return bfail(b, e == hipErrorOutOfMemory ? ELOC_ENOMEM : ELOC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define BATCH_HIP(b, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return bhip(b, e_, #expr);     \
    } while (0)

void drop_graphs(eloc_batch b) {
    for (auto& e : b->exec) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
    }
}

BatchDev dev_view(const eloc_batch b) {
    BatchDev B;
    B.probs = b->probs.as<BatchProb>();
    B.n = b->n;
    B.W = b->W;
    B.pid = b->pid.as<int32_t>();
    B.S = b->S;
    B.tiles = b->tiles_dev.as<RTile>();
    B.n_tiles = static_cast<int>(b->tiles.size());
    B.sched = b->sched.as<int32_t>();
    B.total_items = b->total_items;
    B.narrow_items = b->narrow_items;
    B.R = b->R_dev.as<uint64_t>();
    B.keys = b->keys.as<uint64_t>();
    B.khash = b->khash.as<uint64_t>();
    B.slots = b->kslots.as<uint32_t>();
    B.n_slot_words = b->kslot_bytes / static_cast<int64_t>(sizeof(uint32_t));
    B.stash = b->kstash.as<Stash>();
    B.err = b->err_dev.as<uint32_t>();
    B.sigmin = b->sigmin.as<uint32_t>();
    B.sigmax = b->sigmax.as<uint32_t>();
    B.bitcounts = b->bitcounts.as<uint32_t>();
    B.rad = b->rad.as<unsigned long long>();
    B.shift = b->shift.as<double>();
    B.scal = b->scal.as<double>();
    B.part = b->part.as<double>();
    B.pairs = b->pairs.as<unsigned long long>();
    B.a = b->a.as<double2>();
    B.b = b->b.as<double2>();
    B.af = b->af.as<float4>();
    B.bf = b->bf.as<float4>();
    B.partial = b->partial.p;
    return B;
}

int valid_schedule(const eloc_batch_schedule& s) {
    return (s.rows_per_wave == 4 || s.rows_per_wave == 8) && s.blocks_per_cu >= 0 && s.item_candidates >= 64 &&
           (s.order == 0 || s.order == 1) && s.batch_ratio >= 0.0 && std::isfinite(s.batch_ratio);
}

// Work items and partial layout for schedule s; uploads the descriptors.
int apply_schedule(eloc_batch b, const eloc_batch_schedule& s) {
    const int n = b->n;
    std::vector<int64_t> cost(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) {
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        const ProbInfo& I = b->info[static_cast<size_t>(k)];
        D.variant = (static_cast<double>(I.M) <= s.batch_ratio * static_cast<double>(I.G)) ? 1 : 0;
        const int64_t span = D.variant == 1 ? I.M : I.G;
        // chunks of whole 64-lane steps, split as evenly as the single-problem
        // plan splits them for the same chunk count
        const int64_t steps = (span + 63) / 64;
        const int64_t want = std::max<int64_t>(1, (s.item_candidates + 64 * s.rows_per_wave - 1) /
                                                      (64 * s.rows_per_wave));
        const int64_t nchunks = std::min<int64_t>(steps, (steps + want - 1) / want);
        const int64_t per_steps = (steps + nchunks - 1) / nchunks;
        const int64_t per = per_steps * 64;
        D.per_chunk = static_cast<int32_t>(per);
        D.chunks = static_cast<int32_t>((span + per - 1) / per);
        const int64_t row_tiles = (I.M + s.rows_per_wave - 1) / s.rows_per_wave;
        D.items = row_tiles * D.chunks;
        cost[static_cast<size_t>(k)] = I.M * span;
    }
    std::vector<int32_t> order(static_cast<size_t>(n));
    std::iota(order.begin(), order.end(), 0);
    if (s.order == 0)
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return cost[static_cast<size_t>(x)] > cost[static_cast<size_t>(y)]; });
    // narrow problems first: their items run in the narrow kernel
    std::stable_partition(order.begin(), order.end(),
                          [&](int32_t k) { return b->desc[static_cast<size_t>(k)].narrow != 0; });
    int64_t item = 0, narrow_items = 0;
    for (int32_t k : order) {
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        D.item0 = item;
        item += D.items;
        if (D.narrow) narrow_items = item;
    }
    if (item >= (int64_t(1) << 31)) return bfail(b, ELOC_EINVAL, "too many work items; raise item_candidates");
    int64_t pbase = 0;
    for (int k = 0; k < n; ++k) {
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        D.pbase = pbase;
        pbase += static_cast<int64_t>(D.chunks) * D.M;
    }
    BATCH_HIP(b, b->partial.ensure(sizeof(double2) * static_cast<size_t>(pbase)));
    BATCH_HIP(b, hipMemcpy(b->probs.p, b->desc.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice));
    BATCH_HIP(b, hipMemcpy(b->sched.p, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    b->total_items = item;
    b->narrow_items = narrow_items;
    b->schedule = s;
    drop_graphs(b);
    return ELOC_OK;
}

// Workgroups of a batched pair kernel: one per work item (blocks_per_cu <= 0),
// or blocks_per_cu per CU (at most what fits) striding over the items.
int launch_blocks(eloc_batch b, int precision, bool narrow) {
    const int64_t items = narrow ? b->narrow_items : b->total_items - b->narrow_items;
    int64_t blocks = items;
    if (b->schedule.blocks_per_cu > 0) {
        int per_cu = b->schedule.blocks_per_cu;
        const int fit = batch_blocks_per_cu(b->W, narrow, precision, b->schedule.rows_per_wave);
        if (fit > 0 && per_cu > fit) per_cu = fit;
        blocks = std::min<int64_t>(items, static_cast<int64_t>(per_cu) * b->n_cu);
    }
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(blocks, int64_t(1) << 30)));
}

hipEvent_t batch_event(eloc_batch b) {
    if (!b->ev_pool.empty()) {
        hipEvent_t e = b->ev_pool.back();
        b->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// `timed`: eager run with profiling on; events before prepare, pairs,
// finish and after finish
int enqueue(eloc_batch b, int precision, hipStream_t st, bool timed = false) {
    const BatchDev B = dev_view(b);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (timed)
        for (auto& e : ev)
            if (!(e = batch_event(b))) return bfail(b, ELOC_EHIP, "hipEventCreate");
    auto mark = [&](int k) { return timed ? hipEventRecord(ev[k], st) : hipSuccess; };
    BATCH_HIP(b, mark(0));
    BATCH_HIP(b, launch_batch_prepare(B, precision == ELOC_FP32C, st));
    BATCH_HIP(b, mark(1));
    BATCH_HIP(b, launch_batch_pairs(B, precision, b->schedule.rows_per_wave, launch_blocks(b, precision, true),
                                    launch_blocks(b, precision, false), st));
    BATCH_HIP(b, mark(2));
    BATCH_HIP(b, launch_batch_finish(B, precision, st));
    BATCH_HIP(b, mark(3));
    if (timed) b->prof_ev.insert(b->prof_ev.end(), ev, ev + 4);
    return ELOC_OK;
}

int ensure_graph(eloc_batch b, int precision) {
    if (b->exec[precision]) return ELOC_OK;
    if (!b->cap_stream) BATCH_HIP(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    BATCH_HIP(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(b, precision, b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc != ELOC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return bhip(b, ei, "hipGraphInstantiate");
    b->exec[precision] = x;
    return ELOC_OK;
}

int run(eloc_batch b, int precision) {
    if (b->use_graph) {
        const int rc = ensure_graph(b, precision);
        if (rc) return rc;
        BATCH_HIP(b, hipGraphLaunch(b->exec[precision], b->stream));
        return ELOC_OK;
    }
    return enqueue(b, precision, b->stream, b->prof);
}

// Group membership tables (LoopOverBatch), built once; a new salt is drawn if
// an insertion does not settle.
int build_group_table(eloc_batch b, int tk, const uint64_t* hash, int64_t n, void* slots, Stash* stash,
                      uint64_t cap, Table* out) {
    for (int attempt = 0; attempt < 8; ++attempt) {
        Table T = make_table(slots, stash, cap, n, splitmix64(b->salt_state));
        BATCH_HIP(b, hipMemset(slots, 0, slot_bytes(tk) * cap));
        BATCH_HIP(b, hipMemset(stash, 0, sizeof(Stash)));
        BATCH_HIP(b, hipMemset(b->err_dev.p, 0, sizeof(uint32_t)));
        BATCH_HIP(b, launch_table_insert(tk, hash, n, slots, stash, T, b->err_dev.as<uint32_t>(), nullptr));
        BATCH_HIP(b, hipMemcpy(b->err_host, b->err_dev.p, sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (!(b->err_host[0] & kErrTable)) {
            *out = T;
            return ELOC_OK;
        }
    }
    return bfail(b, ELOC_EHIP, "group membership table could not be built");
}

template <int W>
int ingest_all(eloc_batch b, const eloc_problem* probs) {
    const int n = b->n;
    std::vector<HostHam<W>> hh(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) {
        const eloc_problem& p = probs[k];
        const int wk = (p.n_qubits + 63) / 64;
        std::vector<uint64_t> xy(static_cast<size_t>(p.n_terms) * W, 0), yz(static_cast<size_t>(p.n_terms) * W, 0);
        for (int64_t l = 0; l < p.n_terms; ++l)
            for (int w = 0; w < wk; ++w) {
                xy[static_cast<size_t>(l * W + w)] = p.xy[l * wk + w];
                yz[static_cast<size_t>(l * W + w)] = p.yz[l * wk + w];
            }
        const std::string why = build_host_ham<W>(b->R, p.n_terms, p.coeff, xy.data(), yz.data(), hh[static_cast<size_t>(k)]);
        if (!why.empty()) return bfail(b, ELOC_EINVAL, "problem " + std::to_string(k) + ": " + why);
    }
    // each problem's table format: narrow for one-word batches of problems of
    // at most 32 qubits whose group parts fit the narrow hit queue's 16 bits
    std::vector<int> tk(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) {
        const bool nar = W == 1 && probs[k].n_qubits <= 32 && hh[static_cast<size_t>(k)].maxpart < kNarrowMaxPart;
        tk[static_cast<size_t>(k)] = table_kind(W, nar);
        b->desc[static_cast<size_t>(k)].narrow = nar ? 1 : 0;
    }
    int64_t nt = 0, ng = 0, gcap = 0, kc = 0;
    std::vector<int64_t> toff(static_cast<size_t>(n)), goff(static_cast<size_t>(n)), gcoff(static_cast<size_t>(n)),
        kcoff(static_cast<size_t>(n));
    b->kcap.assign(static_cast<size_t>(n), 0);
    std::vector<uint64_t> gc(static_cast<size_t>(n));
    for (int k = 0; k < n; ++k) {
        const HostHam<W>& h = hh[static_cast<size_t>(k)];
        toff[static_cast<size_t>(k)] = nt;
        goff[static_cast<size_t>(k)] = ng;
        gcoff[static_cast<size_t>(k)] = gcap;   // bytes
        kcoff[static_cast<size_t>(k)] = kc;
        nt += h.n_terms;
        ng += h.G;
        const int64_t sb = static_cast<int64_t>(slot_bytes(tk[static_cast<size_t>(k)]));
        gc[static_cast<size_t>(k)] = table_capacity(h.G);
        gcap += sb * static_cast<int64_t>(gc[static_cast<size_t>(k)]);
        b->kcap[static_cast<size_t>(k)] = table_capacity(probs[k].n_unique);
        kc += sb * static_cast<int64_t>(b->kcap[static_cast<size_t>(k)]);
    }
    BATCH_HIP(b, b->groups.ensure(sizeof(GroupRec<W>) * ng));
    BATCH_HIP(b, b->ghash.ensure(sizeof(uint64_t) * ng));
    BATCH_HIP(b, b->gkeys.ensure(sizeof(uint64_t) * ng * W));
    BATCH_HIP(b, b->gsplit.ensure(sizeof(uint64_t) * ng * W));
    BATCH_HIP(b, b->terms.ensure(sizeof(TermRec<W>) * nt));
    BATCH_HIP(b, b->terms_f.ensure(sizeof(TermRecF<W>) * nt));
    BATCH_HIP(b, b->gslots.ensure(static_cast<size_t>(gcap)));
    BATCH_HIP(b, b->gstash.ensure(sizeof(Stash) * n));
    BATCH_HIP(b, b->kslots.ensure(static_cast<size_t>(kc)));
    b->kslot_bytes = kc;
    BATCH_HIP(b, b->kstash.ensure(sizeof(Stash) * n));
    auto* groups = b->groups.as<GroupRec<W>>();
    auto* terms = b->terms.as<TermRec<W>>();
    auto* terms_f = b->terms_f.as<TermRecF<W>>();
    for (int k = 0; k < n; ++k) {
        const HostHam<W>& h = hh[static_cast<size_t>(k)];
        const size_t go = static_cast<size_t>(goff[static_cast<size_t>(k)]);
        const size_t to = static_cast<size_t>(toff[static_cast<size_t>(k)]);
        BATCH_HIP(b, hipMemcpy(groups + go, h.groups.data(), sizeof(GroupRec<W>) * h.G, hipMemcpyHostToDevice));
        BATCH_HIP(b, hipMemcpy(b->ghash.as<uint64_t>() + go, h.ghash.data(), sizeof(uint64_t) * h.G,
                               hipMemcpyHostToDevice));
        BATCH_HIP(b, hipMemcpy(b->gkeys.as<uint64_t>() + go * W, h.gkeys.data(), sizeof(uint64_t) * h.G * W,
                               hipMemcpyHostToDevice));
        std::vector<uint64_t> split(h.gkeys.size());
        for (size_t i = 0; i < split.size(); ++i) split[i] = spin_split(h.gkeys[i]);
        BATCH_HIP(b, hipMemcpy(b->gsplit.as<uint64_t>() + go * W, split.data(), sizeof(uint64_t) * h.G * W,
                               hipMemcpyHostToDevice));
        BATCH_HIP(b, hipMemcpy(terms + to, h.terms.data(), sizeof(TermRec<W>) * h.n_terms, hipMemcpyHostToDevice));
        BATCH_HIP(b, hipMemcpy(terms_f + to, h.terms_f.data(), sizeof(TermRecF<W>) * h.n_terms,
                               hipMemcpyHostToDevice));
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        D.groups = groups + go;
        D.ghash = b->ghash.as<uint64_t>() + go;
        D.gsplit = b->gsplit.as<uint64_t>() + go * W;
        D.terms = terms + to;
        D.terms_f = terms_f + to;
        D.gkeys = b->gkeys.as<uint64_t>() + go * W;
        void* gs = b->gslots.as<char>() + static_cast<size_t>(gcoff[static_cast<size_t>(k)]);
        Stash* gst = b->gstash.as<Stash>() + k;
        const int rc =
            build_group_table(b, tk[static_cast<size_t>(k)], D.ghash, h.G, gs, gst, gc[static_cast<size_t>(k)], &D.gtable);
        if (rc) return rc;
        D.n_groups = static_cast<int32_t>(h.G);
        D.maxpop = h.maxpop;
        ProbInfo& I = b->info[static_cast<size_t>(k)];
        I.n_terms = h.n_terms;
        I.G = h.G;
        I.maxpop = h.maxpop;
        D.kslots = b->kslots.as<char>() + static_cast<size_t>(kcoff[static_cast<size_t>(k)]);
        D.kstash = b->kstash.as<Stash>() + k;
        D.ktable = make_table(D.kslots, D.kstash, b->kcap[static_cast<size_t>(k)], I.M, splitmix64(b->salt_state));
    }
    return ELOC_OK;
}

int map_bits(eloc_batch b, int k, uint32_t bits) {
    const std::string p = "problem " + std::to_string(k) + ": ";
    if (bits & kErrTable) {
        // draw a new salt for this problem's key table; the next run uses it
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        D.ktable.salt = splitmix64(b->salt_state);
        BATCH_HIP(b, hipMemcpy(b->probs.as<BatchProb>() + k, &D, sizeof(BatchProb), hipMemcpyHostToDevice));
        return bfail(b, ELOC_EAGAIN, p + "membership table overflow; it was rebuilt with a new salt, run again");
    }
    if (bits & kErrBits) return bfail(b, ELOC_EINVAL, p + "a sample key has bits set at or above n_qubits");
    if (bits & kErrDup) return bfail(b, ELOC_EDUP, p + "duplicate keys in the sample batch");
    if (bits & kErrWeights) return bfail(b, ELOC_EINVAL, p + "weights must be finite, >= 0, with a positive sum");
    if (bits & kErrRange)
        return bfail(b, ELOC_ERANGE, p + "log-amplitudes not finite, or Re log psi spread above 60 (FP32 form) or 700 (FP64 form)");
    return ELOC_OK;
}

uint64_t fnv1a(const std::string& s) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 0x100000001b3ull;
    }
    return h;
}

std::string cache_key(eloc_batch b, int precision) {
    std::ostringstream os;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) os << prop.gcnArchName << '|';
    os << b->n_cu << '|' << b->W << '|' << precision << '|' << b->n << '|';
    for (const ProbInfo& I : b->info) os << I.n_qubits << ',' << I.n_terms << ',' << I.G << ',' << I.M << ';';
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%016llx", static_cast<unsigned long long>(fnv1a(os.str())));
    return buf;
}

// Cache file: one line per problem set, "key rows blocks_per_cu
// item_candidates order batch_ratio ms".
bool cache_lookup(const char* path, const std::string& key, eloc_batch_schedule* s) {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        eloc_batch_schedule t{};
        double ms = 0.0;
        long long items = 0;
        if (is >> k >> t.rows_per_wave >> t.blocks_per_cu >> items >> t.order >> t.batch_ratio >> ms && k == key) {
            t.item_candidates = items;
            if (!valid_schedule(t)) return false;
            *s = t;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const eloc_batch_schedule& s, double ms) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.compare(0, key.size() + 1, key + " ") != 0 && !line.empty()) keep.push_back(line);
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s %d %d %lld %d %.17g %.6f", key.c_str(), s.rows_per_wave, s.blocks_per_cu,
                  static_cast<long long>(s.item_candidates), s.order, s.batch_ratio, ms);
    keep.push_back(buf);
    std::ofstream f(path, std::ios::trunc);
    for (const std::string& l : keep) f << l << '\n';
}

// Milliseconds of the whole pipeline under schedule s (best of `reps`
// eager runs after one warm-up run).
int time_schedule(eloc_batch b, int precision, const eloc_batch_schedule& s, int reps, double* ms_out) {
    int rc = apply_schedule(b, s);
    if (rc) return rc;
    hipEvent_t e0, e1;
    BATCH_HIP(b, hipEventCreate(&e0));
    BATCH_HIP(b, hipEventCreate(&e1));
    double best = INFINITY;
    for (int r = 0; r <= reps && rc == ELOC_OK; ++r) {
        if (hipEventRecord(e0, b->stream) != hipSuccess) rc = bfail(b, ELOC_EHIP, "hipEventRecord");
        if (rc == ELOC_OK) rc = enqueue(b, precision, b->stream);
        if (rc == ELOC_OK && hipEventRecord(e1, b->stream) != hipSuccess) rc = bfail(b, ELOC_EHIP, "hipEventRecord");
        if (rc == ELOC_OK && hipEventSynchronize(e1) != hipSuccess) rc = bfail(b, ELOC_EHIP, "hipEventSynchronize");
        float ms = 0.f;
        if (rc == ELOC_OK && r > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, double(ms));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = best;
    return rc;
}

}  // namespace

extern "C" {

int eloc_batch_create(eloc_batch* out, int device, void* hip_stream, int n, const eloc_problem* probs) {
    if (!out) return ELOC_EINVAL;
    *out = nullptr;
    if (n < 1 || n > kMaxBatch || !probs) return ELOC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ELOC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ELOC_EHIP;
    eloc_batch b = new eloc_batch_s();
    *out = b;
    b->device = device;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->n = n;
    make_hash_words(b->R);
    if (hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || b->n_cu < 1)
        return bfail(b, ELOC_EHIP, "compute unit count");
    if (hipHostMalloc(reinterpret_cast<void**>(&b->err_host), sizeof(uint32_t) * kMaxBatch, hipHostMallocDefault) !=
        hipSuccess)
        return bfail(b, ELOC_EHIP, "hipHostMalloc");
    int W = 1;
    b->info.resize(static_cast<size_t>(n));
    b->desc.assign(static_cast<size_t>(n), BatchProb{});
    int64_t S = 0;
    for (int k = 0; k < n; ++k) {
        const eloc_problem& p = probs[k];
        const std::string pre = "problem " + std::to_string(k) + ": ";
        if (p.n_qubits < 1 || p.n_qubits > 128) return bfail(b, ELOC_EINVAL, pre + "n_qubits must be in 1..128");
        if (p.n_terms < 1 || !p.coeff || !p.xy || !p.yz)
            return bfail(b, ELOC_EINVAL, pre + "empty Hamiltonian or null pointer");
        if (p.n_unique < 1 || p.n_unique >= (int64_t(1) << 24) || !p.keys_dev || !p.logpsi_dev || !p.eloc_dev ||
            !p.stats_dev)
            return bfail(b, ELOC_EINVAL, pre + "n_unique must be in 1..2^24-1 with key, log-psi and output pointers");
        const int wk = (p.n_qubits + 63) / 64;
        for (int64_t l = 0; l < p.n_terms; ++l) {
            for (int w = 0; w < wk; ++w) {
                const int valid = p.n_qubits - 64 * w;
                if (valid < 64 && ((p.xy[l * wk + w] | p.yz[l * wk + w]) & ~((1ull << valid) - 1ull)))
                    return bfail(b, ELOC_EINVAL, pre + "a term mask has bits set at or above n_qubits");
            }
            if (!std::isfinite(p.coeff[l])) return bfail(b, ELOC_EINVAL, pre + "non-finite coefficient");
        }
        W = std::max(W, wk);
        ProbInfo& I = b->info[static_cast<size_t>(k)];
        I.n_qubits = p.n_qubits;
        I.M = p.n_unique;
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        D.n_qubits = p.n_qubits;
        D.s0 = S;
        D.M = p.n_unique;
        D.keys_in = p.keys_dev;
        D.w_in = wk;
        D.logpsi = reinterpret_cast<const double2*>(p.logpsi_dev);
        D.weights = p.weights_dev;
        D.eloc = reinterpret_cast<double2*>(p.eloc_dev);
        D.stats = p.stats_dev;
        S += p.n_unique;
    }
    b->W = W;
    b->S = S;
    // reduction tiles and the sample -> problem map
    std::vector<int32_t> pid(static_cast<size_t>(S));
    for (int k = 0; k < n; ++k) {
        BatchProb& D = b->desc[static_cast<size_t>(k)];
        D.rt0 = static_cast<int32_t>(b->tiles.size());
        for (int64_t t = D.s0; t < D.s0 + D.M; t += kBTile)
            b->tiles.push_back(RTile{k, 0, t, std::min(D.s0 + D.M, t + kBTile)});
        D.rtn = static_cast<int32_t>(b->tiles.size()) - D.rt0;
        std::fill(pid.begin() + D.s0, pid.begin() + D.s0 + D.M, k);
    }
    BATCH_HIP(b, b->err_dev.ensure(sizeof(uint32_t) * n));
    const int rc = W == 1 ? ingest_all<1>(b, probs) : ingest_all<2>(b, probs);
    if (rc) return rc;
    const size_t nt = b->tiles.size();
    BATCH_HIP(b, b->R_dev.ensure(sizeof(b->R)));
    BATCH_HIP(b, hipMemcpy(b->R_dev.p, b->R, sizeof(b->R), hipMemcpyHostToDevice));
    BATCH_HIP(b, b->probs.ensure(sizeof(BatchProb) * n));
    BATCH_HIP(b, b->sched.ensure(sizeof(int32_t) * n));
    BATCH_HIP(b, b->pid.ensure(sizeof(int32_t) * S));
    BATCH_HIP(b, hipMemcpy(b->pid.p, pid.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice));
    BATCH_HIP(b, b->tiles_dev.ensure(sizeof(RTile) * nt));
    BATCH_HIP(b, hipMemcpy(b->tiles_dev.p, b->tiles.data(), sizeof(RTile) * nt, hipMemcpyHostToDevice));
    BATCH_HIP(b, b->keys.ensure(sizeof(uint64_t) * S * W));
    BATCH_HIP(b, b->khash.ensure(sizeof(uint64_t) * S));
    BATCH_HIP(b, b->sigmin.ensure(sizeof(uint32_t) * n));
    BATCH_HIP(b, b->sigmax.ensure(sizeof(uint32_t) * n));
    BATCH_HIP(b, b->bitcounts.ensure(sizeof(uint32_t) * 128 * n));
    BATCH_HIP(b, b->rad.ensure(sizeof(unsigned long long) * 3 * n));
    BATCH_HIP(b, b->shift.ensure(sizeof(double) * n));
    BATCH_HIP(b, b->scal.ensure(sizeof(double) * 3 * n));
    BATCH_HIP(b, b->part.ensure(sizeof(double) * 3 * nt));
    BATCH_HIP(b, b->pairs.ensure(sizeof(unsigned long long) * n));
    BATCH_HIP(b, b->a.ensure(sizeof(double2) * S));
    BATCH_HIP(b, b->b.ensure(sizeof(double2) * S));
    BATCH_HIP(b, b->af.ensure(sizeof(float4) * S));
    BATCH_HIP(b, b->bf.ensure(sizeof(float4) * S));
    eloc_batch_schedule s0;
    s0.rows_per_wave = 8;
    s0.blocks_per_cu = 0;
    s0.item_candidates = int64_t(1) << 17;
    s0.order = 0;
    s0.batch_ratio = 1.0;
    return apply_schedule(b, s0);
}

void eloc_batch_destroy(eloc_batch b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    DevBuf* bufs[] = {&b->R_dev, &b->groups, &b->terms, &b->terms_f, &b->ghash, &b->gkeys, &b->gsplit, &b->gslots, &b->gstash,
                      &b->probs, &b->pid, &b->tiles_dev, &b->sched, &b->keys, &b->khash, &b->kslots, &b->kstash,
                      &b->err_dev, &b->sigmin, &b->sigmax, &b->bitcounts, &b->rad, &b->shift, &b->scal, &b->part, &b->pairs,
                      &b->a, &b->b, &b->af, &b->bf, &b->partial};
    for (DevBuf* d : bufs) d->release();
    for (hipEvent_t e : b->prof_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
    if (b->err_host) (void)hipHostFree(b->err_host);
    delete b;
}

const char* eloc_batch_last_error(eloc_batch b) { return b ? b->err.c_str() : "null batch"; }

int eloc_batch_set_stream(eloc_batch b, void* hip_stream) {
    if (!b) return ELOC_EINVAL;
    b->stream = static_cast<hipStream_t>(hip_stream);
    return ELOC_OK;
}

int eloc_batch_set_graph(eloc_batch b, int on) {
    if (!b) return ELOC_EINVAL;
    b->use_graph = on != 0;
    return ELOC_OK;
}

int eloc_batch_run(eloc_batch b, int precision) {
    if (!b) return ELOC_EINVAL;
    if (precision != ELOC_FP64 && precision != ELOC_FP32C) return bfail(b, ELOC_EINVAL, "unknown precision");
    return run(b, precision);
}

int eloc_batch_profile_enable(eloc_batch b, int on) {
    if (!b) return ELOC_EINVAL;
    b->prof = on != 0;
    return ELOC_OK;
}

int eloc_batch_profile_read(eloc_batch b, double* ms_total, int64_t* count) {
    if (!b || !ms_total || !count) return ELOC_EINVAL;
    for (int k = 0; k < 3; ++k) {
        ms_total[k] = 0.0;
        count[k] = 0;
    }
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    for (size_t r = 0; r + 4 <= b->prof_ev.size(); r += 4)
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, b->prof_ev[r + k], b->prof_ev[r + k + 1]) == hipSuccess) {
                ms_total[k] += ms;
                count[k] += 1;
            }
        }
    b->ev_pool.insert(b->ev_pool.end(), b->prof_ev.begin(), b->prof_ev.end());
    b->prof_ev.clear();
    return ELOC_OK;
}

int eloc_batch_check(eloc_batch b, int* bad_problem) {
    if (!b) return ELOC_EINVAL;
    if (bad_problem) *bad_problem = -1;
    BATCH_HIP(b, hipMemcpyAsync(b->err_host, b->err_dev.p, sizeof(uint32_t) * b->n, hipMemcpyDeviceToHost, b->stream));
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    for (int k = 0; k < b->n; ++k)
        if (b->err_host[k]) {
            if (bad_problem) *bad_problem = k;
            return map_bits(b, k, b->err_host[k]);
        }
    return ELOC_OK;
}

int eloc_batch_pair_counts(eloc_batch b, int64_t* counts_host) {
    if (!b || !counts_host) return ELOC_EINVAL;
    BATCH_HIP(b, hipStreamSynchronize(b->stream));
    BATCH_HIP(b, hipMemcpy(counts_host, b->pairs.p, sizeof(int64_t) * b->n, hipMemcpyDeviceToHost));
    return ELOC_OK;
}

int eloc_batch_get_schedule(eloc_batch b, eloc_batch_schedule* s) {
    if (!b || !s) return ELOC_EINVAL;
    *s = b->schedule;
    return ELOC_OK;
}

int eloc_batch_set_schedule(eloc_batch b, const eloc_batch_schedule* s) {
    if (!b || !s) return ELOC_EINVAL;
    if (!valid_schedule(*s)) return bfail(b, ELOC_EINVAL, "bad schedule");
    return apply_schedule(b, *s);
}

int eloc_batch_problem_info(eloc_batch b, int k, int64_t* n_groups, int64_t* n_terms, int* variant, int* chunks) {
    if (!b) return ELOC_EINVAL;
    if (k < 0 || k >= b->n) return bfail(b, ELOC_EINVAL, "problem index out of range");
    const BatchProb& D = b->desc[static_cast<size_t>(k)];
    if (n_groups) *n_groups = b->info[static_cast<size_t>(k)].G;
    if (n_terms) *n_terms = b->info[static_cast<size_t>(k)].n_terms;
    if (variant) *variant = D.variant;
    if (chunks) *chunks = D.chunks;
    return ELOC_OK;
}

int eloc_batch_tune(eloc_batch b, int precision, const char* cache_path, int* from_cache) {
    if (!b) return ELOC_EINVAL;
    if (precision != ELOC_FP64 && precision != ELOC_FP32C) return bfail(b, ELOC_EINVAL, "unknown precision");
    if (from_cache) *from_cache = 0;
    const std::string key = cache_key(b, precision);
    eloc_batch_schedule s{};
    if (cache_path && cache_lookup(cache_path, key, &s)) {
        if (from_cache) *from_cache = 1;
        return apply_schedule(b, s);
    }
    // coordinate search, one dimension at a time from a fixed start
    eloc_batch_schedule best;
    best.rows_per_wave = 8;
    best.blocks_per_cu = 0;
    best.item_candidates = int64_t(1) << 17;
    best.order = 0;
    best.batch_ratio = 1.0;
    double best_ms = INFINITY;
    auto trial = [&](const eloc_batch_schedule& t) -> int {
        double ms = INFINITY;
        const int rc = time_schedule(b, precision, t, 2, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
        return ELOC_OK;
    };
    int rc = trial(best);
    for (int rows : {4, 8})
        for (int64_t items : {int64_t(1) << 15, int64_t(1) << 17, int64_t(1) << 19}) {
            if (rc) break;
            eloc_batch_schedule t = best;
            t.rows_per_wave = rows;
            t.item_candidates = items;
            if (t.rows_per_wave != best.rows_per_wave || t.item_candidates != best.item_candidates) rc = trial(t);
        }
    for (double ratio : {0.0, 0.25, 1.0, 4.0}) {
        if (rc) break;
        eloc_batch_schedule t = best;
        t.batch_ratio = ratio;
        if (t.batch_ratio != best.batch_ratio) rc = trial(t);
    }
    {
        const int fit = batch_blocks_per_cu(b->W, b->narrow_items < b->total_items ? false : true, precision,
                                            best.rows_per_wave);
        for (int bpc : {fit / 2, fit}) {
            if (rc || bpc < 1) continue;
            eloc_batch_schedule t = best;
            t.blocks_per_cu = bpc;
            if (t.blocks_per_cu != best.blocks_per_cu) rc = trial(t);
        }
    }
    for (int order : {0, 1}) {
        if (rc) break;
        eloc_batch_schedule t = best;
        t.order = order;
        if (t.order != best.order) rc = trial(t);
    }
    if (rc) return rc;
    rc = apply_schedule(b, best);
    if (rc) return rc;
    if (cache_path) cache_store(cache_path, key, best, best_ms);
    return ELOC_OK;
}

}  // extern "C"
