// HIP kernels for gfx950 (CDNA4, wave64) of the sample-aware local energy.
//
// Work decomposition of the pair kernels: one lane per sample row x (the
// row's key, its linear hash and its accumulator stay in registers), the
// grid's y dimension splits the loop over the unique XY set (LoopOverTerms)
// or over U (LoopOverBatch) into chunks so that a launch has enough waves to
// cover the chip.  Each (row, chunk) writes one partial sum; a second kernel
// adds the chunks in a fixed order, so results are bitwise reproducible and
// no floating-point atomics are used.
//
// LoopOverTerms (Alg. 2A): the chunk's XY masks are wave-uniform, so the
// group record, the group hash and the group's term run are scalar loads;
// x' = x ^ XY is looked up in the sample table.  LoopOverBatch (Alg. 2B): the
// chunk's sample keys are wave-uniform; x ^ x' is rejected when its popcount
// exceeds the largest XY popcount, otherwise looked up in the XY table.
//
// MatrixElement (supplementary algorithm, Eq. pauli_melem): for a term with
// mask YZ the factor is i^(|XY & YZ|) (-1)^(|ket & YZ|), so a term adds +-h to
// the real or the imaginary part; only additions are rounded.
#include "internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kEven = 0x5555555555555555ull;
constexpr uint64_t kOdd = 0xAAAAAAAAAAAAAAAAull;

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }

template <int W>
__device__ __forceinline__ bool sig_ok(const uint64_t* sig, const uint64_t* k) {
    int pa = 0, pb = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        pa += popc64(k[w] & kEven);
        pb += popc64(k[w] & kOdd);
    }
    return (sig[2 * pa + (pb >> 6)] >> (pb & 63)) & 1ull;
}

// ---------------------------------------------------------------------------
// Compensated FP32 arithmetic (error-free transforms).
//   TwoSum: Knuth, TAOCP vol. 2;  TwoProduct via fused multiply-add;
//   accumulation as in Ogita, Rump, Oishi, "Accurate sum and dot product",
//   SIAM J. Sci. Comput. 26(6), 2005 (Sum2 / Dot2): the running sum s and
// the running sum c of all rounding errors are kept separately.
// ---------------------------------------------------------------------------
struct F2 {      // value = s + c
    float s, c;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void acc_add(F2& acc, float hi, float lo) {
    float s, e;
    two_sum(acc.s, hi, s, e);
    acc.s = s;
    acc.c += e + lo;
}

// (x.s + x.c) * (y.s + y.c) as hi + lo, exact in the leading product.
__device__ __forceinline__ void df_mul(F2 x, F2 y, float& hi, float& lo) {
    hi = x.s * y.s;
    lo = fmaf(x.s, y.s, -hi);
    lo = fmaf(x.s, y.c, lo);
    lo = fmaf(x.c, y.s, lo);
}

struct AccD {
    double re = 0.0, im = 0.0;
};
struct AccF {
    F2 re{0.f, 0.f}, im{0.f, 0.f};
};

// ---------------------------------------------------------------------------
// MatrixElement over a run of terms.  `xy` is the group's mask, `ket` the key
// the phase is evaluated on.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void melem_f64(const TermRec<W>* __restrict__ terms, int b, int e,
                                          const uint64_t* xy, const uint64_t* ket, double& hr,
                                          double& hi) {
    hr = 0.0;
    hi = 0.0;
    for (int t = b; t < e; ++t) {
        const TermRec<W> tr = terms[t];
        int ny = 0, pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            ny += popc64(xy[w] & tr.yz[w]);
            pc += popc64(ket[w] & tr.yz[w]);
        }
        const double v = (((ny >> 1) ^ pc) & 1) ? -tr.h : tr.h;
        if (ny & 1)
            hi += v;
        else
            hr += v;
    }
}

template <int W>
__device__ __forceinline__ void melem_f32(const TermRecF<W>* __restrict__ terms, int b, int e,
                                          const uint64_t* xy, const uint64_t* ket, F2& hr,
                                          F2& hi) {
    hr = F2{0.f, 0.f};
    hi = F2{0.f, 0.f};
    for (int t = b; t < e; ++t) {
        const TermRecF<W> tr = terms[t];
        int ny = 0, pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            ny += popc64(xy[w] & tr.yz[w]);
            pc += popc64(ket[w] & tr.yz[w]);
        }
        const bool neg = ((ny >> 1) ^ pc) & 1;
        const float vh = neg ? -tr.h_hi : tr.h_hi;
        const float vl = neg ? -tr.h_lo : tr.h_lo;
        if (ny & 1)
            acc_add(hi, vh, vl);
        else
            acc_add(hr, vh, vl);
    }
}

// acc += H * v (complex).
__device__ __forceinline__ void mac(AccD& acc, double hr, double hi, double2 v) {
    acc.re = fma(hr, v.x, fma(-hi, v.y, acc.re));
    acc.im = fma(hr, v.y, fma(hi, v.x, acc.im));
}

__device__ __forceinline__ void mac(AccF& acc, F2 hr, F2 hi, float4 v) {
    const F2 vr{v.x, v.y}, vi{v.z, v.w};
    float p, q;
    df_mul(hr, vr, p, q);
    acc_add(acc.re, p, q);
    df_mul(hi, vi, p, q);
    acc_add(acc.re, -p, -q);
    df_mul(hr, vi, p, q);
    acc_add(acc.im, p, q);
    df_mul(hi, vr, p, q);
    acc_add(acc.im, p, q);
}

// ---------------------------------------------------------------------------
// Kernel arguments shared by the pair kernels.
// ---------------------------------------------------------------------------
struct PairArgs {
    const void* groups;
    const uint64_t* ghash;
    const void* terms;
    const void* terms_f;
    const uint64_t* gkeys;
    Table gtable;
    int n_groups;
    int maxpop;
    const uint64_t* keys;
    const uint64_t* khash;
    Table ktable;
    const uint64_t* sig;
    int sig_filter;
    int64_t M;
    int per_chunk;
};

PairArgs make_args(const HamDev& H, const SampleDev& S, const Plan& P) {
    PairArgs a;
    a.groups = H.groups;
    a.ghash = H.group_hash;
    a.terms = H.terms;
    a.terms_f = H.terms_f;
    a.gkeys = H.group_keys;
    a.gtable = H.group_table;
    a.n_groups = static_cast<int>(H.n_groups);
    a.maxpop = H.maxpop;
    a.keys = S.keys;
    a.khash = S.hash;
    a.ktable = S.table;
    a.sig = S.sig;
    a.sig_filter = P.sig_filter ? 1 : 0;
    a.M = S.n;
    a.per_chunk = P.per_chunk;
    return a;
}

// Visit every coupled pair (row, j) of the row owned by this lane inside the
// chunk; on_hit(g, xy_of_group, xprime, j, term_begin, term_end).
template <int W, class OnHit>
__device__ __forceinline__ void visit_terms(const PairArgs& A, const uint64_t* __restrict__ sig_lds,
                                            bool live, const uint64_t (&x)[W], uint64_t hx,
                                            int chunk, OnHit&& on_hit) {
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(A.groups);
    const uint64_t* __restrict__ ghash = A.ghash;
    const int g0 = chunk * A.per_chunk;
    const int g1 = min(A.n_groups, g0 + A.per_chunk);
    for (int g = g0; g < g1; ++g) {
        const GroupRec<W> gr = groups[g];
        const uint64_t gh = ghash[g];
        uint64_t xp[W];
#pragma unroll
        for (int w = 0; w < W; ++w) xp[w] = x[w] ^ gr.xy[w];
        bool cand = live;
        if (A.sig_filter) cand = cand && sig_ok<W>(sig_lds, xp);
        if (cand) {
            const int j = table_find<W>(A.ktable, A.keys, hx ^ gh, xp);
            if (j >= 0) on_hit(g, gr.xy, xp, j, gr.begin, gr.end);
        }
    }
}

template <int W, class OnHit>
__device__ __forceinline__ void visit_batch(const PairArgs& A, bool live, const uint64_t (&x)[W],
                                            uint64_t hx, int chunk, OnHit&& on_hit) {
    const GroupRec<W>* __restrict__ groups = static_cast<const GroupRec<W>*>(A.groups);
    const uint64_t* __restrict__ keys = A.keys;
    const uint64_t* __restrict__ khash = A.khash;
    const int64_t j0 = static_cast<int64_t>(chunk) * A.per_chunk;
    const int64_t j1 = min(A.M, j0 + A.per_chunk);
    for (int64_t j = j0; j < j1; ++j) {
        uint64_t xj[W], m[W];
        int pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            xj[w] = keys[j * W + w];
            m[w] = x[w] ^ xj[w];
            pc += popc64(m[w]);
        }
        if (live && pc <= A.maxpop) {
            const int g = table_find<W>(A.gtable, A.gkeys, hx ^ khash[j], m);
            if (g >= 0) {
                const GroupRec<W> gr = groups[g];
                on_hit(g, gr.xy, xj, static_cast<int>(j), gr.begin, gr.end);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fused pair kernel: FindCoupledPairs + MatrixElement + row accumulation.
//   forward (ADJ = false): acc_x = sum_{x' coupled} H_xx' a_x'   (ket x')
//   adjoint (ADJ = true):  acc_y = sum_{x coupled}  H_xy v_x     (ket y)
// `vec` is a (forward) or v = w / a (adjoint).
// ---------------------------------------------------------------------------
template <int W, int VARIANT, int PREC, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_pairs(PairArgs A, const double2* __restrict__ vec,
                                                  const float4* __restrict__ vecf,
                                                  void* __restrict__ partial) {
    __shared__ uint64_t sig_lds[kSigWords];
    if (VARIANT == 0) {
        for (int t = threadIdx.x; t < kSigWords; t += kBlock) sig_lds[t] = A.sig[t];
        __syncthreads();
    }
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool live = row < A.M;
    const int chunk = blockIdx.y;
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = live ? A.keys[row * W + w] : 0ull;
    const uint64_t hx = live ? A.khash[row] : 0ull;

    if (PREC == 0) {
        const TermRec<W>* __restrict__ terms = static_cast<const TermRec<W>*>(A.terms);
        AccD acc;
        auto hit = [&](int, const uint64_t* gxy, const uint64_t* xp, int j, int b, int e) {
            double hr, hi;
            melem_f64<W>(terms, b, e, gxy, ADJ ? x : xp, hr, hi);
            mac(acc, hr, hi, vec[j]);
        };
        if (VARIANT == 0)
            visit_terms<W>(A, sig_lds, live, x, hx, chunk, hit);
        else
            visit_batch<W>(A, live, x, hx, chunk, hit);
        if (live) static_cast<double2*>(partial)[chunk * A.M + row] = make_double2(acc.re, acc.im);
    } else {
        const TermRecF<W>* __restrict__ terms = static_cast<const TermRecF<W>*>(A.terms_f);
        AccF acc;
        auto hit = [&](int, const uint64_t* gxy, const uint64_t* xp, int j, int b, int e) {
            F2 hr, hi;
            melem_f32<W>(terms, b, e, gxy, ADJ ? x : xp, hr, hi);
            mac(acc, hr, hi, vecf[j]);
        };
        if (VARIANT == 0)
            visit_terms<W>(A, sig_lds, live, x, hx, chunk, hit);
        else
            visit_batch<W>(A, live, x, hx, chunk, hit);
        if (live)
            static_cast<float4*>(partial)[chunk * A.M + row] =
                make_float4(acc.re.s, acc.re.c, acc.im.s, acc.im.c);
    }
}

// Count coupled pairs per (row, chunk): counts[row * chunks + chunk].
template <int W, int VARIANT>
__global__ __launch_bounds__(kBlock) void k_count(PairArgs A, int chunks, int32_t* __restrict__ counts) {
    __shared__ uint64_t sig_lds[kSigWords];
    if (VARIANT == 0) {
        for (int t = threadIdx.x; t < kSigWords; t += kBlock) sig_lds[t] = A.sig[t];
        __syncthreads();
    }
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool live = row < A.M;
    const int chunk = blockIdx.y;
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = live ? A.keys[row * W + w] : 0ull;
    const uint64_t hx = live ? A.khash[row] : 0ull;
    int n = 0;
    auto hit = [&](int, const uint64_t*, const uint64_t*, int, int, int) { ++n; };
    if (VARIANT == 0)
        visit_terms<W>(A, sig_lds, live, x, hx, chunk, hit);
    else
        visit_batch<W>(A, live, x, hx, chunk, hit);
    if (live) counts[row * chunks + chunk] = n;
}

// Write the pairs of (row, chunk) at offsets[row * chunks + chunk]:
// key = (row << jbits) | j, value = group id.
template <int W, int VARIANT>
__global__ __launch_bounds__(kBlock) void k_fill(PairArgs A, int chunks, int jbits,
                                                 const int64_t* __restrict__ offsets,
                                                 uint64_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
    __shared__ uint64_t sig_lds[kSigWords];
    if (VARIANT == 0) {
        for (int t = threadIdx.x; t < kSigWords; t += kBlock) sig_lds[t] = A.sig[t];
        __syncthreads();
    }
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool live = row < A.M;
    const int chunk = blockIdx.y;
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = live ? A.keys[row * W + w] : 0ull;
    const uint64_t hx = live ? A.khash[row] : 0ull;
    int64_t pos = live ? offsets[row * chunks + chunk] : 0;
    auto hit = [&](int g, const uint64_t*, const uint64_t*, int j, int, int) {
        pkey[pos] = (static_cast<uint64_t>(row) << jbits) | static_cast<uint64_t>(j);
        pval[pos] = static_cast<uint32_t>(g);
        ++pos;
    };
    if (VARIANT == 0)
        visit_terms<W>(A, sig_lds, live, x, hx, chunk, hit);
    else
        visit_batch<W>(A, live, x, hx, chunk, hit);
}

// ---------------------------------------------------------------------------
// Sample preparation.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_sample_hash(const uint64_t* __restrict__ keys, int64_t n,
                                                        const uint64_t* __restrict__ R, int n_qubits,
                                                        uint64_t* __restrict__ hash,
                                                        uint32_t* __restrict__ err) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    uint64_t h = 0;
    bool bad = false;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t v = keys[i * W + w];
        const int valid = n_qubits - 64 * w;
        if (valid < 64) {
            const uint64_t allowed = valid <= 0 ? 0ull : ((1ull << valid) - 1ull);
            bad = bad || (v & ~allowed) != 0ull;
            v &= allowed;
        }
        while (v) {
            const int q = __ffsll(static_cast<unsigned long long>(v)) - 1;
            h ^= R[64 * w + q];
            v &= v - 1ull;
        }
    }
    hash[i] = h;
    if (bad) atomicOr(err, static_cast<uint32_t>(kErrBits));
}

__global__ __launch_bounds__(kBlock) void k_table_insert(const uint64_t* __restrict__ hash, int64_t n,
                                                         uint32_t* __restrict__ slots, Table T) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t h = hash[i];
    uint32_t s = static_cast<uint32_t>(h) & T.mask;
    const uint32_t fp = static_cast<uint32_t>(h >> T.fpshift);
    const uint32_t v = (fp << T.ibits) | static_cast<uint32_t>(i + 1);
    while (atomicCAS(slots + s, 0u, v) != 0u) s = (s + 1u) & T.mask;
}

// Duplicate check (every key must find itself) and the signature bitmap of
// (popcount on even qubits, popcount on odd qubits) over U.
template <int W>
__global__ __launch_bounds__(kBlock) void k_sample_verify(const uint64_t* __restrict__ keys,
                                                          const uint64_t* __restrict__ hash, int64_t n,
                                                          Table T, uint64_t* __restrict__ sig,
                                                          uint32_t* __restrict__ err) {
    __shared__ unsigned long long lsig[kSigWords];
    for (int t = threadIdx.x; t < kSigWords; t += kBlock) lsig[t] = 0ull;
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) {
        uint64_t k[W];
        int pa = 0, pb = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            k[w] = keys[i * W + w];
            pa += popc64(k[w] & kEven);
            pb += popc64(k[w] & kOdd);
        }
        const int j = table_find<W>(T, keys, hash[i], k);
        if (j != static_cast<int>(i)) atomicOr(err, static_cast<uint32_t>(kErrDup));
        atomicOr(&lsig[2 * pa + (pb >> 6)], 1ull << (pb & 63));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSigWords; t += kBlock)
        if (lsig[t]) atomicOr(reinterpret_cast<unsigned long long*>(sig + t), lsig[t]);
}

// ---------------------------------------------------------------------------
// Block reductions (fixed tree, deterministic).
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*lds)[kBlock]) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < K; ++k) lds[k][threadIdx.x] += lds[k][threadIdx.x + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = lds[k][0];
    __syncthreads();
}

constexpr int kRedBlocks = 256;   // fixed partition of reductions over U

__global__ __launch_bounds__(kBlock) void k_minmax_partial(const double2* __restrict__ L, int64_t n,
                                                           double* __restrict__ part) {
    __shared__ double lds[2][kBlock];
    double mx = -INFINITY, mn = INFINITY;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(kRedBlocks) * kBlock) {
        const double r = L[i].x;
        mx = fmax(mx, r);
        mn = fmin(mn, r);
    }
    lds[0][threadIdx.x] = mx;
    lds[1][threadIdx.x] = mn;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            lds[0][threadIdx.x] = fmax(lds[0][threadIdx.x], lds[0][threadIdx.x + s]);
            lds[1][threadIdx.x] = fmin(lds[1][threadIdx.x], lds[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lds[0][0];
        part[2 * blockIdx.x + 1] = lds[1][0];
    }
}

__device__ __forceinline__ float4 split_c(double re, double im) {
    const float rh = static_cast<float>(re);
    const float ih = static_cast<float>(im);
    return make_float4(rh, static_cast<float>(re - static_cast<double>(rh)), ih,
                       static_cast<float>(im - static_cast<double>(ih)));
}

// a = exp(L - c), b = exp(c - L) (FP64 and, if fp32, hi/lo float pairs).
__global__ __launch_bounds__(kBlock) void k_amp_prep(const double2* __restrict__ L, int64_t n,
                                                     const double* __restrict__ part, int fp32,
                                                     double2* __restrict__ a, double2* __restrict__ b,
                                                     float4* __restrict__ af, float4* __restrict__ bf,
                                                     double* __restrict__ shift, uint32_t* __restrict__ err) {
    __shared__ double cmax;
    if (threadIdx.x == 0) {
        double mx = -INFINITY, mn = INFINITY;
        for (int k = 0; k < kRedBlocks; ++k) {
            mx = fmax(mx, part[2 * k]);
            mn = fmin(mn, part[2 * k + 1]);
        }
        cmax = mx;
        if (blockIdx.x == 0) {
            *shift = mx;
            if (!(mx - mn <= 60.0) && fp32) atomicOr(err, static_cast<uint32_t>(kErrRange));
            if (!isfinite(mx) || !isfinite(mn)) atomicOr(err, static_cast<uint32_t>(kErrRange));
        }
    }
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const double2 l = L[i];
    double s, c;
    sincos(l.y, &s, &c);
    const double ea = exp(l.x - cmax);
    const double eb = exp(cmax - l.x);
    a[i] = make_double2(ea * c, ea * s);
    b[i] = make_double2(eb * c, -eb * s);
    if (fp32) {
        af[i] = split_c(ea * c, ea * s);
        bf[i] = split_c(eb * c, -eb * s);
    }
}

// v = w b (counts) or conj(a) (|psi|^2 weights, since |a|^2 / a = conj(a)).
__global__ __launch_bounds__(kBlock) void k_adj_vec(const double2* __restrict__ a, const double2* __restrict__ b,
                                                    const double* __restrict__ weights, int64_t n, int fp32,
                                                    double2* __restrict__ v, float4* __restrict__ vf) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double2 r;
    if (weights) {
        const double w = weights[i];
        r = make_double2(w * b[i].x, w * b[i].y);
    } else {
        r = make_double2(a[i].x, -a[i].y);
    }
    v[i] = r;
    if (fp32) vf[i] = split_c(r.x, r.y);
}

// Sum the chunk partials of a row in chunk order and multiply by b_row.
__global__ __launch_bounds__(kBlock) void k_finish_f64(const double2* __restrict__ partial, int chunks,
                                                       int64_t n, const double2* __restrict__ b,
                                                       double2* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < chunks; ++c) {
        const double2 p = partial[c * n + i];
        re += p.x;
        im += p.y;
    }
    const double2 bi = b[i];
    out[i] = make_double2(re * bi.x - im * bi.y, re * bi.y + im * bi.x);
}

__global__ __launch_bounds__(kBlock) void k_finish_f32(const float4* __restrict__ partial, int chunks,
                                                       int64_t n, const float4* __restrict__ bf,
                                                       double2* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    F2 re{0.f, 0.f}, im{0.f, 0.f};
    for (int c = 0; c < chunks; ++c) {
        const float4 p = partial[c * n + i];
        acc_add(re, p.x, p.y);
        acc_add(im, p.z, p.w);
    }
    AccF r;
    mac(r, re, im, bf[i]);
    out[i] = make_double2(static_cast<double>(r.re.s) + static_cast<double>(r.re.c),
                          static_cast<double>(r.im.s) + static_cast<double>(r.im.c));
}

// Adjoint finish: S_y = sum of partials; G_y = (a_y S_y - w_y E_y) / W;
// grad_y = ge conj(G_y) [+ 2 w~_y Re(conj(ge)(E_y - E)) for |psi|^2 weights].
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_adj_finish(const void* __restrict__ partial, int chunks, int64_t n,
                                                       const double2* __restrict__ a,
                                                       const float4* __restrict__ af,
                                                       const double2* __restrict__ eloc,
                                                       const double* __restrict__ weights,
                                                       const double* __restrict__ stats,
                                                       const double* __restrict__ shift, double2 ge,
                                                       double2* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double sr, si;
    if (PREC == 0) {
        sr = 0.0;
        si = 0.0;
        for (int c = 0; c < chunks; ++c) {
            const double2 p = static_cast<const double2*>(partial)[c * n + i];
            sr += p.x;
            si += p.y;
        }
        const double2 ai = a[i];
        const double tr = sr * ai.x - si * ai.y;
        si = sr * ai.y + si * ai.x;
        sr = tr;
    } else {
        F2 re{0.f, 0.f}, im{0.f, 0.f};
        for (int c = 0; c < chunks; ++c) {
            const float4 p = static_cast<const float4*>(partial)[c * n + i];
            acc_add(re, p.x, p.y);
            acc_add(im, p.z, p.w);
        }
        AccF r;
        mac(r, re, im, af[i]);
        sr = static_cast<double>(r.re.s) + static_cast<double>(r.re.c);
        si = static_cast<double>(r.im.s) + static_cast<double>(r.im.c);
    }
    // raw weight of the row relative to the normaliser stats[3]
    double wrow;
    double inv_total;
    if (weights) {
        wrow = weights[i];
        inv_total = 1.0 / stats[3];
    } else {
        // |psi|^2 weights are used relative to exp(2c): v = conj(a) carried |a|^2 / a.
        const double2 ai = a[i];
        wrow = ai.x * ai.x + ai.y * ai.y;
        inv_total = exp(2.0 * shift[0]) / stats[3];
    }
    const double2 e = eloc[i];
    const double gr = (sr - wrow * e.x) * inv_total;
    const double gi = (si - wrow * e.y) * inv_total;
    // ge * conj(G)
    double outr = ge.x * gr + ge.y * gi;
    const double outi = ge.y * gr - ge.x * gi;
    if (!weights) {
        const double dre = e.x - stats[0], dim = e.y - stats[1];
        outr += 2.0 * wrow * inv_total * (ge.x * dre + ge.y * dim);
    }
    out[i] = make_double2(outr, outi);
}

// ---------------------------------------------------------------------------
// Weighted energy and variance (FP64, fixed partition).
//   pass 1: partials of (sum w, sum w Re E, sum w Im E)
//   pass 2: E = ..., partials of sum w |E_loc - E|^2
//   pass 3: Var
// Weights are the caller's (validated: finite, >= 0) or |a|^2 = |psi|^2 e^{-2c}.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double row_weight(const double* weights, const double2* L, int64_t i,
                                             double c, bool& bad) {
    if (weights) {
        const double w = weights[i];
        if (!(w >= 0.0) || !isfinite(w)) bad = true;
        return w;
    }
    return exp(2.0 * (L[i].x - c));
}

__global__ __launch_bounds__(kBlock) void k_energy_p1(const double2* __restrict__ eloc,
                                                      const double2* __restrict__ L,
                                                      const double* __restrict__ weights,
                                                      const double* __restrict__ shift, int64_t n,
                                                      double* __restrict__ part, uint32_t* __restrict__ err) {
    __shared__ double lds[3][kBlock];
    const double c = shift[0];
    double v[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(kRedBlocks) * kBlock) {
        const double w = row_weight(weights, L, i, c, bad);
        const double2 e = eloc[i];
        v[0] += w;
        v[1] += w * e.x;
        v[2] += w * e.y;
    }
    if (bad) atomicOr(err, static_cast<uint32_t>(kErrWeights));
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_mid(const double* __restrict__ part,
                                                       const double* __restrict__ weights,
                                                       const double* __restrict__ shift,
                                                       double* __restrict__ stats, double* __restrict__ scal,
                                                       uint32_t* __restrict__ err) {
    __shared__ double lds[3][kBlock];
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < kRedBlocks; k += kBlock) {
        v[0] += part[3 * k];
        v[1] += part[3 * k + 1];
        v[2] += part[3 * k + 2];
    }
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        const double tot = v[0];
        if (!(tot > 0.0) || !isfinite(tot)) atomicOr(err, static_cast<uint32_t>(kErrWeights));
        const double er = v[1] / tot, ei = v[2] / tot;
        stats[0] = er;
        stats[1] = ei;
        stats[3] = weights ? tot : tot * exp(2.0 * shift[0]);
        scal[0] = er;
        scal[1] = ei;
        scal[2] = tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_p2(const double2* __restrict__ eloc,
                                                      const double2* __restrict__ L,
                                                      const double* __restrict__ weights,
                                                      const double* __restrict__ shift, int64_t n,
                                                      const double* __restrict__ scal, double* __restrict__ part) {
    __shared__ double lds[1][kBlock];
    const double c = shift[0];
    const double er = scal[0], ei = scal[1];
    double v[1] = {0.0};
    bool bad = false;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(kRedBlocks) * kBlock) {
        const double w = row_weight(weights, L, i, c, bad);
        const double2 e = eloc[i];
        const double dr = e.x - er, di = e.y - ei;
        v[0] += w * (dr * dr + di * di);
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_energy_p3(const double* __restrict__ part,
                                                      const double* __restrict__ scal,
                                                      double* __restrict__ stats) {
    __shared__ double lds[1][kBlock];
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < kRedBlocks; k += kBlock) v[0] += part[k];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) stats[2] = v[0] / scal[2];
}

// ---------------------------------------------------------------------------
// Exclusive scan int32 -> int64 (3-level, blocks of 2048 elements).
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_tile(const T* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ out, int64_t* __restrict__ sums) {
    __shared__ int64_t lds[kBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k;
        v[k] = idx < n ? static_cast<int64_t>(in[idx]) : 0;
        run += v[k];
    }
    lds[threadIdx.x] = run;
    __syncthreads();
    for (int s = 1; s < kBlock; s <<= 1) {
        const int64_t t = threadIdx.x >= s ? lds[threadIdx.x - s] : 0;
        __syncthreads();
        lds[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t pre = lds[threadIdx.x] - run;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k;
        if (idx < n) out[idx] = pre;
        pre += v[k];
    }
    if (threadIdx.x == kBlock - 1 && sums) sums[blockIdx.x] = lds[kBlock - 1];
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int64_t* __restrict__ out, int64_t n,
                                                     const int64_t* __restrict__ sums) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) out[i] += sums[i / kScanTile];
}

// total = out[n-1] + in[n-1] written to out[n]
template <class T>
__global__ void k_scan_total(const T* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    out[n] = n > 0 ? out[n - 1] + static_cast<int64_t>(in[n - 1]) : 0;
}

template <class T>
hipError_t scan_rec(const T* in, int64_t n, int64_t* out, int64_t* scratch, hipStream_t st) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        hipLaunchKernelGGL(k_scan_tile<T>, dim3(1), dim3(kBlock), 0, st, in, n, out,
                           static_cast<int64_t*>(nullptr));
        return hipGetLastError();
    }
    int64_t* sums = scratch;
    int64_t* sums_scan = scratch + tiles;
    int64_t* next = scratch + 2 * tiles;
    hipLaunchKernelGGL(k_scan_tile<T>, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, st, in, n, out, sums);
    hipError_t e = scan_rec<int64_t>(sums, tiles, sums_scan, next, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       out, n, sums_scan);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, uint32 value), 8 bits per pass.
// hist layout digit-major [256][tiles] so that an exclusive scan yields the
// destination of every (digit, tile) bucket in stable order.
// ---------------------------------------------------------------------------
constexpr int kSortItems = 8;
constexpr int kSortTile = kBlock * kSortItems;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                       uint32_t* __restrict__ hist, int64_t tiles) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + k * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ vals, int64_t n,
                                                          int shift, const int64_t* __restrict__ offs,
                                                          int64_t tiles, uint64_t* __restrict__ okeys,
                                                          uint32_t* __restrict__ ovals) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    __shared__ int64_t base_off[256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    run[threadIdx.x] = 0;
    base_off[threadIdx.x] = offs[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x];
    for (int w = 0; w < kBlock / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + k * kBlock + threadIdx.x;
        const bool valid = idx < n;
        uint64_t key = 0;
        uint32_t val = 0;
        uint32_t d = 255u;
        if (valid) {
            key = keys[idx];
            val = vals[idx];
            d = static_cast<uint32_t>((key >> shift) & 255u);
        }
        // lanes of this wave holding the same digit
        uint64_t same = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t wrank = static_cast<uint32_t>(__popcll(same & lt));
        if (wrank == 0) wcnt[wave][d] = static_cast<uint32_t>(__popcll(same));
        __syncthreads();
        uint32_t before = run[d];
        for (int w = 0; w < wave; ++w) before += wcnt[w][d];
        if (valid) {
            const int64_t dst = base_off[d] + before + wrank;
            okeys[dst] = key;
            ovals[dst] = val;
        }
        __syncthreads();
        {
            uint32_t tot = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                tot += wcnt[w][threadIdx.x];
                wcnt[w][threadIdx.x] = 0;
            }
            run[threadIdx.x] += tot;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_split_pairs(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals, int64_t n, int jbits,
                                                        int32_t* __restrict__ pi, int32_t* __restrict__ pj,
                                                        int32_t* __restrict__ pg) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= n) return;
    const uint64_t k = keys[t];
    pi[t] = static_cast<int32_t>(k >> jbits);
    pj[t] = static_cast<int32_t>(k & ((1ull << jbits) - 1ull));
    pg[t] = static_cast<int32_t>(vals[t]);
}

// MatrixElement for given sample pairs (ket x_j).
template <int W>
__global__ __launch_bounds__(kBlock) void k_pair_elements(PairArgs A, int64_t n, const int32_t* __restrict__ pi,
                                                          const int32_t* __restrict__ pj,
                                                          double2* __restrict__ out, uint32_t* __restrict__ err) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= n) return;
    const int64_t i = pi[t], j = pj[t];
    if (i < 0 || j < 0 || i >= A.M || j >= A.M) {
        atomicOr(err, static_cast<uint32_t>(kErrIndex));
        out[t] = make_double2(0.0, 0.0);
        return;
    }
    uint64_t xi[W], xj[W], m[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        xi[w] = A.keys[i * W + w];
        xj[w] = A.keys[j * W + w];
        m[w] = xi[w] ^ xj[w];
    }
    const int g = table_find<W>(A.gtable, A.gkeys, A.khash[i] ^ A.khash[j], m);
    double hr = 0.0, hi = 0.0;
    if (g >= 0) {
        const GroupRec<W> gr = static_cast<const GroupRec<W>*>(A.groups)[g];
        melem_f64<W>(static_cast<const TermRec<W>*>(A.terms), gr.begin, gr.end, gr.xy, xj, hr, hi);
    }
    out[t] = make_double2(hr, hi);
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

template <int W, int VARIANT, int PREC, bool ADJ>
hipError_t launch_pairs_t(const PairArgs& A, const Plan& P, const double2* vec, const float4* vecf,
                          void* partial, hipStream_t st) {
    dim3 grid(blocks_for(A.M), static_cast<unsigned>(P.chunks));
    hipLaunchKernelGGL((k_pairs<W, VARIANT, PREC, ADJ>), grid, dim3(kBlock), 0, st, A, vec, vecf, partial);
    return hipGetLastError();
}

template <bool ADJ>
hipError_t dispatch_pairs(int W, int variant, int precision, const PairArgs& A, const Plan& P,
                          const double2* vec, const float4* vecf, void* partial, hipStream_t st) {
#define ELOC_CASE(w, v, p)                                                               \
    if (W == w && variant == v && precision == p)                                       \
        return launch_pairs_t<w, v, p, ADJ>(A, P, vec, vecf, partial, st);
    ELOC_CASE(1, 0, 0) ELOC_CASE(1, 0, 1) ELOC_CASE(1, 1, 0) ELOC_CASE(1, 1, 1)
    ELOC_CASE(2, 0, 0) ELOC_CASE(2, 0, 1) ELOC_CASE(2, 1, 0) ELOC_CASE(2, 1, 1)
#undef ELOC_CASE
    return hipErrorInvalidValue;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_sample_hash(int W, const uint64_t* keys, int64_t n, const uint64_t* R, int n_qubits,
                              uint64_t* hash, uint32_t* err, hipStream_t st) {
    if (W == 1)
        hipLaunchKernelGGL(k_sample_hash<1>, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, n, R, n_qubits, hash, err);
    else
        hipLaunchKernelGGL(k_sample_hash<2>, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, n, R, n_qubits, hash, err);
    return hipGetLastError();
}

hipError_t launch_table_insert(int, const uint64_t* hash, int64_t n, uint32_t* slots, const Table& T,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_table_insert, dim3(blocks_for(n)), dim3(kBlock), 0, st, hash, n, slots, T);
    return hipGetLastError();
}

hipError_t launch_sample_verify(int W, const SampleDev& S, uint64_t* sig, uint32_t* err, hipStream_t st) {
    if (W == 1)
        hipLaunchKernelGGL(k_sample_verify<1>, dim3(blocks_for(S.n)), dim3(kBlock), 0, st, S.keys, S.hash, S.n,
                           S.table, sig, err);
    else
        hipLaunchKernelGGL(k_sample_verify<2>, dim3(blocks_for(S.n)), dim3(kBlock), 0, st, S.keys, S.hash, S.n,
                           S.table, sig, err);
    return hipGetLastError();
}

hipError_t launch_amp_prep(const double2* logpsi, int64_t n, bool fp32, double2* a, double2* b, float4* af,
                           float4* bf, double* shift, double* scratch, uint32_t* err, hipStream_t st) {
    hipLaunchKernelGGL(k_minmax_partial, dim3(kRedBlocks), dim3(kBlock), 0, st, logpsi, n, scratch);
    hipLaunchKernelGGL(k_amp_prep, dim3(blocks_for(n)), dim3(kBlock), 0, st, logpsi, n, scratch, fp32 ? 1 : 0, a,
                       b, af, bf, shift, err);
    return hipGetLastError();
}

hipError_t launch_adj_vec(const double2* a, const double2* b, const double* weights, int64_t n, bool fp32,
                          double2* v, float4* vf, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_vec, dim3(blocks_for(n)), dim3(kBlock), 0, st, a, b, weights, n, fp32 ? 1 : 0, v, vf);
    return hipGetLastError();
}

hipError_t launch_pairs(bool adjoint, int variant, int precision, const HamDev& H, const SampleDev& S,
                        const Plan& P, const double2* vec, const float4* vecf, void* partial, hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    if (adjoint) return dispatch_pairs<true>(H.W, variant, precision, A, P, vec, vecf, partial, st);
    return dispatch_pairs<false>(H.W, variant, precision, A, P, vec, vecf, partial, st);
}

hipError_t launch_finish(int precision, int64_t n, const Plan& P, const void* partial, const double2* b,
                         const float4* bf, double2* out, hipStream_t st) {
    if (precision == 0)
        hipLaunchKernelGGL(k_finish_f64, dim3(blocks_for(n)), dim3(kBlock), 0, st,
                           static_cast<const double2*>(partial), P.chunks, n, b, out);
    else
        hipLaunchKernelGGL(k_finish_f32, dim3(blocks_for(n)), dim3(kBlock), 0, st,
                           static_cast<const float4*>(partial), P.chunks, n, bf, out);
    return hipGetLastError();
}

hipError_t launch_adj_finish(int precision, int64_t n, const Plan& P, const void* partial, const double2* a,
                             const float4* af, const double2* eloc, const double* weights, const double* stats,
                             const double* shift, double2 ge, double2* out, hipStream_t st) {
    if (precision == 0)
        hipLaunchKernelGGL(k_adj_finish<0>, dim3(blocks_for(n)), dim3(kBlock), 0, st, partial, P.chunks, n, a, af,
                           eloc, weights, stats, shift, ge, out);
    else
        hipLaunchKernelGGL(k_adj_finish<1>, dim3(blocks_for(n)), dim3(kBlock), 0, st, partial, P.chunks, n, a, af,
                           eloc, weights, stats, shift, ge, out);
    return hipGetLastError();
}

hipError_t launch_energy(const double2* eloc, const double2* logpsi, const double* weights, const double* shift,
                         int64_t n, double* stats, double* scratch, uint32_t* err, hipStream_t st) {
    double* part = scratch;                 // 3 * kRedBlocks
    double* scal = scratch + 3 * kRedBlocks;  // 3
    hipLaunchKernelGGL(k_energy_p1, dim3(kRedBlocks), dim3(kBlock), 0, st, eloc, logpsi, weights, shift, n, part, err);
    hipLaunchKernelGGL(k_energy_mid, dim3(1), dim3(kBlock), 0, st, part, weights, shift, stats, scal, err);
    hipLaunchKernelGGL(k_energy_p2, dim3(kRedBlocks), dim3(kBlock), 0, st, eloc, logpsi, weights, shift, n, scal,
                       part);
    hipLaunchKernelGGL(k_energy_p3, dim3(1), dim3(kBlock), 0, st, part, scal, stats);
    return hipGetLastError();
}

int64_t energy_scratch_len() { return 3 * kRedBlocks + 4; }
int64_t amp_scratch_len() { return 2 * kRedBlocks; }

hipError_t launch_pairs_count(int variant, const HamDev& H, const SampleDev& S, const Plan& P, int32_t* counts,
                              hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    dim3 grid(blocks_for(S.n), static_cast<unsigned>(P.chunks));
    if (H.W == 1 && variant == 0) hipLaunchKernelGGL((k_count<1, 0>), grid, dim3(kBlock), 0, st, A, P.chunks, counts);
    else if (H.W == 1) hipLaunchKernelGGL((k_count<1, 1>), grid, dim3(kBlock), 0, st, A, P.chunks, counts);
    else if (variant == 0) hipLaunchKernelGGL((k_count<2, 0>), grid, dim3(kBlock), 0, st, A, P.chunks, counts);
    else hipLaunchKernelGGL((k_count<2, 1>), grid, dim3(kBlock), 0, st, A, P.chunks, counts);
    return hipGetLastError();
}

hipError_t launch_pairs_fill(int variant, const HamDev& H, const SampleDev& S, const Plan& P, int jbits,
                             const int64_t* offsets, uint64_t* pkey, uint32_t* pval, hipStream_t st) {
    const PairArgs A = make_args(H, S, P);
    dim3 grid(blocks_for(S.n), static_cast<unsigned>(P.chunks));
    if (H.W == 1 && variant == 0)
        hipLaunchKernelGGL((k_fill<1, 0>), grid, dim3(kBlock), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
    else if (H.W == 1)
        hipLaunchKernelGGL((k_fill<1, 1>), grid, dim3(kBlock), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
    else if (variant == 0)
        hipLaunchKernelGGL((k_fill<2, 0>), grid, dim3(kBlock), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
    else
        hipLaunchKernelGGL((k_fill<2, 1>), grid, dim3(kBlock), 0, st, A, P.chunks, jbits, offsets, pkey, pval);
    return hipGetLastError();
}

int64_t scan_scratch_len(int64_t n) {
    int64_t total = 0;
    while (n > kScanTile) {
        const int64_t tiles = (n + kScanTile - 1) / kScanTile;
        total += 2 * tiles;
        n = tiles;
    }
    return total + 1;
}

hipError_t launch_scan_i32(const int32_t* in, int64_t n, int64_t* out, int64_t* scratch, hipStream_t st) {
    hipError_t e = scan_rec<int32_t>(in, n, out, scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_total<int32_t>, dim3(1), dim3(1), 0, st, in, n, out);
    return hipGetLastError();
}

int64_t radix_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

hipError_t launch_radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                                   int64_t n, int end_bit, uint32_t* hist, int64_t* hist_off,
                                   int64_t* scan_scratch, int* result_in_alt, hipStream_t st) {
    const int64_t tiles = radix_tiles(n);
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys_alt;
    uint32_t* vb = vals_alt;
    int flips = 0;
    for (int shift = 0; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, st, ka, n, shift, hist,
                           tiles);
        hipError_t e = scan_rec<uint32_t>(hist, 256 * tiles, hist_off, scan_scratch, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, st, ka, va, n, shift,
                           hist_off, tiles, kb, vb);
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
        ++flips;
    }
    *result_in_alt = flips & 1;
    return hipGetLastError();
}

hipError_t launch_split_pairs(const uint64_t* keys, const uint32_t* vals, int64_t n, int jbits, int32_t* pi,
                              int32_t* pj, int32_t* pg, hipStream_t st) {
    hipLaunchKernelGGL(k_split_pairs, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, vals, n, jbits, pi, pj, pg);
    return hipGetLastError();
}

hipError_t launch_pair_elements(const HamDev& H, const SampleDev& S, int64_t n, const int32_t* pi,
                                const int32_t* pj, double2* out, uint32_t* err, hipStream_t st) {
    Plan P;
    const PairArgs A = make_args(H, S, P);
    if (H.W == 1)
        hipLaunchKernelGGL(k_pair_elements<1>, dim3(blocks_for(n)), dim3(kBlock), 0, st, A, n, pi, pj, out, err);
    else
        hipLaunchKernelGGL(k_pair_elements<2>, dim3(blocks_for(n)), dim3(kBlock), 0, st, A, n, pi, pj, out, err);
    return hipGetLastError();
}

}  // namespace eloc
