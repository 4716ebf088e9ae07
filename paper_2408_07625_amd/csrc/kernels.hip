// HIP kernels for gfx950 (CDNA4, wave64) around the pair kernels of
// pairs.hip: sample preparation (linear hash, membership table, duplicate
// and bit checks), amplitudes relative to the largest |psi|, per-row
// combination of chunk partials, the weighted energy / variance reductions,
// an exclusive scan, a stable LSD radix sort, and the parallel construction
// of the prefix trees used by LoopOverTrie.
#include "device.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

namespace eloc {

namespace {

constexpr int kBlock = 256;
// ---------------------------------------------------------------------------
// Sample preparation.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_sample_hash(const uint64_t* __restrict__ keys, int64_t n,
                                                        const uint64_t* __restrict__ R, int n_qubits,
                                                        uint64_t* __restrict__ hash, uint32_t* __restrict__ counts,
                                                        uint32_t* __restrict__ err) {
    __shared__ uint32_t lc[64 * W];   // per-qubit counts of set bits in this block
    for (int t = threadIdx.x; t < 64 * W; t += kBlock) lc[t] = 0u;
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) {
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
                atomicAdd(&lc[64 * w + q], 1u);
                v &= v - 1ull;
            }
        }
        hash[i] = h;
        if (bad) atomicOr(err, static_cast<uint32_t>(kErrBits));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * W; t += kBlock)
        if (lc[t]) atomicAdd(counts + t, lc[t]);
}

// Blocked Bloom filter of U for the LoopOverTerms probes: each key sets two
// bits of one 32-bit word, both chosen from the high half of its linear hash.
__global__ __launch_bounds__(kBlock) void k_bloom_build(const uint64_t* __restrict__ hash, int64_t n,
                                                        uint32_t* __restrict__ filt, uint32_t fmask) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t hf = static_cast<uint32_t>(hash[i] >> 32);
    atomicOr(filt + bloom_word(hf, fmask), bloom_bits(hf));
}

// Radius filter of LoopOverTerms: reference key c = per-qubit majority of U
// (rad[0..W-1]), then rad[2] = max over U of |x ^ c|.  A candidate farther
// than that from c is not in U.
template <int W>
__global__ void k_radius_ref(const uint32_t* __restrict__ counts, int64_t n, unsigned long long* __restrict__ rad) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int w = 0; w < W; ++w) {
        uint64_t c = 0;
        for (int q = 0; q < 64; ++q)
            if (2 * static_cast<int64_t>(counts[64 * w + q]) > n) c |= 1ull << q;
        rad[w] = c;
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_radius_max(const uint64_t* __restrict__ keys, int64_t n,
                                                       unsigned long long* __restrict__ rad) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    int d = 0;
    if (i < n) {
#pragma unroll
        for (int w = 0; w < W; ++w) d += popc64(keys[i * W + w] ^ rad[w]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) d = max(d, __shfl_xor(d, m, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(rad + 2, static_cast<unsigned long long>(d));
}

template <int TK>
__global__ __launch_bounds__(kBlock) void k_table_insert(const uint64_t* __restrict__ hash, int64_t n, void* slots,
                                                         Stash* __restrict__ stash, Table T,
                                                         uint32_t* __restrict__ err) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    table_insert_one<TK>(hash, i, slots, stash, T, err, static_cast<uint32_t>(kErrTable));
}

// Duplicate check (every key must find itself) and the signature bitmap of
// (popcount on even qubits, popcount on odd qubits) over U.
template <int W, int TK>
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
        const int j = table_find<TK, W>(T, keys, hash[i], k);
        if (j != static_cast<int>(i)) atomicOr(err, static_cast<uint32_t>(kErrDup));
        atomicOr(&lsig[2 * pa + (pb >> 6)], 1ull << (pb & 63));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSigWords; t += kBlock)
        if (lsig[t]) atomicOr(reinterpret_cast<unsigned long long*>(sig + t), lsig[t]);
}

// Prefilter parameters of U from the signature bitmap (a single set bit:
// U's only (even, odd) popcount signature) and the radius words (majority
// key, largest distance from it; used when under half the qubits).
__global__ void k_sample_params(const uint64_t* __restrict__ sig, const unsigned long long* __restrict__ rad,
                                int n_qubits, SampleParams* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int nsig = 0, first = -1;
    for (int k = 0; k < kSigWords; ++k) {
        const uint64_t v = sig[k];
        if (v && first < 0) first = k;
        nsig += popc64(v);
    }
    SampleParams p;
    p.sig_all = nsig == 1 ? 0 : 1;
    p.sig_pa = 0;
    p.sig_n = 0;
    if (nsig == 1) {
        const int pa = first / 2;
        const int pb = (first % 2) * 64 + (__ffsll(static_cast<unsigned long long>(sig[first])) - 1);
        p.sig_pa = pa;
        p.sig_n = pa + pb;
    }
    const int rmax = static_cast<int>(rad[2]);
    p.rad_max = 2 * rmax < n_qubits ? rmax : 128;
    p.rad_ref[0] = rad[0];
    p.rad_ref[1] = n_qubits > 64 ? rad[1] : 0ull;
    *out = p;
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
            // exp(L - c) and exp(c - L) stay finite and normal over the spread:
            // 60 for the FP32 form, 700 for FP64 (exp overflows past 709.78)
            if (!(mx - mn <= (fp32 ? 60.0 : 700.0))) atomicOr(err, static_cast<uint32_t>(kErrRange));
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
                                                       const double* __restrict__ atotal, double2 ge,
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
    // raw weight of the row relative to the normaliser: the caller's
    // weights over their sum stats[3], or |psi|^2 weights relative to
    // exp(2c) (v = conj(a) carried |a|^2 / a) over the shifted total
    // sum |a|^2, which stays finite for any offset of Re log psi
    double wrow;
    double inv_total;
    if (weights) {
        wrow = weights[i];
        inv_total = 1.0 / stats[3];
    } else {
        const double2 ai = a[i];
        wrow = ai.x * ai.x + ai.y * ai.y;
        inv_total = 1.0 / atotal[0];
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

// Sum of |a_i|^2 = |psi_i|^2 exp(-2c) over U in a fixed partition (the
// |psi|^2 normaliser of the adjoint, relative to exp(2c)).
__global__ __launch_bounds__(kBlock) void k_asum_partial(const double2* __restrict__ a, int64_t n,
                                                         double* __restrict__ part);
__global__ __launch_bounds__(kBlock) void k_asum_total(const double* __restrict__ part, double* __restrict__ total);

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
    block_sum<3, kBlock>(v, lds);
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
    block_sum<3, kBlock>(v, lds);
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
    block_sum<1, kBlock>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_energy_p3(const double* __restrict__ part,
                                                      const double* __restrict__ scal,
                                                      double* __restrict__ stats) {
    __shared__ double lds[1][kBlock];
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < kRedBlocks; k += kBlock) v[0] += part[k];
    block_sum<1, kBlock>(v, lds);
    if (threadIdx.x == 0) stats[2] = v[0] / scal[2];
}

__global__ __launch_bounds__(kBlock) void k_asum_partial(const double2* __restrict__ a, int64_t n,
                                                         double* __restrict__ part) {
    __shared__ double lds[1][kBlock];
    double v[1] = {0.0};
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(kRedBlocks) * kBlock) {
        const double2 ai = a[i];
        v[0] += ai.x * ai.x + ai.y * ai.y;
    }
    block_sum<1, kBlock>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_asum_total(const double* __restrict__ part, double* __restrict__ total) {
    __shared__ double lds[1][kBlock];
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < kRedBlocks; k += kBlock) v[0] += part[k];
    block_sum<1, kBlock>(v, lds);
    if (threadIdx.x == 0) total[0] = v[0];
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

// ---------------------------------------------------------------------------
// Prefix trees: sorted keys with a permutation, then one thread per internal
// node of each segment's radix tree (segment s = leaves [s * per, ...)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_iota(uint32_t* __restrict__ v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) v[i] = static_cast<uint32_t>(i);
}

// out[i] = keys[(perm ? perm[i] : i) * W + w]
__global__ __launch_bounds__(kBlock) void k_gather_word(const uint64_t* __restrict__ keys, int W, int w,
                                                        const uint32_t* __restrict__ perm, int64_t n,
                                                        uint64_t* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t src = perm ? static_cast<int64_t>(perm[i]) : i;
    out[i] = keys[src * W + w];
}

__global__ __launch_bounds__(kBlock) void k_gather_keys(const uint64_t* __restrict__ keys, int W,
                                                        const uint32_t* __restrict__ perm, int64_t n,
                                                        uint64_t* __restrict__ out, int32_t* __restrict__ perm_out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t src = perm[i];
    for (int w = 0; w < W; ++w) out[i * W + w] = keys[src * W + w];
    perm_out[i] = static_cast<int32_t>(src);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_trie_build(const uint64_t* __restrict__ K, int64_t n_total, int64_t per,
                                                       int64_t segs, TNode* __restrict__ nodes,
                                                       uint64_t* __restrict__ nkeys) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t s = t / (per - 1);
    const int64_t i = t % (per - 1);
    if (s >= segs) return;
    const int64_t base = s * per;
    const int64_t n = min(per, n_total - base);
    if (i >= n - 1) return;
    const TNode nd = trie_node<W>(K + base * W, n, i);
    const int64_t o = s * (per - 1) + i;
    nodes[o] = nd;
#pragma unroll
    for (int w = 0; w < W; ++w) nkeys[o * W + w] = K[(base + nd.rep) * W + w];
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// Partition classes of U's rows (hash_part of the unsalted hash).
__global__ void k_class_keys(const uint64_t* __restrict__ hash, int64_t n, int shift, int bits,
                             uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = static_cast<uint64_t>(hash_part(hash[i], shift, bits));
    val[i] = static_cast<uint32_t>(i);
}

// class_off[c] = first sorted position with class >= c; tile_off[c] = tiles
// of kPartRows rows before class c; perm = the sorted row indices.
__global__ void k_class_bounds(const uint64_t* __restrict__ key, const uint32_t* __restrict__ val, int64_t n,
                               int nparts, int32_t* __restrict__ perm, int64_t* __restrict__ class_off,
                               int64_t* __restrict__ tile_off) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = static_cast<int32_t>(val[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t off[kMaxParts + 1];
        for (int c = 0; c <= nparts; ++c) {
            int64_t lo = 0, hi = n;   // first position with key >= c
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (key[mid] < static_cast<uint64_t>(c))
                    lo = mid + 1;
                else
                    hi = mid;
            }
            off[c] = lo;
        }
        int64_t t = 0;
        for (int c = 0; c <= nparts; ++c) {
            class_off[c] = off[c];
            tile_off[c] = t;
            if (c < nparts) t += (off[c + 1] - off[c] + kPartRows - 1) / kPartRows;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_sample_hash(int W, const uint64_t* keys, int64_t n, const uint64_t* R, int n_qubits,
                              uint64_t* hash, uint32_t* counts, uint32_t* err, hipStream_t st) {
    if (W == 1)
        hipLaunchKernelGGL(k_sample_hash<1>, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, n, R, n_qubits, hash,
                           counts, err);
    else
        hipLaunchKernelGGL(k_sample_hash<2>, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, n, R, n_qubits, hash,
                           counts, err);
    return hipGetLastError();
}

hipError_t launch_bloom_build(const uint64_t* hash, int64_t n, uint32_t* filt, uint32_t words, hipStream_t st) {
    hipLaunchKernelGGL(k_bloom_build, dim3(blocks_for(n)), dim3(kBlock), 0, st, hash, n, filt, words - 1u);
    return hipGetLastError();
}

hipError_t launch_sample_radius(int W, const uint64_t* keys, int64_t n, const uint32_t* counts,
                                unsigned long long* rad, hipStream_t st) {
    if (W == 1) {
        hipLaunchKernelGGL(k_radius_ref<1>, dim3(1), dim3(64), 0, st, counts, n, rad);
        hipLaunchKernelGGL(k_radius_max<1>, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, n, rad);
    } else {
        hipLaunchKernelGGL(k_radius_ref<2>, dim3(1), dim3(64), 0, st, counts, n, rad);
        hipLaunchKernelGGL(k_radius_max<2>, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, n, rad);
    }
    return hipGetLastError();
}

hipError_t launch_table_insert(int table_kind, const uint64_t* hash, int64_t n, void* slots, Stash* stash,
                               const Table& T, uint32_t* err, hipStream_t st) {
    const dim3 grid(blocks_for(n)), block(kBlock);
    if (table_kind == kTabNarrow)
        hipLaunchKernelGGL(k_table_insert<kTabNarrow>, grid, block, 0, st, hash, n, slots, stash, T, err);
    else if (table_kind == kTabWide)
        hipLaunchKernelGGL(k_table_insert<kTabWide>, grid, block, 0, st, hash, n, slots, stash, T, err);
    else
        hipLaunchKernelGGL(k_table_insert<kTabVerify>, grid, block, 0, st, hash, n, slots, stash, T, err);
    return hipGetLastError();
}

hipError_t launch_sample_verify(int W, bool narrow, const SampleDev& S, uint64_t* sig, uint32_t* err, hipStream_t st) {
    const dim3 grid(blocks_for(S.n)), block(kBlock);
    if (W == 2)
        hipLaunchKernelGGL((k_sample_verify<2, kTabVerify>), grid, block, 0, st, S.keys, S.hash, S.n, S.table, sig, err);
    else if (narrow)
        hipLaunchKernelGGL((k_sample_verify<1, kTabNarrow>), grid, block, 0, st, S.keys, S.hash, S.n, S.table, sig, err);
    else
        hipLaunchKernelGGL((k_sample_verify<1, kTabWide>), grid, block, 0, st, S.keys, S.hash, S.n, S.table, sig, err);
    return hipGetLastError();
}

hipError_t launch_sample_params(const uint64_t* sig, const unsigned long long* rad, int n_qubits, SampleParams* out,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_sample_params, dim3(1), dim3(64), 0, st, sig, rad, n_qubits, out);
    return hipGetLastError();
}

hipError_t launch_row_classes(const uint64_t* hash, int64_t n, int shift, int bits, uint64_t* key, uint32_t* val,
                              uint64_t* key2, uint32_t* val2, uint32_t* hist, int64_t* hist_off, int64_t* scan,
                              int32_t* perm, int64_t* class_off, int64_t* tile_off, hipStream_t st) {
    if (bits < 1 || bits > kMaxPartBits) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_class_keys, dim3(blocks_for(n)), dim3(kBlock), 0, st, hash, n, shift, bits, key, val);
    int alt = 0;
    const hipError_t e = launch_radix_sort_pairs(key, val, key2, val2, n, 8, hist, hist_off, scan, &alt, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_class_bounds, dim3(blocks_for(n)), dim3(kBlock), 0, st, alt ? key2 : key, alt ? val2 : val, n,
                       1 << bits, perm, class_off, tile_off);
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
                             double* scratch, double2 ge, double2* out, hipStream_t st) {
    // scratch: kRedBlocks partials, then the total of |a|^2
    double* atotal = scratch + kRedBlocks;
    if (!weights) {
        hipLaunchKernelGGL(k_asum_partial, dim3(kRedBlocks), dim3(kBlock), 0, st, a, n, scratch);
        hipLaunchKernelGGL(k_asum_total, dim3(1), dim3(kBlock), 0, st, scratch, atotal);
    }
    if (precision == 0)
        hipLaunchKernelGGL(k_adj_finish<0>, dim3(blocks_for(n)), dim3(kBlock), 0, st, partial, P.chunks, n, a, af,
                           eloc, weights, stats, atotal, ge, out);
    else
        hipLaunchKernelGGL(k_adj_finish<1>, dim3(blocks_for(n)), dim3(kBlock), 0, st, partial, P.chunks, n, a, af,
                           eloc, weights, stats, atotal, ge, out);
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


hipError_t launch_trie_build(int W, const uint64_t* keys, int64_t n_total, int64_t per, TNode* nodes,
                             uint64_t* nkeys, hipStream_t st) {
    if (per < 2 || n_total < 2) return hipSuccess;
    const int64_t segs = (n_total + per - 1) / per;
    const int64_t threads = segs * (per - 1);
    if (W == 1)
        hipLaunchKernelGGL(k_trie_build<1>, dim3(blocks_for(threads)), dim3(kBlock), 0, st, keys, n_total, per, segs,
                           nodes, nkeys);
    else
        hipLaunchKernelGGL(k_trie_build<2>, dim3(blocks_for(threads)), dim3(kBlock), 0, st, keys, n_total, per, segs,
                           nodes, nkeys);
    return hipGetLastError();
}

// Sort keys[n][W] ascending (word W-1 most significant; only the low n_bits
// bits can be set) into sorted[n][W] with perm[i] = source row.
hipError_t launch_sort_keys(int W, int n_bits, const uint64_t* keys, int64_t n, const SortScratch& S,
                            uint64_t* sorted, int32_t* perm, hipStream_t st) {
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(n)), dim3(kBlock), 0, st, S.val, n);
    hipLaunchKernelGGL(k_gather_word, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, W, 0,
                       static_cast<const uint32_t*>(nullptr), n, S.key);
    int alt = 0;
    hipError_t e = launch_radix_sort_pairs(S.key, S.val, S.key2, S.val2, n, W == 1 ? n_bits : 64, S.hist, S.hist_off,
                                           S.scan, &alt, st);
    if (e != hipSuccess) return e;
    uint32_t* pv = alt ? S.val2 : S.val;
    if (W == 2) {
        uint32_t* other = alt ? S.val : S.val2;
        uint64_t* k2 = alt ? S.key : S.key2;
        uint64_t* k3 = alt ? S.key2 : S.key;
        (void)k3;
        hipLaunchKernelGGL(k_gather_word, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, W, 1, pv, n, k2);
        int alt2 = 0;
        // second pass: sort by the high word, carrying the permutation (stable)
        e = launch_radix_sort_pairs(k2, pv, alt ? S.key2 : S.key, other, n, n_bits - 64, S.hist, S.hist_off, S.scan,
                                    &alt2, st);
        if (e != hipSuccess) return e;
        pv = alt2 ? other : pv;
    }
    hipLaunchKernelGGL(k_gather_keys, dim3(blocks_for(n)), dim3(kBlock), 0, st, keys, W, pv, n, sorted, perm);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device workspace of eloc_local_energy_noalloc: amplitudes, partial
// row sums and reduction scratch of the forward pass, for callers that cannot
// allocate device memory.  Every GPU the library runs on holds its own copy
// of this array (kNoAllocBytes) until the process ends.  Host code never uses
// the array's name as an address: its device address is taken once per
// device with hipGetSymbolAddress and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_ws_mu;
void* g_ws_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_workspace(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    if (!g_ws_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ws_ptr[device] = ptr;
    }
    *out = g_ws_ptr[device];
    return hipSuccess;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace eloc
