// Autoregressive sampling without replacement (Methods, "Autoregressive
// sampling without replacement", Algorithm ARGumbelTopK) over an ansatz of
// per-qudit perceptrons (Methods, "Ansatz architecture", "Grouping qubits
// into qudits", "Global activation", "Local pruning strategy").
//
// One level per qudit k (D_k qubits, O_k = 2^D_k outcomes), for the B kept
// prefixes:
//   k_ar_level   a workgroup takes 64 prefixes; four waves evaluate the
//                qudit's perceptron for them with FP64 MFMA (16 x 16 tiles,
//                v_mfma_f64_16x16x4f64): the prefix bits as +-1 inputs (0
//                past the prefix) times W1, tanh; times W2 plus the first
//                layer's output, tanh; times W3 -> the O_k outputs z, kept in
//                LDS.  Then one wave per prefix, one lane per outcome: the
//                mean shift of z, the mask of outcomes that cannot reach the
//                electron targets, the normalised log p(c | prefix), l + log p,
//                its Gumbel perturbation, the siblings' maximum Z and the
//                conditioned value Ltil; a sort key (descending Ltil, masked
//                outcomes last) and the candidate index b O_k + c.
//   select       the first min(K, allowed) candidates in (key, index) order:
//                for large levels, two 12-bit digit histograms of the keys
//                (k_sel_hist, k_sel_pick) find the 24-bit key prefix that
//                holds the K-th candidate, the candidates at or below it are
//                compacted in index order (k_sel_flags, scan, k_sel_scatter)
//                and only those are sorted; small levels sort all candidates.
//                The sort is a stable radix sort on 64 bits, so equal values
//                keep the (prefix, outcome) order either way.
//   k_ar_gather  the first min(K, allowed) candidates become the next level's
//                prefixes (key with the outcome's bits set, l, Ltil).
#include "device.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kArH = 64;        // hidden width
constexpr int kArRows = 64;     // prefixes per workgroup
constexpr int kArMaxOut = 64;   // outcomes per qudit (D <= 6)

struct ArLevel {
    int N, W, D, Dk, O, level, q0;
    int n_up, n_down;           // electron targets (-1: no mask)
    int rest_up, rest_down;     // spin-up / spin-down qubits after this qudit
    uint64_t seed;
    const double* W1;           // [H][N] of this qudit
    const double* b1;           // [H]
    const double* W2;           // [H][H]
    const double* b2;
    const double* W3;           // [2^D][H] (first O rows used)
    const double* b3;
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Standard Gumbel variable of the node (level, prefix, outcome): the
// SplitMix64 output function chained over (seed, level, prefix words,
// outcome), u from the top 53 bits, G = -log(-log u).
__device__ __forceinline__ double gumbel(uint64_t seed, int level, const uint64_t* prefix, int W, int outcome) {
    uint64_t h = mix64(seed + 0x9E3779B97F4A7C15ull * static_cast<uint64_t>(level + 1));
    for (int w = 0; w < W; ++w) h = mix64(h ^ prefix[w]);
    h = mix64(h ^ static_cast<uint64_t>(outcome));
    const double u = (static_cast<double>(h >> 11) + 0.5) * 0x1.0p-53;
    return -log(-log(u));
}

__device__ __forceinline__ double wave_max(double v) {
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, shfl_xor_d(v, m));
    return v;
}
__device__ __forceinline__ double wave_add(double v) {
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
    return v;
}

// log(1 - exp(a)) for a < 0
__device__ __forceinline__ double log1mexp(double a) {
    return a > -0.69314718055994531 ? log(-expm1(a)) : log1p(-exp(a));
}

__device__ __forceinline__ int key_bit(const uint64_t* k, int q) { return static_cast<int>((k[q >> 6] >> (q & 63)) & 1ull); }

// acc[t] (the 16 x 16 output tile of columns 16 t ..) = A[rows][0..kend) *
// B[cols][0..kend)^T for t < nt, A from a callback (row, k) read once per
// k step for all tiles, B row-major [out][in] with row pitch ldb (global or
// LDS).  Lane l feeds A[l % 16][k + l / 16] and B[k + l / 16][l % 16];
// register c of lane l holds D[4 c + l / 16][l % 16] (measured layout of
// v_mfma_f64_16x16x4f64 on gfx950).
template <int NT, class AF>
__device__ __forceinline__ void tiles_mma(d4 (&acc)[NT], AF a_of, const double* __restrict__ Bw, int ldb, int ncols,
                                          int kend, int nt, int lane) {
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < kend; k += 4) {
        const int kk = k + (lane >> 4);
        const bool kin = kk < kend;
        const double a = kin ? a_of(lane & 15, kk) : 0.0;
        double b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int col = 16 * t + (lane & 15);
            b[t] = (t < nt && kin && col < ncols) ? Bw[col * ldb + kk] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (t < nt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[t], acc[t], 0, 0, 0);
    }
}

__global__ __launch_bounds__(256) void k_ar_level(ArLevel A, int64_t B, const uint64_t* __restrict__ keys,
                                                  const double* __restrict__ lin, const double* __restrict__ Tin,
                                                  double* __restrict__ cand_l, double* __restrict__ cand_T,
                                                  uint64_t* __restrict__ cand_key, uint32_t* __restrict__ cand_idx,
                                                  unsigned long long* __restrict__ n_allowed) {
    __shared__ uint64_t kbuf[kArRows * kMaxWords];
    __shared__ double h[kArRows][kArH + 1];   // h1, then h2, then z (per wave's own rows)
    __shared__ double wb[kArMaxOut][kArH + 1];   // W2, then W3 ([out][in], padded rows)
    const int wave = static_cast<int>(threadIdx.x) / 64;
    const int lane = lane_id();
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kArRows;
    for (int e = threadIdx.x; e < kArRows * A.W; e += 256) {
        const int64_t b = min(b0 + e / A.W, B - 1);
        kbuf[e] = keys[b * A.W + e % A.W];
    }
    __syncthreads();
    const int r0 = 16 * wave;   // this wave's row tile
    // layer 1: inputs +-1 for the prefix qubits (q < q0), 0 after
    {
        auto a_of = [&](int r, int q) -> double {
            return key_bit(kbuf + (r0 + r) * A.W, q) ? 1.0 : -1.0;
        };
        d4 acc[kArH / 16];
        tiles_mma(acc, a_of, A.W1, A.N, kArH, A.q0, kArH / 16, lane);
#pragma unroll
        for (int t = 0; t < kArH / 16; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int row = r0 + 4 * c + (lane >> 4), col = 16 * t + (lane & 15);
                h[row][col] = tanh(acc[t][c] + A.b1[col]);
            }
    }
    for (int e = threadIdx.x; e < kArH * kArH; e += 256) wb[e / kArH][e % kArH] = A.W2[e];
    __syncthreads();
    // layer 2 with the residual of layer 1
    {
        auto a_of = [&](int r, int k) -> double { return h[r0 + r][k]; };
        d4 acc[kArH / 16];
        tiles_mma(acc, a_of, &wb[0][0], kArH + 1, kArH, kArH, kArH / 16, lane);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kArH / 16; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int row = r0 + 4 * c + (lane >> 4), col = 16 * t + (lane & 15);
                h[row][col] = tanh(acc[t][c] + A.b2[col] + h[row][col]);
            }
    }
    for (int e = threadIdx.x; e < A.O * kArH; e += 256) wb[e / kArH][e % kArH] = A.W3[e];
    __syncthreads();
    // output layer: z for the O outcomes
    {
        auto a_of = [&](int r, int k) -> double { return h[r0 + r][k]; };
        d4 acc[kArMaxOut / 16];
        const int nt = (A.O + 15) / 16;
        tiles_mma(acc, a_of, &wb[0][0], kArH + 1, A.O, kArH, nt, lane);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kArMaxOut / 16; ++t) {
            if (t >= nt) continue;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int row = r0 + 4 * c + (lane >> 4), col = 16 * t + (lane & 15);
                if (col < A.O) h[row][col] = acc[t][c] + A.b3[col];
            }
        }
    }
    __syncthreads();
    // per prefix: one wave, one lane per outcome
    unsigned long long allowed_total = 0;
    for (int r = wave; r < kArRows; r += 4) {
        const int64_t b = b0 + r;
        if (b >= B) break;   // wave-uniform
        const uint64_t* key = kbuf + r * A.W;
        const bool live = lane < A.O;
        const double z = live ? h[r][lane] : 0.0;
        const double mean = wave_add(z) / A.O;
        const double a = 2.0 * (z - mean);
        bool ok = live;
        if (A.n_up >= 0 && live) {
            // electrons of the prefix: even qubits spin up, odd spin down
            // (word boundaries are even, so a bit's parity is its qubit's)
            int up = 0, dn = 0;
            for (int w = 0; w < A.W && 64 * w < A.q0; ++w) {
                const int nb = A.q0 - 64 * w;
                const uint64_t v = key[w] & (nb >= 64 ? ~0ull : ((1ull << nb) - 1ull));
                up += __popcll(v & kEven);
                dn += __popcll(v & kOdd);
            }
            for (int t = 0; t < A.Dk; ++t)
                if ((lane >> t) & 1) {
                    if ((A.q0 + t) & 1)
                        ++dn;
                    else
                        ++up;
                }
            ok = up <= A.n_up && A.n_up <= up + A.rest_up && dn <= A.n_down && A.n_down <= dn + A.rest_down;
        }
        const double m = wave_max(ok ? a : -INFINITY);
        const double s = wave_add(ok ? exp(a - m) : 0.0);
        const double lc = lin[b] + (a - (m + log(s)));
        const double Lp = lc + gumbel(A.seed, A.level, key, A.W, lane);
        const double Z = wave_max(ok ? Lp : -INFINITY);
        const double T = Tin[b];
        double Lt = T;
        if (ok && Lp < Z) {
            const double v = T - Lp + log1mexp(Lp - Z);
            Lt = T - (fmax(v, 0.0) + log1p(exp(-fabs(v))));
        }
        const int64_t i = b * A.O + lane;
        if (live) {
            uint64_t bits = static_cast<uint64_t>(__double_as_longlong(Lt));
            bits = (bits >> 63) ? ~bits : (bits | (1ull << 63));
            cand_key[i] = ok ? ~bits : ~0ull;
            cand_idx[i] = static_cast<uint32_t>(i);
            cand_l[i] = lc;
            cand_T[i] = Lt;
        }
        allowed_total += static_cast<unsigned long long>(__popcll(__ballot(ok)));
    }
    if (lane == 0 && allowed_total) atomicAdd(n_allowed, allowed_total);
}

__global__ void k_ar_gather(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ sorted_idx, int64_t n,
                            int O, int W, int q0, const double* __restrict__ cand_l, const double* __restrict__ cand_T,
                            uint64_t* __restrict__ out_keys, double* __restrict__ out_l, double* __restrict__ out_T) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t idx = sorted_idx[i];
    const int64_t b = idx / O;
    const uint64_t c = idx % O;
    for (int w = 0; w < W; ++w) {
        uint64_t v = keys[b * W + w];
        const int lo = q0 - 64 * w;
        if (lo >= 0 && lo < 64) v |= c << lo;
        if (lo < 0 && lo > -64) v |= c >> (-lo);
        out_keys[i * W + w] = v;
    }
    out_l[i] = cand_l[idx];
    out_T[i] = cand_T[idx];
}

__global__ void k_ar_root(uint64_t* keys, int W, double* l, double* T) {
    if (threadIdx.x < W) keys[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        l[0] = 0.0;
        T[0] = 0.0;
    }
}

// Top-K selection.  Histogram of the 12-bit digit (key >> shift) & 4095
// over the candidates whose key agrees above the digit with the digit chosen
// by the previous pass (prev[0]; all candidates for the top digit, shift
// 52): per block in LDS, then its non-zero counts added to total[4096]
// (integer counts: the order of the additions does not matter).
constexpr int kSelBuckets = 4096;
constexpr int kSelPerBlock = 16384;

__global__ __launch_bounds__(256) void k_sel_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                  const int64_t* __restrict__ prev, uint32_t* __restrict__ total) {
    __shared__ uint32_t h[kSelBuckets];
    for (int t = threadIdx.x; t < kSelBuckets; t += 256) h[t] = 0u;
    __syncthreads();
    const bool filt = shift + 12 < 64;
    const uint64_t prefix = filt ? static_cast<uint64_t>(prev[0]) : 0ull;
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kSelPerBlock;
    const int64_t i1 = min(n, i0 + kSelPerBlock);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const uint64_t k = key[i];
        if (!filt || (k >> (shift + 12)) == prefix) atomicAdd(&h[(k >> shift) & (kSelBuckets - 1)], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSelBuckets; t += 256)
        if (h[t]) atomicAdd(total + t, h[t]);
}

__global__ void k_sel_clear(uint32_t* __restrict__ total) {
    for (int t = threadIdx.x; t < kSelBuckets; t += blockDim.x) total[t] = 0u;
}

// The digit in which the running count over ascending digits reaches `need`
// = need_total - prev[1] (the candidates before the previous pass's digit):
// sel[0] = the digit, sel[1] = the candidates before it over both passes.
// One workgroup, four digits per thread; need >= 1 and at most the total.
// The totals are cleared for the next pass as they are read.
__global__ __launch_bounds__(1024) void k_sel_pick(uint32_t* __restrict__ total, int64_t need_total,
                                                   const int64_t* __restrict__ prev, int64_t* __restrict__ sel) {
    __shared__ int64_t part[1024];
    const int t = static_cast<int>(threadIdx.x);
    int64_t c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c[q] = total[4 * t + q];
        total[4 * t + q] = 0u;
    }
    part[t] = c[0] + c[1] + c[2] + c[3];
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int64_t base = prev ? prev[1] : 0;
    const int64_t need = need_total - base;
    const int64_t before = t ? part[t - 1] : 0;
    if (before < need && need <= part[t]) {
        int64_t run = before;
        int q = 0;
        for (; q < 3; ++q) {
            if (run + c[q] >= need) break;
            run += c[q];
        }
        sel[0] = 4 * t + q;
        sel[1] = base + run;
    }
}

// keep[i] = 1 for the candidates whose 24-bit key prefix is at most the
// selected one (sel1: top digit, sel2: next digit).
__global__ void k_sel_flags(const uint64_t* __restrict__ key, int64_t n, const int64_t* __restrict__ sel1,
                            const int64_t* __restrict__ sel2, int32_t* __restrict__ keep) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const uint64_t thr = (static_cast<uint64_t>(sel1[0]) << 12) | static_cast<uint64_t>(sel2[0]);
    keep[i] = (key[i] >> 40) <= thr ? 1 : 0;
}

// The kept candidates, in index order, with their candidate index.
__global__ void k_sel_scatter(const uint64_t* __restrict__ key, int64_t n, const int32_t* __restrict__ keep,
                              const int64_t* __restrict__ off, uint64_t* __restrict__ okey,
                              uint32_t* __restrict__ oidx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n || !keep[i]) return;
    okey[off[i]] = key[i];
    oidx[off[i]] = static_cast<uint32_t>(i);
}

inline unsigned blocks256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

int64_t ar_select_blocks(int64_t n) { return (n + kSelPerBlock - 1) / kSelPerBlock; }

hipError_t launch_ar_select(const uint64_t* key, int64_t n, int64_t need, uint32_t* hist, int64_t* sel,
                            int32_t* keep, int64_t* off, int64_t* scan, uint64_t* okey, uint32_t* oidx,
                            hipStream_t st) {
    const int nb = static_cast<int>(ar_select_blocks(n));
    uint32_t* total = hist;
    hipLaunchKernelGGL(k_sel_clear, dim3(1), dim3(1024), 0, st, total);
    hipLaunchKernelGGL(k_sel_hist, dim3(nb), dim3(256), 0, st, key, n, 52, static_cast<const int64_t*>(nullptr), total);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, st, total, need, static_cast<const int64_t*>(nullptr), sel);
    hipLaunchKernelGGL(k_sel_hist, dim3(nb), dim3(256), 0, st, key, n, 40, sel, total);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, st, total, need, sel, sel + 2);
    hipLaunchKernelGGL(k_sel_flags, dim3(blocks256(n)), dim3(256), 0, st, key, n, sel, sel + 2, keep);
    const hipError_t e = launch_scan_i32(keep, n, off, scan, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_scatter, dim3(blocks256(n)), dim3(256), 0, st, key, n, keep, off, okey, oidx);
    return hipGetLastError();
}

hipError_t launch_ar_root(uint64_t* keys, int W, double* l, double* T, hipStream_t st) {
    hipLaunchKernelGGL(k_ar_root, dim3(1), dim3(64), 0, st, keys, W, l, T);
    return hipGetLastError();
}

hipError_t launch_ar_level(const ArModelDev& M, int level, int64_t B, uint64_t seed, const uint64_t* keys,
                           const double* l, const double* T, double* cand_l, double* cand_T, uint64_t* cand_key,
                           uint32_t* cand_idx, unsigned long long* n_allowed, hipStream_t st) {
    ArLevel A;
    A.N = M.n_qubits;
    A.W = (M.n_qubits + 63) / 64;
    A.D = M.qudit;
    A.q0 = level * M.qudit;
    A.Dk = min(M.qudit, M.n_qubits - A.q0);
    A.O = 1 << A.Dk;
    A.level = level;
    A.n_up = M.n_up;
    A.n_down = M.n_down;
    A.rest_up = 0;
    A.rest_down = 0;
    for (int q = A.q0 + A.Dk; q < A.N; ++q) {
        if (q & 1)
            ++A.rest_down;
        else
            ++A.rest_up;
    }
    A.seed = seed;
    const int O_full = 1 << M.qudit;
    A.W1 = M.W1 + static_cast<int64_t>(level) * kArH * A.N;
    A.b1 = M.b1 + static_cast<int64_t>(level) * kArH;
    A.W2 = M.W2 + static_cast<int64_t>(level) * kArH * kArH;
    A.b2 = M.b2 + static_cast<int64_t>(level) * kArH;
    A.W3 = M.W3 + static_cast<int64_t>(level) * O_full * kArH;
    A.b3 = M.b3 + static_cast<int64_t>(level) * O_full;
    const unsigned grid = static_cast<unsigned>((B + kArRows - 1) / kArRows);
    hipLaunchKernelGGL(k_ar_level, dim3(grid), dim3(256), 0, st, A, B, keys, l, T, cand_l, cand_T, cand_key,
                       cand_idx, n_allowed);
    return hipGetLastError();
}

hipError_t launch_ar_gather(const uint64_t* keys, const uint32_t* sorted_idx, int64_t n, int O, int W, int q0,
                            const double* cand_l, const double* cand_T, uint64_t* out_keys, double* out_l, double* out_T,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_ar_gather, dim3(blocks256(n)), dim3(256), 0, st, keys, sorted_idx, n, O, W, q0, cand_l,
                       cand_T, out_keys, out_l, out_T);
    return hipGetLastError();
}

}  // namespace eloc
