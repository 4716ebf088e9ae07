// Kernels of the batched pipeline around the batched pair kernel: one
// launch of each covers every problem of the batch.  Per-sample kernels run
// over the global sample index and find their problem through the pid map;
// reductions run over tiles that never straddle two problems and are then
// summed per problem in tile order, so results are deterministic.
//
//   prepare: clear -> copy + hash + bit check + signature range -> table
//            insert -> duplicate check -> Re L max / min -> per-problem
//            shift -> amplitudes
//   finish:  chunk partials -> E_loc -> weighted energy -> variance
#include "device.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_bt_clear(BatchDev B) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    for (int64_t i = t0; i < B.n_slot_words; i += stride) B.slots[i] = 0u;
    for (int64_t i = t0; i < static_cast<int64_t>(B.n) * 128; i += stride) B.bitcounts[i] = 0u;
    for (int64_t i = t0; i < static_cast<int64_t>(B.n) * 3; i += stride) B.rad[i] = 0ull;
    if (t0 < B.n) {
        B.stash[t0].count = 0u;
        B.err[t0] = 0u;
        B.sigmin[t0] = 0xFFFFFFFFu;
        B.sigmax[t0] = 0u;
        B.pairs[t0] = 0ull;
    }
}

// Copy of the caller keys (words beyond the problem's own are zero), linear
// hash, bits >= n_qubits, and the range of the (even popcount, popcount)
// signature over U_k.
template <int W>
__global__ __launch_bounds__(kBlock) void k_bt_hash(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool valid = i < B.S;
    const int k = valid ? B.pid[i] : 0;
    uint32_t code = 0u;
    if (valid) {
        const BatchProb& P = B.probs[k];
        const int64_t li = i - P.s0;
        uint64_t h = 0;
        bool bad = false;
        int pa = 0, n = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint64_t v = w < P.w_in ? P.keys_in[li * P.w_in + w] : 0ull;
            const int nv = P.n_qubits - 64 * w;
            if (nv < 64) {
                const uint64_t allowed = nv <= 0 ? 0ull : ((1ull << nv) - 1ull);
                bad = bad || (v & ~allowed) != 0ull;
                v &= allowed;
            }
            B.keys[i * W + w] = v;
            pa += popc64(v & kEven);
            n += popc64(v);
            while (v) {
                const int q = __ffsll(static_cast<unsigned long long>(v)) - 1;
                h ^= B.R[64 * w + q];
                v &= v - 1ull;
            }
        }
        B.khash[i] = h;
        if (bad) atomicOr(B.err + k, static_cast<uint32_t>(kErrBits));
        code = (static_cast<uint32_t>(pa) << 8) | static_cast<uint32_t>(n);
    }
    // one atomic pair per wave when the wave lies inside one problem
    const int k0 = __builtin_amdgcn_readfirstlane(k);
    const uint64_t all = __ballot(1);
    const bool one = __ballot(valid && k == k0) == all && __ballot(valid) == all;
    // per-qubit counts of set bits: lane q adds the wave's count of qubit q
    const int lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t v = valid ? B.keys[i * W + w] : 0ull;
        if (one) {
            uint32_t mine = 0u;
            for (int q = 0; q < 64; ++q) {
                const uint32_t c = static_cast<uint32_t>(__popcll(__ballot((v >> q) & 1ull)));
                if (lane == q) mine = c;
            }
            if (mine) atomicAdd(B.bitcounts + static_cast<int64_t>(k0) * 128 + 64 * w + lane, mine);
        } else if (valid) {
            for (uint64_t u = v; u; u &= u - 1ull)
                atomicAdd(B.bitcounts + static_cast<int64_t>(k) * 128 + 64 * w + (__ffsll(static_cast<unsigned long long>(u)) - 1), 1u);
        }
    }
    if (one) {
        uint32_t mn = code, mx = code;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            mn = min(mn, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mn), m, 64)));
            mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), m, 64)));
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin(B.sigmin + k0, mn);
            atomicMax(B.sigmax + k0, mx);
        }
    } else if (valid) {
        atomicMin(B.sigmin + k, code);
        atomicMax(B.sigmax + k, code);
    }
}

// one thread per problem: majority key of U_k (radius filter reference)
__global__ __launch_bounds__(kBlock) void k_bt_radius_ref(BatchDev B) {
    const int k = static_cast<int>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= B.n) return;
    const int64_t M = B.probs[k].M;
    for (int w = 0; w < 2; ++w) {
        uint64_t c = 0;
        if (w < B.W)
            for (int q = 0; q < 64; ++q)
                if (2 * static_cast<int64_t>(B.bitcounts[static_cast<int64_t>(k) * 128 + 64 * w + q]) > M) c |= 1ull << q;
        B.rad[3 * k + w] = c;
    }
}

// max distance of U_k's keys from that key
template <int W>
__global__ __launch_bounds__(kBlock) void k_bt_radius_max(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool valid = i < B.S;
    const int k = valid ? B.pid[i] : 0;
    int d = 0;
    if (valid) {
#pragma unroll
        for (int w = 0; w < W; ++w) d += popc64(B.keys[i * W + w] ^ B.rad[3 * k + w]);
    }
    const int k0 = __builtin_amdgcn_readfirstlane(k);
    const uint64_t all = __ballot(1);
    if (__ballot(valid && k == k0) == all && __ballot(valid) == all) {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) d = max(d, __shfl_xor(d, m, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(B.rad + 3 * k0 + 2, static_cast<unsigned long long>(d));
    } else if (valid) {
        atomicMax(B.rad + 3 * k + 2, static_cast<unsigned long long>(d));
    }
}

template <int TK>
__global__ __launch_bounds__(kBlock) void k_bt_insert(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= B.S) return;
    const int k = B.pid[i];
    const BatchProb& P = B.probs[k];
    table_insert_one<TK>(B.khash + P.s0, i - P.s0, P.kslots, P.kstash, P.ktable, B.err + k,
                        static_cast<uint32_t>(kErrTable));
}

// one-word keys: each problem's key table in its own format (narrow or wide)
__global__ __launch_bounds__(kBlock) void k_bt_insert1(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= B.S) return;
    const int k = B.pid[i];
    const BatchProb& P = B.probs[k];
    if (P.narrow)
        table_insert_one<kTabNarrow>(B.khash + P.s0, i - P.s0, P.kslots, P.kstash, P.ktable, B.err + k,
                                     static_cast<uint32_t>(kErrTable));
    else
        table_insert_one<kTabWide>(B.khash + P.s0, i - P.s0, P.kslots, P.kstash, P.ktable, B.err + k,
                                   static_cast<uint32_t>(kErrTable));
}

__global__ __launch_bounds__(kBlock) void k_bt_verify1(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= B.S) return;
    const int k = B.pid[i];
    const BatchProb& P = B.probs[k];
    const uint64_t key[1] = {B.keys[i]};
    const int j = P.narrow ? table_find<kTabNarrow, 1>(P.ktable, B.keys + P.s0, B.khash[i], key)
                           : table_find<kTabWide, 1>(P.ktable, B.keys + P.s0, B.khash[i], key);
    if (j != static_cast<int>(i - P.s0)) atomicOr(B.err + k, static_cast<uint32_t>(kErrDup));
}

// every key must find itself (U unique)
template <int W, int TK>
__global__ __launch_bounds__(kBlock) void k_bt_verify(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= B.S) return;
    const int k = B.pid[i];
    const BatchProb& P = B.probs[k];
    uint64_t key[W];
#pragma unroll
    for (int w = 0; w < W; ++w) key[w] = B.keys[i * W + w];
    const int j = table_find<TK, W>(P.ktable, B.keys + P.s0 * W, B.khash[i], key);
    if (j != static_cast<int>(i - P.s0)) atomicOr(B.err + k, static_cast<uint32_t>(kErrDup));
}

// per tile: max and min of Re L
__global__ __launch_bounds__(kBlock) void k_bt_minmax(BatchDev B) {
    __shared__ double lds[2][kBlock];
    const RTile T = B.tiles[blockIdx.x];
    const BatchProb& P = B.probs[T.prob];
    double mx = -INFINITY, mn = INFINITY;
    for (int64_t i = T.begin + threadIdx.x; i < T.end; i += kBlock) {
        const double r = P.logpsi[i - P.s0].x;
        mx = fmax(mx, r);
        mn = fmin(mn, r);
    }
    lds[0][threadIdx.x] = mx;
    lds[1][threadIdx.x] = mn;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) {
            lds[0][threadIdx.x] = fmax(lds[0][threadIdx.x], lds[0][threadIdx.x + s]);
            lds[1][threadIdx.x] = fmin(lds[1][threadIdx.x], lds[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        B.part[3 * blockIdx.x] = lds[0][0];
        B.part[3 * blockIdx.x + 1] = lds[1][0];
    }
}

// one thread per problem: shift c_k = max Re L, range checks
__global__ __launch_bounds__(kBlock) void k_bt_shift(BatchDev B, int fp32) {
    const int k = static_cast<int>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= B.n) return;
    const BatchProb& P = B.probs[k];
    double mx = -INFINITY, mn = INFINITY;
    for (int t = P.rt0; t < P.rt0 + P.rtn; ++t) {
        mx = fmax(mx, B.part[3 * t]);
        mn = fmin(mn, B.part[3 * t + 1]);
    }
    B.shift[k] = mx;
    // exp(L - c) and exp(c - L) finite and normal: spread <= 60 (FP32 form), 700 (FP64)
    if (!(mx - mn <= (fp32 ? 60.0 : 700.0)) || !isfinite(mx) || !isfinite(mn))
        atomicOr(B.err + k, static_cast<uint32_t>(kErrRange));
}

// a = exp(L - c), b = exp(c - L), FP64 and (fp32) hi/lo pairs
__global__ __launch_bounds__(kBlock) void k_bt_amp(BatchDev B, int fp32) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= B.S) return;
    const int k = B.pid[i];
    const BatchProb& P = B.probs[k];
    const double c = B.shift[k];
    const double2 l = P.logpsi[i - P.s0];
    double s, co;
    sincos(l.y, &s, &co);
    const double ea = exp(l.x - c);
    const double eb = exp(c - l.x);
    B.a[i] = make_double2(ea * co, ea * s);
    B.b[i] = make_double2(eb * co, -eb * s);
    if (fp32) {
        B.af[i] = split_c(ea * co, ea * s);
        B.bf[i] = split_c(eb * co, -eb * s);
    }
}

// E_loc(x) = b_x * (sum of the row's chunk partials in chunk order)
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_bt_finish(BatchDev B) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= B.S) return;
    const BatchProb& P = B.probs[B.pid[i]];
    const int64_t li = i - P.s0;
    if (PREC == 0) {
        const double2* part = static_cast<const double2*>(B.partial) + P.pbase;
        double re = 0.0, im = 0.0;
        for (int c = 0; c < P.chunks; ++c) {
            const double2 p = part[c * P.M + li];
            re += p.x;
            im += p.y;
        }
        const double2 bi = B.b[i];
        P.eloc[li] = make_double2(re * bi.x - im * bi.y, re * bi.y + im * bi.x);
    } else {
        const float4* part = static_cast<const float4*>(B.partial) + P.pbase;
        F2 re{0.f, 0.f}, im{0.f, 0.f};
        for (int c = 0; c < P.chunks; ++c) {
            const float4 p = part[c * P.M + li];
            acc_add(re, p.x, p.y);
            acc_add(im, p.z, p.w);
        }
        AccF r;
        mac(r, re, im, B.bf[i]);
        P.eloc[li] = make_double2(static_cast<double>(r.re.s) + static_cast<double>(r.re.c),
                                  static_cast<double>(r.im.s) + static_cast<double>(r.im.c));
    }
}

__device__ __forceinline__ double bt_weight(const BatchProb& P, int64_t li, double c, bool& bad) {
    if (P.weights) {
        const double w = P.weights[li];
        if (!(w >= 0.0) || !isfinite(w)) bad = true;
        return w;
    }
    return exp(2.0 * (P.logpsi[li].x - c));
}

// per tile: sum w, sum w Re E_loc, sum w Im E_loc
__global__ __launch_bounds__(kBlock) void k_bt_energy1(BatchDev B) {
    __shared__ double lds[3][kBlock];
    const RTile T = B.tiles[blockIdx.x];
    const BatchProb& P = B.probs[T.prob];
    const double c = B.shift[T.prob];
    double v[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    for (int64_t i = T.begin + threadIdx.x; i < T.end; i += kBlock) {
        const int64_t li = i - P.s0;
        const double w = bt_weight(P, li, c, bad);
        const double2 e = P.eloc[li];
        v[0] += w;
        v[1] += w * e.x;
        v[2] += w * e.y;
    }
    if (bad) atomicOr(B.err + T.prob, static_cast<uint32_t>(kErrWeights));
    block_sum<3, kBlock>(v, lds);
    if (threadIdx.x == 0) {
        B.part[3 * blockIdx.x] = v[0];
        B.part[3 * blockIdx.x + 1] = v[1];
        B.part[3 * blockIdx.x + 2] = v[2];
    }
}

// one thread per problem: E = sum w E_loc / sum w
__global__ __launch_bounds__(kBlock) void k_bt_energy2(BatchDev B) {
    const int k = static_cast<int>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= B.n) return;
    const BatchProb& P = B.probs[k];
    double tot = 0.0, sr = 0.0, si = 0.0;
    for (int t = P.rt0; t < P.rt0 + P.rtn; ++t) {
        tot += B.part[3 * t];
        sr += B.part[3 * t + 1];
        si += B.part[3 * t + 2];
    }
    if (!(tot > 0.0) || !isfinite(tot)) atomicOr(B.err + k, static_cast<uint32_t>(kErrWeights));
    const double er = sr / tot, ei = si / tot;
    P.stats[0] = er;
    P.stats[1] = ei;
    P.stats[3] = P.weights ? tot : tot * exp(2.0 * B.shift[k]);
    B.scal[3 * k] = er;
    B.scal[3 * k + 1] = ei;
    B.scal[3 * k + 2] = tot;
}

// per tile: sum w |E_loc - E|^2
__global__ __launch_bounds__(kBlock) void k_bt_energy3(BatchDev B) {
    __shared__ double lds[1][kBlock];
    const RTile T = B.tiles[blockIdx.x];
    const BatchProb& P = B.probs[T.prob];
    const double c = B.shift[T.prob];
    const double er = B.scal[3 * T.prob], ei = B.scal[3 * T.prob + 1];
    double v[1] = {0.0};
    bool bad = false;
    for (int64_t i = T.begin + threadIdx.x; i < T.end; i += kBlock) {
        const int64_t li = i - P.s0;
        const double w = bt_weight(P, li, c, bad);
        const double2 e = P.eloc[li];
        const double dr = e.x - er, di = e.y - ei;
        v[0] += w * (dr * dr + di * di);
    }
    block_sum<1, kBlock>(v, lds);
    if (threadIdx.x == 0) B.part[3 * blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_bt_energy4(BatchDev B) {
    const int k = static_cast<int>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= B.n) return;
    const BatchProb& P = B.probs[k];
    double v = 0.0;
    for (int t = P.rt0; t < P.rt0 + P.rtn; ++t) v += B.part[3 * t];
    P.stats[2] = v / B.scal[3 * k + 2];
}

}  // namespace

hipError_t launch_batch_prepare(const BatchDev& B, bool fp32, hipStream_t st) {
    const int64_t clear_n = B.n_slot_words > B.S ? B.n_slot_words : B.S;
    const unsigned clear_blocks = blocks_for(clear_n) < 4096u ? blocks_for(clear_n) : 4096u;
    hipLaunchKernelGGL(k_bt_clear, dim3(clear_blocks), dim3(kBlock), 0, st, B);
    const dim3 grid(blocks_for(B.S)), block(kBlock);
    if (B.W == 2) {
        hipLaunchKernelGGL(k_bt_hash<2>, grid, block, 0, st, B);
        hipLaunchKernelGGL(k_bt_radius_ref, dim3(blocks_for(B.n)), block, 0, st, B);
        hipLaunchKernelGGL(k_bt_radius_max<2>, grid, block, 0, st, B);
        hipLaunchKernelGGL(k_bt_insert<kTabVerify>, grid, block, 0, st, B);
        hipLaunchKernelGGL((k_bt_verify<2, kTabVerify>), grid, block, 0, st, B);
    } else {
        hipLaunchKernelGGL(k_bt_hash<1>, grid, block, 0, st, B);
        hipLaunchKernelGGL(k_bt_radius_ref, dim3(blocks_for(B.n)), block, 0, st, B);
        hipLaunchKernelGGL(k_bt_radius_max<1>, grid, block, 0, st, B);
        hipLaunchKernelGGL(k_bt_insert1, grid, block, 0, st, B);
        hipLaunchKernelGGL(k_bt_verify1, grid, block, 0, st, B);
    }
    hipLaunchKernelGGL(k_bt_minmax, dim3(static_cast<unsigned>(B.n_tiles)), dim3(kBlock), 0, st, B);
    hipLaunchKernelGGL(k_bt_shift, dim3(blocks_for(B.n)), dim3(kBlock), 0, st, B, fp32 ? 1 : 0);
    hipLaunchKernelGGL(k_bt_amp, dim3(blocks_for(B.S)), dim3(kBlock), 0, st, B, fp32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchDev& B, int precision, hipStream_t st) {
    if (precision == 0)
        hipLaunchKernelGGL(k_bt_finish<0>, dim3(blocks_for(B.S)), dim3(kBlock), 0, st, B);
    else
        hipLaunchKernelGGL(k_bt_finish<1>, dim3(blocks_for(B.S)), dim3(kBlock), 0, st, B);
    hipLaunchKernelGGL(k_bt_energy1, dim3(static_cast<unsigned>(B.n_tiles)), dim3(kBlock), 0, st, B);
    hipLaunchKernelGGL(k_bt_energy2, dim3(blocks_for(B.n)), dim3(kBlock), 0, st, B);
    hipLaunchKernelGGL(k_bt_energy3, dim3(static_cast<unsigned>(B.n_tiles)), dim3(kBlock), 0, st, B);
    hipLaunchKernelGGL(k_bt_energy4, dim3(blocks_for(B.n)), dim3(kBlock), 0, st, B);
    return hipGetLastError();
}

}  // namespace eloc
