// Device-side helpers shared by the pair kernels: bit counting, the sample
// signature prefilter, MatrixElement over a term run, and the two
// accumulators (FP64, compensated FP32).
#pragma once

#include "internal.h"
#include "trie.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

constexpr uint64_t kEven = 0x5555555555555555ull;
constexpr uint64_t kOdd = 0xAAAAAAAAAAAAAAAAull;

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }

// Lane of the thread in its wave, and a wave-scope barrier: LDS written by a
// lane is visible to the other lanes of its wave afterwards (the wave runs
// in lockstep; this orders the memory operations around it).  Used where a
// workgroup holds several independent waves.
__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & 63u); }
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact prefilter of LoopOverTerms: a candidate x' can be in U only if its
// (popcount on even qubits, popcount on odd qubits) occurs in U.
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
//   SIAM J. Sci. Comput. 26(6), 2005 (Sum2 / Dot2): the running sum s and the
//   running sum c of all rounding errors are kept apart; the value is s + c.
// The library is compiled without floating-point contraction so that every
// product below is rounded exactly where it is written.
// ---------------------------------------------------------------------------
struct F2 {
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

__device__ __forceinline__ void acc_add(F2& acc, F2 v) { acc_add(acc, v.s, v.c); }

// (x.s + x.c)(y.s + y.c) as hi + lo; hi * lo exact in the leading product.
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

__device__ __forceinline__ void acc_plus(AccD& a, const AccD& b) {
    a.re += b.re;
    a.im += b.im;
}
__device__ __forceinline__ void acc_plus(AccF& a, const AccF& b) {
    acc_add(a.re, b.re);
    acc_add(a.im, b.im);
}

__device__ __forceinline__ AccD masked(const AccD& v, bool on) {
    AccD t;
    t.re = on ? v.re : 0.0;
    t.im = on ? v.im : 0.0;
    return t;
}
__device__ __forceinline__ AccF masked(const AccF& v, bool on) {
    AccF t;
    t.re.s = on ? v.re.s : 0.f;
    t.re.c = on ? v.re.c : 0.f;
    t.im.s = on ? v.im.s : 0.f;
    t.im.c = on ? v.im.c : 0.f;
    return t;
}

// acc += H * v (complex).
__device__ __forceinline__ void mac(AccD& acc, double hr, double hi, double2 v) {
    acc.re = fma(hr, v.x, fma(-hi, v.y, acc.re));
    acc.im = fma(hr, v.y, fma(hi, v.x, acc.im));
}

// The imaginary part of H is exactly zero for a group without odd-|Y| terms
// (every term of a real Hamiltonian); its two products would add exact
// zeros, so they are skipped.
__device__ __forceinline__ void mac(AccF& acc, F2 hr, F2 hi, float4 v) {
    const F2 vr{v.x, v.y}, vi{v.z, v.w};
    float p, q;
    df_mul(hr, vr, p, q);
    acc_add(acc.re, p, q);
    df_mul(hr, vi, p, q);
    acc_add(acc.im, p, q);
    if (hi.s != 0.f || hi.c != 0.f) {
        df_mul(hi, vi, p, q);
        acc_add(acc.re, -p, -q);
        df_mul(hi, vr, p, q);
        acc_add(acc.im, p, q);
    }
}

// ---------------------------------------------------------------------------
// MatrixElement (supplementary algorithm, Eq. pauli_melem) over one group's
// run: real part from [b, m), imaginary part from [m, e); each term adds
// h' (-1)^|ket & YZ|.  Terms are visited with stride `step` from offset
// `off` (step 1: one lane evaluates the whole run; step 64: the wave splits
// it).  NW: keys of at most 32 qubits (the parity needs the low word only).
// ---------------------------------------------------------------------------
template <int W, bool NW>
__device__ __forceinline__ int ket_parity(const uint64_t* yz, const uint64_t* ket) {
    if constexpr (NW) {
        return __popc(static_cast<uint32_t>(ket[0]) & static_cast<uint32_t>(yz[0])) & 1;
    } else {
        int pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) pc += popc64(ket[w] & yz[w]);
        return pc & 1;
    }
}

template <int W, bool NW = false>
__device__ __forceinline__ double term_f64(const TermRec<W>& tr, const uint64_t* ket) {
    return ket_parity<W, NW>(tr.yz, ket) ? -tr.h : tr.h;
}

// One lane's sum over terms [b, e) in order, reading four records per
// round so that their loads overlap; records past e are clamped reads whose
// value is replaced by an exact zero (the sum does not change).
template <int W, bool NW>
__device__ __forceinline__ double run_sum(const TermRec<W>* __restrict__ terms, int b, int e, const uint64_t* ket) {
    double h = 0.0;
    for (int t = b; t < e; t += 4) {
        TermRec<W> tr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) tr[u] = terms[min(t + u, e - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double v = term_f64<W, NW>(tr[u], ket);
            h += (t + u < e) ? v : 0.0;
        }
    }
    return h;
}

template <int W, bool NW = false>
__device__ __forceinline__ void melem(const TermRec<W>* __restrict__ terms, int b, int m, int e, int off, int step,
                                      const uint64_t* ket, double& hr, double& hi) {
    if (step == 1 && off == 0) {
        hr = run_sum<W, NW>(terms, b, m, ket);
        hi = run_sum<W, NW>(terms, m, e, ket);
        return;
    }
    hr = 0.0;
    hi = 0.0;
    for (int t = b + off; t < m; t += step) hr += term_f64<W, NW>(terms[t], ket);
    for (int t = m + off; t < e; t += step) hi += term_f64<W, NW>(terms[t], ket);
}

template <int W, bool NW = false>
__device__ __forceinline__ void term_f32(const TermRecF<W>& tr, const uint64_t* ket, float& vh, float& vl) {
    const bool odd = ket_parity<W, NW>(tr.yz, ket);
    vh = odd ? -tr.h_hi : tr.h_hi;
    vl = odd ? -tr.h_lo : tr.h_lo;
}

template <int W, bool NW>
__device__ __forceinline__ F2 run_sum(const TermRecF<W>* __restrict__ terms, int b, int e, const uint64_t* ket) {
    F2 h{0.f, 0.f};
    for (int t = b; t < e; t += 4) {
        TermRecF<W> tr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) tr[u] = terms[min(t + u, e - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float vh, vl;
            term_f32<W, NW>(tr[u], ket, vh, vl);
            const bool in = t + u < e;
            acc_add(h, in ? vh : 0.f, in ? vl : 0.f);
        }
    }
    return h;
}

template <int W, bool NW = false>
__device__ __forceinline__ void melem(const TermRecF<W>* __restrict__ terms, int b, int m, int e, int off, int step,
                                      const uint64_t* ket, F2& hr, F2& hi) {
    if (step == 1 && off == 0) {
        hr = run_sum<W, NW>(terms, b, m, ket);
        hi = run_sum<W, NW>(terms, m, e, ket);
        return;
    }
    hr = F2{0.f, 0.f};
    hi = F2{0.f, 0.f};
    float vh, vl;
    for (int t = b + off; t < m; t += step) {
        term_f32<W, NW>(terms[t], ket, vh, vl);
        acc_add(hr, vh, vl);
    }
    for (int t = m + off; t < e; t += step) {
        term_f32<W, NW>(terms[t], ket, vh, vl);
        acc_add(hi, vh, vl);
    }
}

// Precision traits: accumulator, term record and gathered vector types.
template <int PREC>
struct Prec;

template <>
struct Prec<0> {
    using Acc = AccD;
    template <int W>
    using Term = TermRec<W>;
    using Vec = double2;
    using H = double;
    static __device__ __forceinline__ void zero(H& h) { h = 0.0; }
    static __device__ __forceinline__ void madd(Acc& a, H hr, H hi, Vec v) { mac(a, hr, hi, v); }
};

template <>
struct Prec<1> {
    using Acc = AccF;
    template <int W>
    using Term = TermRecF<W>;
    using Vec = float4;
    using H = F2;
    static __device__ __forceinline__ void zero(H& h) { h = F2{0.f, 0.f}; }
    static __device__ __forceinline__ void madd(Acc& a, H hr, H hi, Vec v) { mac(a, hr, hi, v); }
};

// ---------------------------------------------------------------------------
// Fixed-order cross-lane reduction (butterfly over the 64 lanes): every lane
// ends with the same total, independent of scheduling.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shfl_xor_d(double v, int m) {
    const int2 p = *reinterpret_cast<int2*>(&v);
    int2 q;
    q.x = __shfl_xor(p.x, m, 64);
    q.y = __shfl_xor(p.y, m, 64);
    return *reinterpret_cast<double*>(&q);
}

// Value of lane k's v in this lane (k per lane).
template <class T>
__device__ __forceinline__ T lane_shfl(const T& v, int k) {
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    constexpr int n = sizeof(T) / 4;
    int w[n];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < n; ++i) w[i] = __shfl(w[i], k, 64);
    T o;
    __builtin_memcpy(&o, w, sizeof(T));
    return o;
}

// First strided term of a run [b, e) for this lane (b + lane, stride S), or
// an exact zero past the run; the read is clamped into the run.
template <int W, bool NW, int S = 64>
__device__ __forceinline__ double strided_first(const TermRec<W>* __restrict__ terms, int b, int e, int lane,
                                                const uint64_t* ket) {
    const int t = b + lane;
    const TermRec<W> tr = terms[min(t, max(e - 1, b))];
    return t < e ? term_f64<W, NW>(tr, ket) : 0.0;
}
template <int W, bool NW, int S = 64>
__device__ __forceinline__ F2 strided_first(const TermRecF<W>* __restrict__ terms, int b, int e, int lane,
                                            const uint64_t* ket) {
    const int t = b + lane;
    const TermRecF<W> tr = terms[min(t, max(e - 1, b))];
    float vh, vl;
    term_f32<W, NW>(tr, ket, vh, vl);
    return t < e ? F2{vh, vl} : F2{0.f, 0.f};
}
// The rest of the strided sum (runs longer than the stride).
template <int W, bool NW, int S = 64>
__device__ __forceinline__ void strided_rest(const TermRec<W>* __restrict__ terms, int b, int e, int lane,
                                             const uint64_t* ket, double& h) {
    for (int t = b + lane + S; t < e; t += S) h += term_f64<W, NW>(terms[t], ket);
}
template <int W, bool NW, int S = 64>
__device__ __forceinline__ void strided_rest(const TermRecF<W>* __restrict__ terms, int b, int e, int lane,
                                             const uint64_t* ket, F2& h) {
    float vh, vl;
    for (int t = b + lane + S; t < e; t += S) {
        term_f32<W, NW>(terms[t], ket, vh, vl);
        acc_add(h, vh, vl);
    }
}

__device__ __forceinline__ void wave_sum(AccD& a) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        a.re += shfl_xor_d(a.re, m);
        a.im += shfl_xor_d(a.im, m);
    }
}

__device__ __forceinline__ void wave_sum(AccF& a) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        AccF o;
        o.re.s = __shfl_xor(a.re.s, m, 64);
        o.re.c = __shfl_xor(a.re.c, m, 64);
        o.im.s = __shfl_xor(a.im.s, m, 64);
        o.im.c = __shfl_xor(a.im.c, m, 64);
        // add in a lane-independent order so both partners get the same bits
        const bool low = (lane_id() & m) == 0;
        AccF first = low ? a : o;
        const AccF second = low ? o : a;
        acc_plus(first, second);
        a = first;
    }
}

// A complex double as FP32 hi + lo pairs (re_hi, re_lo, im_hi, im_lo).
__device__ __forceinline__ float4 split_c(double re, double im) {
    const float rh = static_cast<float>(re);
    const float ih = static_cast<float>(im);
    return make_float4(rh, static_cast<float>(re - static_cast<double>(rh)), ih,
                       static_cast<float>(im - static_cast<double>(ih)));
}

// Block-wide sums of K doubles over NT threads (fixed tree, deterministic);
// every thread ends with the totals.
template <int K, int NT>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*lds)[NT]) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) {
#pragma unroll
            for (int k = 0; k < K; ++k) lds[k][threadIdx.x] += lds[k][threadIdx.x + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = lds[k][0];
    __syncthreads();
}

__device__ __forceinline__ void store_acc(void* partial, int64_t idx, const AccD& a) {
    static_cast<double2*>(partial)[idx] = make_double2(a.re, a.im);
}
__device__ __forceinline__ void store_acc(void* partial, int64_t idx, const AccF& a) {
    static_cast<float4*>(partial)[idx] = make_float4(a.re.s, a.re.c, a.im.s, a.im.c);
}

}  // namespace eloc
