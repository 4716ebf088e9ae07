// Stochastic reconfiguration restricted to the highest-probability samples
// (Sec. "ANQS-tailored stochastic reconfiguration"): the SR sample set, and
// the SR-transformed gradient d = (Re S + lambda I)^{-1} F with S the quantum
// geometric tensor of Eq. qgt_definition estimated over that set with
// renormalised probabilities.
//
// With R = 2 N_SR real rows X = [sqrt(w) (O_re - Obar_re); sqrt(w) (O_im -
// Obar_im)] (N_SR x N_p each), Re S = X^T X, and since N_SR << N_p the solve
// goes through the N_SR-sized side (the identity the min-SR recipe rests
// on): (lambda I + X^T X)^{-1} F = (F - X^T (lambda I + X X^T)^{-1} X F) / lambda.
//
//   k_sr_weights  w_x = |psi_x|^2 / sum over the set, and sqrt(w_x)
//   k_sr_mean     Obar_p = sum_x w_x O_xp (real and imaginary parts)
//   k_sr_gram     the Gram matrix of [X; F] (R + 1 rows) over N_p: each
//                 workgroup stages a slab of columns of [X; F] in LDS and its
//                 eight waves accumulate 16 x 16 tiles of the upper triangle
//                 with FP64 MFMA (v_mfma_f64_16x16x4f64); one partial Gram
//                 per workgroup, added in fixed order by k_sr_reduce
//   k_sr_chol_reg Cholesky of X X^T + lambda I and the two triangular solves
//                 for y = (X X^T + lambda I)^{-1} X F: one workgroup whose
//                 threads hold the lower triangle in registers (N_SR <= 127)
//   k_sr_chol     the same from global memory, one wave (larger sets)
//   k_sr_update   d_p = (F_p - sum_r X_rp y_r) / lambda
#include "device.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kSrWaves = 8;            // waves of a Gram workgroup
constexpr int kSrTilesPerWave = 12;    // accumulator tiles a wave holds
constexpr int kSrTilesPerGroup = kSrWaves * kSrTilesPerWave;

struct SrArgs {
    int nsr;              // samples in the set
    int64_t np;           // parameters
    int R;                // rows of [X; F] = 2 nsr + 1
    int R16;              // R rounded up to 16
    int KS;               // columns per LDS slab
    int pitch;            // LDS row pitch in doubles (KS + 1: rows start in different banks)
    const double* ore;    // [nsr][np]
    const double* oim;
    const double* F;      // [np]
    const double* w;      // [nsr] weights, then [nsr] square roots
    const double* mean;   // [2][np]
};

__device__ __forceinline__ double x_elem(const SrArgs& A, int r, int64_t p) {
    if (p >= A.np || r >= A.R) return 0.0;
    if (r < A.nsr) return A.w[A.nsr + r] * (A.ore[static_cast<int64_t>(r) * A.np + p] - A.mean[p]);
    if (r < 2 * A.nsr) {
        const int x = r - A.nsr;
        return A.w[A.nsr + x] * (A.oim[static_cast<int64_t>(x) * A.np + p] - A.mean[A.np + p]);
    }
    return A.F[p];
}

__global__ __launch_bounds__(256) void k_sr_weights(const double2* __restrict__ logpsi, int nsr,
                                                    double* __restrict__ w) {
    __shared__ double red[256];
    double m = -INFINITY;
    for (int x = threadIdx.x; x < nsr; x += 256) m = fmax(m, logpsi[x].x);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    m = red[0];
    __syncthreads();
    double sum = 0.0;
    for (int x = threadIdx.x; x < nsr; x += 256) sum += exp(2.0 * (logpsi[x].x - m));
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    sum = red[0];
    for (int x = threadIdx.x; x < nsr; x += 256) {
        const double v = exp(2.0 * (logpsi[x].x - m)) / sum;
        w[x] = v;
        w[nsr + x] = sqrt(v);
    }
}

__global__ __launch_bounds__(256) void k_sr_mean(SrArgs A, double* __restrict__ mean) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= A.np) return;
    double mr = 0.0, mi = 0.0;
    for (int x = 0; x < A.nsr; ++x) {
        mr += A.w[x] * A.ore[static_cast<int64_t>(x) * A.np + p];
        mi += A.w[x] * A.oim[static_cast<int64_t>(x) * A.np + p];
    }
    mean[p] = mr;
    mean[A.np + p] = mi;
}

// Tile t of the upper triangle (row tile i <= column tile j), row-major over
// i, then j.
__device__ __forceinline__ void tile_ij(int t, int nt, int& i, int& j) {
    i = 0;
    int left = t;
    while (left >= nt - i) {
        left -= nt - i;
        ++i;
    }
    j = i + left;
}

// grid: (column ranges, tile groups); block: kSrWaves waves.  LDS holds one
// slab [R16][KS] of [X; F].
__global__ __launch_bounds__(64 * kSrWaves) void k_sr_gram(SrArgs A, int64_t cols_per_block,
                                                         double* __restrict__ partial) {
    extern __shared__ double slab[];
    const int wave = static_cast<int>(threadIdx.x) / 64;
    const int lane = lane_id();
    const int nt = A.R16 / 16;
    const int ntiles = nt * (nt + 1) / 2;
    const int t0 = static_cast<int>(blockIdx.y) * kSrTilesPerGroup;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * cols_per_block;
    const int64_t c1 = min(A.np, c0 + cols_per_block);
    d4 acc[kSrTilesPerWave];
    int ti[kSrTilesPerWave], tj[kSrTilesPerWave];
#pragma unroll
    for (int k = 0; k < kSrTilesPerWave; ++k) {
        acc[k] = d4{0.0, 0.0, 0.0, 0.0};
        const int t = t0 + wave + kSrWaves * k;
        if (t < ntiles) {
            tile_ij(t, nt, ti[k], tj[k]);
        } else {
            ti[k] = -1;
            tj[k] = -1;
        }
    }
    const int nthreads = 64 * kSrWaves;
    for (int64_t base = c0; base < c1; base += A.KS) {
        __syncthreads();
        // stage [R16][KS]: consecutive threads take consecutive columns
        for (int e = static_cast<int>(threadIdx.x); e < A.R16 * A.KS; e += nthreads) {
            const int r = e / A.KS;
            const int k = e - r * A.KS;
            const int64_t p = base + k;
            slab[r * A.pitch + k] = p < c1 ? x_elem(A, r, p) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSrTilesPerWave; ++k) {
            if (ti[k] < 0) continue;   // wave-uniform
            const double* ra = slab + (16 * ti[k] + (lane & 15)) * A.pitch;
            const double* rb = slab + (16 * tj[k] + (lane & 15)) * A.pitch;
            for (int kk = 0; kk < A.KS; kk += 4) {
                // lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of this
                // 4-column step: both are the slab rows' columns kk + l / 16
                const double a = ra[kk + (lane >> 4)];
                const double b = rb[kk + (lane >> 4)];
                acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
            }
        }
    }
    // register c of lane l holds D[4 c + l / 16][l % 16] of its tile (measured layout of
    // v_mfma_f64_16x16x4f64 on gfx950)
    double* out = partial + static_cast<int64_t>(blockIdx.x) * A.R16 * A.R16;
#pragma unroll
    for (int k = 0; k < kSrTilesPerWave; ++k) {
        if (ti[k] < 0) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int row = 16 * ti[k] + 4 * c + (lane >> 4);
            const int col = 16 * tj[k] + (lane & 15);
            out[static_cast<int64_t>(row) * A.R16 + col] = acc[k][c];
        }
    }
}

// T[r][c] (r <= c by tiles) = sum over blocks of the partials in a fixed
// order, mirrored into the lower triangle: pass 1 (blockIdx.y = g) adds the
// partials of blocks g, g + kSrRed, ... into tmp[g], pass 2 adds tmp[0..kSrRed).
constexpr int kSrRed = 8;

__global__ __launch_bounds__(256) void k_sr_reduce(const double* __restrict__ partial, int nblocks, int R16, int R,
                                                   double* __restrict__ tmp) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t RR = static_cast<int64_t>(R) * R;
    if (e >= RR) return;
    const int r = static_cast<int>(e / R), c = static_cast<int>(e % R);
    // the upper tile holding (min, max) carries both orders inside a
    // diagonal tile; off the diagonal tiles only the tile with row <= column
    int rr = r, cc = c;
    if (r / 16 > c / 16) {
        rr = c;
        cc = r;
    }
    double s = 0.0;
    for (int b = static_cast<int>(blockIdx.y); b < nblocks; b += kSrRed)
        s += partial[static_cast<int64_t>(b) * R16 * R16 + static_cast<int64_t>(rr) * R16 + cc];
    tmp[static_cast<int64_t>(blockIdx.y) * RR + e] = s;
}

__global__ __launch_bounds__(256) void k_sr_reduce2(const double* __restrict__ tmp, int64_t RR, double* __restrict__ T) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= RR) return;
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < kSrRed; ++g) s += tmp[g * RR + e];
    T[e] = s;
}

// Cholesky of A = T[0..n)[0..n) + lambda I (n = 2 nsr) into L (row-major n x n,
// lower triangle), then y = A^{-1} T[0..n)[n]: forward substitution by rows
// (a dot product over the row, reduced across the wave), back substitution by
// columns of L^T (an update with row j of L).  One wave: its steps are
// ordered by workgroup barriers, which cost little for a single wave.
__global__ __launch_bounds__(64) void k_sr_chol(const double* __restrict__ T, int n, int R, double lambda,
                                                double* __restrict__ L, double* __restrict__ y,
                                                uint32_t* __restrict__ err) {
    const int lane = threadIdx.x;
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e % n;
        L[e] = T[r * R + c] + (r == c ? lambda : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double d = L[k * n + k];
        if (lane == 0 && !(d > 0.0)) atomicOr(err, static_cast<uint32_t>(kErrRange));
        const double piv = sqrt(fmax(d, 1e-300));
        __syncthreads();
        if (lane == 0) L[k * n + k] = piv;
        for (int i = k + 1 + lane; i < n; i += 64) L[i * n + k] /= piv;
        __syncthreads();
        // trailing lower triangle: A[i][j] -= L[i][k] L[j][k], k < j <= i; lane
        // takes rows i, each row's columns in order
        for (int i = k + 1 + lane; i < n; i += 64) {
            const double lik = L[i * n + k];
            for (int j = k + 1; j <= i; ++j) L[i * n + j] -= lik * L[j * n + k];
        }
        __syncthreads();
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = lane; j < i; j += 64) s += L[i * n + j] * y[j];
        for (int m = 32; m >= 1; m >>= 1) s += shfl_xor_d(s, m);
        if (lane == 0) y[i] = (T[i * R + n] - s) / L[i * n + i];
        __syncthreads();
    }
    for (int j = n - 1; j >= 0; --j) {
        const double yj = y[j] / L[j * n + j];
        __syncthreads();
        if (lane == 0) y[j] = yj;
        for (int i = lane; i < j; i += 64) y[i] -= L[j * n + i] * yj;
        __syncthreads();
    }
}

// The factorisation of the augmented matrix [[A, b], [b^T, *]] (A = T[0..n)^2
// + lambda I, b = T[n][0..n)): its last row of L is z = L^{-1} b, so the
// forward substitution comes with the factorisation.  The lower triangle
// (rows 0..n) is held in registers, cyclically over a 32 x 32 grid of
// threads: thread (tr, tc) owns the elements (tr + 32 p, tc + 32 q), p >= q.
// Step k publishes column k unnormalised (a_ik, i >= k) in LDS,
// double-buffered so that one barrier per step suffices; then a_ij -= a_ik
// a_jk / a_kk for j > k, and column k becomes L's (a_ik / sqrt(a_kk)).  The
// back substitution L^T y = z runs over the rows j of L from the last: the
// owners of (j, i < j) take L_ji y_j off z_i.
constexpr int kCholThreads = 1024;
constexpr int kCholMaxRows = 256;   // rows of the augmented matrix (n + 1) the register form takes

template <int P>
__global__ __launch_bounds__(kCholThreads) void k_sr_chol_reg(const double* __restrict__ T, int n, int R, double lambda,
                                                             double* __restrict__ y, uint32_t* __restrict__ err) {
    static_assert(32 * P <= kCholMaxRows, "rows of the register grid");
    __shared__ double col[2][kCholMaxRows];
    __shared__ double zbuf[kCholMaxRows];
    // pivot terms of step k: sqrt(a_kk), 1 / a_kk, 1 / sqrt(a_kk), written by
    // the owner of (k, k) as soon as a_kk is final (the step before)
    __shared__ double prm[kCholMaxRows][3];
    const int tid = static_cast<int>(threadIdx.x);
    const int tr = tid >> 5, tc = tid & 31;
    auto pivot = [&](int k, double akk) {
        if (!(akk > 0.0)) atomicOr(err, static_cast<uint32_t>(kErrRange));
        const double dk = fmax(akk, 1e-300);
        const double piv = sqrt(dk);
        prm[k][0] = piv;
        prm[k][1] = 1.0 / dk;
        prm[k][2] = 1.0 / piv;
    };
    double a[P][P];   // [p][q], p >= q used
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q <= p; ++q) {
            const int i = tr + 32 * p, j = tc + 32 * q;
            a[p][q] = (i <= n && j <= i) ? T[static_cast<int64_t>(i) * R + j] + (i == j && i < n ? lambda : 0.0) : 0.0;
        }
    if (tid == 0) pivot(0, a[0][0]);
    for (int k = 0; k < n; ++k) {
        double* c = col[k & 1];
        const int kb = k >> 5;   // row / column blocks below kb hold nothing left to do (uniform)
        if (tc == (k & 31)) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int q = 0; q <= p; ++q) {
                    const int i = tr + 32 * p;
                    if (q == kb && i >= k && i <= n) c[i] = a[p][q];
                }
        }
        __syncthreads();
        const double piv = prm[k][0], inv = prm[k][1], rpiv = prm[k][2];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (p < kb) continue;
            const double cr = c[tr + 32 * p];
#pragma unroll
            for (int q = 0; q <= p; ++q) {
                if (q < kb) continue;
                const int i = tr + 32 * p, j = tc + 32 * q;
                if (i > n || j > i) continue;
                if (j == k)
                    a[p][q] = i == k ? piv : a[p][q] * rpiv;
                else if (j > k)
                    a[p][q] -= cr * c[j] * inv;
            }
        }
        // the next pivot, from its owner's final a_{k+1,k+1}
        const int k1 = k + 1;
        if (k1 < n && tr == (k1 & 31) && tc == (k1 & 31)) {
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (p == (k1 >> 5)) pivot(k1, a[p][p]);
        }
    }
    if (tr == (n & 31)) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int q = 0; q <= p; ++q) {
                const int j = tc + 32 * q;
                if (p == (n >> 5) && j < n) zbuf[j] = a[p][q];
            }
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
        const double yj = zbuf[j] * prm[j][2];
        if (tr == (j & 31)) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int q = 0; q <= p; ++q) {
                    const int i = tc + 32 * q;
                    if (p == (j >> 5) && i < j) zbuf[i] -= a[p][q] * yj;
                }
        }
        __syncthreads();
    }
    for (int j = tid; j < n; j += kCholThreads) y[j] = zbuf[j] * prm[j][2];
}

template <int P>
void launch_chol_reg(const double* T, int n, int R, double lambda, double* y, uint32_t* err, hipStream_t st) {
    hipLaunchKernelGGL((k_sr_chol_reg<P>), dim3(1), dim3(kCholThreads), 0, st, T, n, R, lambda, y, err);
}

__global__ __launch_bounds__(256) void k_sr_update(SrArgs A, const double* __restrict__ y, double lambda,
                                                   double* __restrict__ d) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (p >= A.np) return;
    double s = 0.0;
    for (int r = 0; r < 2 * A.nsr; ++r) s += x_elem(A, r, p) * y[r];
    d[p] = (A.F[p] - s) / lambda;
}

__global__ void k_sr_select_keys(const double2* __restrict__ logpsi, int64_t n, uint64_t* __restrict__ key,
                                 uint32_t* __restrict__ idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    uint64_t b = __double_as_longlong(logpsi[i].x);
    // order-preserving map of doubles to unsigned integers, then reversed so
    // that an ascending sort puts the largest Re log psi first
    b = (b >> 63) ? ~b : (b | (1ull << 63));
    key[i] = ~b;
    idx[i] = static_cast<uint32_t>(i);
}

__global__ void k_sr_take(const uint32_t* __restrict__ idx, int n, int32_t* __restrict__ out) {
    const int i = static_cast<int>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) out[i] = static_cast<int32_t>(idx[i]);
}

inline unsigned blocks256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

int64_t sr_partial_blocks(int64_t np) { return std::max<int64_t>(1, std::min<int64_t>(512, (np + 255) / 256)); }

// Doubles of the Gram scratch: the per-block partials, then kSrRed R^2 of the
// first reduction pass.
int64_t sr_partial_len(int64_t np, int R16, int R) {
    return sr_partial_blocks(np) * R16 * R16 + static_cast<int64_t>(kSrRed) * R * R;
}

// LDS slab of the Gram kernel under 64 KB: R16 rows of KS + 1 doubles
size_t sr_gram_slab_cols(int R16) { return R16 <= 240 ? 32 : (R16 <= 480 ? 16 : 8); }

hipError_t launch_sr_select(const double2* logpsi, int64_t n, int nsr, uint64_t* key, uint32_t* val, uint64_t* key2,
                            uint32_t* val2, uint32_t* hist, int64_t* hist_off, int64_t* scan, int32_t* out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_sr_select_keys, dim3(blocks256(n)), dim3(256), 0, st, logpsi, n, key, val);
    int alt = 0;
    hipError_t e = launch_radix_sort_pairs(key, val, key2, val2, n, 64, hist, hist_off, scan, &alt, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sr_take, dim3(blocks256(nsr)), dim3(256), 0, st, alt ? val2 : val, nsr, out);
    return hipGetLastError();
}

hipError_t launch_sr_solve(int nsr, int64_t np, const double* ore, const double* oim, const double2* logpsi,
                           const double* F, double lambda, double* w, double* mean, double* partial, double* T,
                           double* L, double* y, double* d, uint32_t* err, hipStream_t st) {
    SrArgs A;
    A.nsr = nsr;
    A.np = np;
    A.R = 2 * nsr + 1;
    A.R16 = (A.R + 15) / 16 * 16;
    A.KS = static_cast<int>(sr_gram_slab_cols(A.R16));
    A.pitch = A.KS + 1;
    A.ore = ore;
    A.oim = oim;
    A.F = F;
    A.w = w;
    A.mean = mean;
    hipLaunchKernelGGL(k_sr_weights, dim3(1), dim3(256), 0, st, logpsi, nsr, w);
    hipLaunchKernelGGL(k_sr_mean, dim3(blocks256(np)), dim3(256), 0, st, A, mean);
    const int64_t nb = sr_partial_blocks(np);
    const int64_t cols = (np + nb - 1) / nb;
    const int nt = A.R16 / 16;
    const int groups = (nt * (nt + 1) / 2 + kSrTilesPerGroup - 1) / kSrTilesPerGroup;
    const size_t lds = sizeof(double) * static_cast<size_t>(A.R16) * A.pitch;
    hipLaunchKernelGGL(k_sr_gram, dim3(static_cast<unsigned>(nb), static_cast<unsigned>(groups)), dim3(64 * kSrWaves),
                       lds, st, A, cols, partial);
    const int64_t RR = static_cast<int64_t>(A.R) * A.R;
    double* tmp = partial + nb * A.R16 * A.R16;   // kSrRed R^2 doubles after the partials
    hipLaunchKernelGGL(k_sr_reduce, dim3(blocks256(RR), kSrRed), dim3(256), 0, st, partial, static_cast<int>(nb), A.R16,
                       A.R, tmp);
    hipLaunchKernelGGL(k_sr_reduce2, dim3(blocks256(RR)), dim3(256), 0, st, tmp, RR, T);
    const int n = 2 * nsr;
    const int P = (n + 1 + 31) / 32;   // row blocks of the augmented matrix
    if (P > kCholMaxRows / 32)
        hipLaunchKernelGGL(k_sr_chol, dim3(1), dim3(64), 0, st, T, n, A.R, lambda, L, y, err);
    else if (P <= 2)
        launch_chol_reg<2>(T, n, A.R, lambda, y, err, st);
    else if (P <= 4)
        launch_chol_reg<4>(T, n, A.R, lambda, y, err, st);
    else if (P <= 6)
        launch_chol_reg<6>(T, n, A.R, lambda, y, err, st);
    else if (P == 7)
        launch_chol_reg<7>(T, n, A.R, lambda, y, err, st);
    else
        launch_chol_reg<8>(T, n, A.R, lambda, y, err, st);
    hipLaunchKernelGGL(k_sr_update, dim3(blocks256(np)), dim3(256), 0, st, A, y, lambda, d);
    return hipGetLastError();
}

}  // namespace eloc
