/*
 * Oracle for the sample-aware local energy E_loc^var (plain CPU, FP64).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is compared against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code with the
 * GPU library.
 *
 * What it computes, in the paper's order and notation (arXiv 2408.07625):
 *
 *   - terms (h_l, XY_l, YZ_l), Y_l = XY_l & YZ_l (Sec. "Hamiltonian
 *     arithmetic"; XY = X|Y, YZ = Y|Z);
 *   - the unique set of XY masks in first-appearance order, each with its
 *     term set P_XY kept in caller order (Sec. "Unique XY", Eq. xy_to_yz_set);
 *   - FindCoupledPairs by looping over the unique XY set (Algorithm 2A):
 *     for each sampled x, for each XY, x' = x ^ XY, keep x' if it is in U
 *     (membership by binary search in a sorted copy of U, the lookup the
 *     paper attributes to Wu et al.);
 *   - MatrixElement (supplementary algorithm): H_xx' = sum over P_{x^x'} of
 *     h_l exp(i phi), phi = (pi/2)|Y_l| + pi |x' & YZ_l|  (Eq. pauli_melem),
 *     evaluated as i^k, k = (|Y_l| + 2|x' & YZ_l|) mod 4, which is exact;
 *   - E_loc^var(x) = sum_{x' in U coupled to x} H_xx' psi(x')/psi(x)
 *     (Eq. local_energy restricted to U), psi(x')/psi(x) = exp(L' - L);
 *   - the weighted energy of Eq. variational_energy (weights |psi|^2
 *     renormalised over U) or of Eq. energy_estimator_via_unique (occurrence
 *     counts), plus the weighted variance sum w~ |E_loc - E|^2;
 *   - the derivative of that energy with respect to the log-amplitudes.
 *
 * Keys and masks: W = ceil(N/64) uint64 words, qubit q in word q/64, bit
 * q%64.  Complex numbers are (re, im) double pairs.
 */
#include <complex.h>
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXW 2

typedef struct {
    uint64_t k[MAXW];
    int64_t idx;
} rec_t;

static int W_cmp;  /* words compared by rec_cmp (set before qsort/bsearch) */

static int rec_cmp(const void* a, const void* b) {
    const rec_t* x = (const rec_t*)a;
    const rec_t* y = (const rec_t*)b;
    for (int w = W_cmp - 1; w >= 0; --w) {
        if (x->k[w] < y->k[w]) return -1;
        if (x->k[w] > y->k[w]) return 1;
    }
    return 0;
}

static int rec_cmp_idx(const void* a, const void* b) {
    int c = rec_cmp(a, b);
    if (c) return c;
    const rec_t* x = (const rec_t*)a;
    const rec_t* y = (const rec_t*)b;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* ---------------------------------------------------------------------- */
/* Hamiltonian tables: unique XY set in first-appearance order              */
/* ---------------------------------------------------------------------- */
typedef struct {
    int N, W;
    int64_t n_terms, n_groups;
    const double* coeff;
    const uint64_t* xy;
    const uint64_t* yz;
    uint64_t* grp_xy;      /* [G][W]                                      */
    int64_t* grp_begin;    /* [G+1] into term_of                           */
    int64_t* term_of;      /* term indices, grouped, caller order inside   */
    rec_t* xy_sorted;      /* [G] (XY, group id) sorted by XY for lookup  */
} ham_t;

typedef struct {
    int64_t first;
    int64_t begin, end;   /* run in the sorted term records */
} run_t;

static int run_cmp(const void* a, const void* b) {
    const run_t* x = (const run_t*)a;
    const run_t* y = (const run_t*)b;
    return (x->first > y->first) - (x->first < y->first);
}

static void ham_free(ham_t* H) {
    free(H->grp_xy);
    free(H->grp_begin);
    free(H->term_of);
    free(H->xy_sorted);
}

static int ham_build(ham_t* H, int N, int64_t n_terms, const double* coeff,
                     const uint64_t* xy, const uint64_t* yz) {
    memset(H, 0, sizeof(*H));
    H->N = N;
    H->W = (N + 63) / 64;
    H->n_terms = n_terms;
    H->coeff = coeff;
    H->xy = xy;
    H->yz = yz;
    int W = H->W;
    if (W > MAXW || n_terms <= 0) return -1;
    rec_t* r = (rec_t*)malloc(sizeof(rec_t) * (size_t)n_terms);
    for (int64_t l = 0; l < n_terms; ++l) {
        memset(r[l].k, 0, sizeof(r[l].k));
        for (int w = 0; w < W; ++w) r[l].k[w] = xy[l * W + w];
        r[l].idx = l;
    }
    W_cmp = W;
    qsort(r, (size_t)n_terms, sizeof(rec_t), rec_cmp_idx);
    /* runs of equal XY; the smallest caller index of a run is its first appearance */
    int64_t G = 0;
    run_t* runs = (run_t*)malloc(sizeof(run_t) * (size_t)n_terms);
    for (int64_t a = 0; a < n_terms;) {
        int64_t b = a + 1;
        while (b < n_terms && rec_cmp(&r[a], &r[b]) == 0) ++b;
        runs[G].first = r[a].idx;
        runs[G].begin = a;
        runs[G].end = b;
        ++G;
        a = b;
    }
    qsort(runs, (size_t)G, sizeof(run_t), run_cmp);
    H->n_groups = G;
    H->grp_xy = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(G * W));
    H->grp_begin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(G + 1));
    H->term_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_terms);
    H->xy_sorted = (rec_t*)malloc(sizeof(rec_t) * (size_t)G);
    int64_t pos = 0;
    for (int64_t g = 0; g < G; ++g) {
        H->grp_begin[g] = pos;
        for (int64_t t = runs[g].begin; t < runs[g].end; ++t) H->term_of[pos++] = r[t].idx;
        for (int w = 0; w < W; ++w) H->grp_xy[g * W + w] = r[runs[g].begin].k[w];
        H->xy_sorted[g] = r[runs[g].begin];
        H->xy_sorted[g].idx = g;
    }
    H->grp_begin[G] = pos;
    qsort(H->xy_sorted, (size_t)G, sizeof(rec_t), rec_cmp);
    free(runs);
    free(r);
    return 0;
}

/* XY -> group id, or -1 if XY is not in the unique set */
static int64_t ham_find_group(const ham_t* H, const uint64_t* xymask) {
    rec_t q;
    memset(&q, 0, sizeof(q));
    for (int w = 0; w < H->W; ++w) q.k[w] = xymask[w];
    W_cmp = H->W;
    const rec_t* f = (const rec_t*)bsearch(&q, H->xy_sorted, (size_t)H->n_groups, sizeof(rec_t), rec_cmp);
    return f ? f->idx : -1;
}

/* ---------------------------------------------------------------------- */
/* U as an ordered table                                                    */
/* ---------------------------------------------------------------------- */
typedef struct {
    int W;
    int64_t M;
    rec_t* sorted;
} table_t;

static int table_build(table_t* T, int W, int64_t M, const uint64_t* keys) {
    T->W = W;
    T->M = M;
    T->sorted = (rec_t*)malloc(sizeof(rec_t) * (size_t)(M > 0 ? M : 1));
    for (int64_t i = 0; i < M; ++i) {
        memset(T->sorted[i].k, 0, sizeof(T->sorted[i].k));
        for (int w = 0; w < W; ++w) T->sorted[i].k[w] = keys[i * W + w];
        T->sorted[i].idx = i;
    }
    W_cmp = W;
    qsort(T->sorted, (size_t)M, sizeof(rec_t), rec_cmp);
    for (int64_t i = 1; i < M; ++i)
        if (rec_cmp(&T->sorted[i - 1], &T->sorted[i]) == 0) return -2;  /* U must be unique */
    return 0;
}

static int64_t table_find(const table_t* T, const uint64_t* key) {
    rec_t q;
    memset(&q, 0, sizeof(q));
    for (int w = 0; w < T->W; ++w) q.k[w] = key[w];
    const rec_t* f = (const rec_t*)bsearch(&q, T->sorted, (size_t)T->M, sizeof(rec_t), rec_cmp);
    return f ? f->idx : -1;
}

/* ---------------------------------------------------------------------- */
/* MatrixElement                                                            */
/* ---------------------------------------------------------------------- */
static const double complex I_POW[4] = {1.0, I, -1.0, -I};

/* <x|P_l|x'> for a term of the group g (x ^ x' == XY_g already holds) */
static double complex pauli_element(const ham_t* H, int64_t l, const uint64_t* xprime) {
    int W = H->W;
    int ny = 0, nxz = 0;
    for (int w = 0; w < W; ++w) {
        uint64_t yzw = H->yz[l * W + w];
        ny += __builtin_popcountll(H->xy[l * W + w] & yzw);
        nxz += __builtin_popcountll(xprime[w] & yzw);
    }
    return I_POW[(ny + 2 * nxz) & 3];
}

static double complex matrix_element(const ham_t* H, int64_t g, const uint64_t* xprime) {
    double complex acc = 0.0;
    for (int64_t t = H->grp_begin[g]; t < H->grp_begin[g + 1]; ++t) {
        int64_t l = H->term_of[t];
        acc += H->coeff[l] * pauli_element(H, l, xprime);
    }
    return acc;
}

static double complex load_c(const double* a, int64_t i) { return a[2 * i] + I * a[2 * i + 1]; }

/* ---------------------------------------------------------------------- */
/* exported                                                                 */
/* ---------------------------------------------------------------------- */

void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* group id (first-appearance order) of every term; returns the group count */
int64_t oracle_groups(int n_qubits, int64_t n_terms, const uint64_t* xy, int64_t* group_of_term) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, NULL, xy, xy) != 0) return -1;
    for (int64_t g = 0; g < H.n_groups; ++g)
        for (int64_t t = H.grp_begin[g]; t < H.grp_begin[g + 1]; ++t) group_of_term[H.term_of[t]] = g;
    int64_t G = H.n_groups;
    ham_free(&H);
    return G;
}

/* E_loc^var for rows [row_begin, row_end) of U (caller order), plus the
 * number of coupled x' per row.  Returns 0, -1 bad input, -2 duplicate keys. */
int oracle_local_energy(int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                        const uint64_t* yz, int64_t n_unique, const uint64_t* keys,
                        const double* logpsi, int64_t row_begin, int64_t row_end,
                        double* eloc_out, int64_t* pairs_out) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, coeff, xy, yz) != 0) return -1;
    table_t T;
    int rc = table_build(&T, H.W, n_unique, keys);
    if (rc != 0) { ham_free(&H); free(T.sorted); return rc; }
    int W = H.W;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = row_begin; i < row_end; ++i) {
        const uint64_t* x = keys + i * W;
        double complex Li = load_c(logpsi, i);
        double complex e = 0.0;
        int64_t npairs = 0;
        uint64_t xp[MAXW] = {0, 0};
        for (int64_t g = 0; g < H.n_groups; ++g) {           /* Algorithm 2A */
            for (int w = 0; w < W; ++w) xp[w] = x[w] ^ H.grp_xy[g * W + w];
            int64_t j = table_find(&T, xp);
            if (j < 0) continue;
            double complex Hij = matrix_element(&H, g, xp);
            e += Hij * cexp(load_c(logpsi, j) - Li);
            ++npairs;
        }
        eloc_out[2 * (i - row_begin)] = creal(e);
        eloc_out[2 * (i - row_begin) + 1] = cimag(e);
        if (pairs_out) pairs_out[i - row_begin] = npairs;
    }
    free(T.sorted);
    ham_free(&H);
    return 0;
}

/* Coupled pairs (i, j, g) with i in [row_begin, row_end), sorted by (i, j),
 * plus H_ij.  Writes at most `capacity` pairs, returns the total count in
 * *n_pairs (so a too-small capacity can be detected), or <0 on error. */
typedef struct { int64_t j, g; } jg_t;
static int jg_cmp(const void* a, const void* b) {
    const jg_t* x = (const jg_t*)a;
    const jg_t* y = (const jg_t*)b;
    return (x->j > y->j) - (x->j < y->j);
}

int oracle_find_pairs(int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                      const uint64_t* yz, int64_t n_unique, const uint64_t* keys,
                      int64_t row_begin, int64_t row_end, int64_t capacity,
                      int32_t* pi, int32_t* pj, int32_t* pg, double* hij, int64_t* n_pairs) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, coeff, xy, yz) != 0) return -1;
    table_t T;
    int rc = table_build(&T, H.W, n_unique, keys);
    if (rc != 0) { ham_free(&H); free(T.sorted); return rc; }
    int W = H.W;
    int64_t count = 0;
    jg_t* buf = (jg_t*)malloc(sizeof(jg_t) * (size_t)(H.n_groups > 0 ? H.n_groups : 1));
    uint64_t xp[MAXW] = {0, 0};
    for (int64_t i = row_begin; i < row_end; ++i) {
        const uint64_t* x = keys + i * W;
        int64_t nb = 0;
        for (int64_t g = 0; g < H.n_groups; ++g) {
            for (int w = 0; w < W; ++w) xp[w] = x[w] ^ H.grp_xy[g * W + w];
            int64_t j = table_find(&T, xp);
            if (j >= 0) { buf[nb].j = j; buf[nb].g = g; ++nb; }
        }
        qsort(buf, (size_t)nb, sizeof(jg_t), jg_cmp);
        for (int64_t b = 0; b < nb; ++b, ++count) {
            if (count >= capacity) continue;
            pi[count] = (int32_t)i;
            pj[count] = (int32_t)buf[b].j;
            pg[count] = (int32_t)buf[b].g;
            if (hij) {
                double complex h = matrix_element(&H, buf[b].g, keys + buf[b].j * W);
                hij[2 * count] = creal(h);
                hij[2 * count + 1] = cimag(h);
            }
        }
    }
    *n_pairs = count;
    free(buf);
    free(T.sorted);
    ham_free(&H);
    return 0;
}

/* MatrixElement(x, x') for arbitrary pairs of keys: 0 if x ^ x' is not an XY
 * of the Hamiltonian. */
int oracle_matrix_elements(int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                           const uint64_t* yz, int64_t n, const uint64_t* x, const uint64_t* xprime,
                           double* out) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, coeff, xy, yz) != 0) return -1;
    int W = H.W;
    uint64_t d[MAXW] = {0, 0};
    for (int64_t p = 0; p < n; ++p) {
        for (int w = 0; w < W; ++w) d[w] = x[p * W + w] ^ xprime[p * W + w];
        int64_t g = ham_find_group(&H, d);
        double complex h = g < 0 ? 0.0 : matrix_element(&H, g, xprime + p * W);
        out[2 * p] = creal(h);
        out[2 * p + 1] = cimag(h);
    }
    ham_free(&H);
    return 0;
}

/* Phase exponents of Eq. pauli_melem for arbitrary pairs of keys: for pair
 * p, with g the group of x ^ x' (none: no terms), offsets[p + 1] - offsets[p]
 * = |P_g| and k[offsets[p] + t] = (|Y_l| + 2 |x' & YZ_l|) mod 4 for the t-th
 * term l of P_g in ascending caller index, so <x|P_l|x'> = i^k.  offsets has
 * n + 1 entries (offsets[0] = 0); k is written only while it fits in
 * `capacity`.  Returns the total number of exponents, or < 0 on error. */
int64_t oracle_phase_exponents(int n_qubits, int64_t n_terms, const uint64_t* xy, const uint64_t* yz,
                               int64_t n, const uint64_t* x, const uint64_t* xprime,
                               int64_t* offsets, uint8_t* k, int64_t capacity) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, NULL, xy, yz) != 0) return -1;
    int W = H.W;
    uint64_t d[MAXW] = {0, 0};
    int64_t pos = 0;
    offsets[0] = 0;
    for (int64_t p = 0; p < n; ++p) {
        for (int w = 0; w < W; ++w) d[w] = x[p * W + w] ^ xprime[p * W + w];
        int64_t g = ham_find_group(&H, d);
        if (g >= 0) {
            for (int64_t t = H.grp_begin[g]; t < H.grp_begin[g + 1]; ++t, ++pos) {
                int64_t l = H.term_of[t];
                int ny = 0, nxz = 0;
                for (int w = 0; w < W; ++w) {
                    ny += __builtin_popcountll(xy[l * W + w] & yz[l * W + w]);
                    nxz += __builtin_popcountll(xprime[p * W + w] & yz[l * W + w]);
                }
                if (pos < capacity) k[pos] = (uint8_t)((ny + 2 * nxz) & 3);
            }
        }
        offsets[p + 1] = pos;
    }
    ham_free(&H);
    return pos;
}

/* Normalised weights: w_i / sum w (counts) or |psi_i|^2 / sum |psi|^2. */
static double* normalised_weights(int64_t M, const double* logpsi, const double* weights, double* total) {
    double* wt = (double*)malloc(sizeof(double) * (size_t)M);
    double s = 0.0;
    if (weights) {
        for (int64_t i = 0; i < M; ++i) { wt[i] = weights[i]; s += wt[i]; }
        *total = s;
    } else {
        double c = -INFINITY;
        for (int64_t i = 0; i < M; ++i) c = fmax(c, logpsi[2 * i]);
        for (int64_t i = 0; i < M; ++i) { wt[i] = exp(2.0 * (logpsi[2 * i] - c)); s += wt[i]; }
        *total = s * exp(2.0 * c);
    }
    for (int64_t i = 0; i < M; ++i) wt[i] /= s;
    return wt;
}

/* stats = {Re E, Im E, Var, sum of raw weights}. */
int oracle_energy(int64_t n_unique, const double* eloc, const double* logpsi, const double* weights,
                  double* stats) {
    double total;
    double* wt = normalised_weights(n_unique, logpsi, weights, &total);
    double complex E = 0.0;
    for (int64_t i = 0; i < n_unique; ++i) E += wt[i] * load_c(eloc, i);
    double var = 0.0;
    for (int64_t i = 0; i < n_unique; ++i) {
        double complex d = load_c(eloc, i) - E;
        var += wt[i] * (creal(d) * creal(d) + cimag(d) * cimag(d));
    }
    stats[0] = creal(E);
    stats[1] = cimag(E);
    stats[2] = var;
    stats[3] = total;
    free(wt);
    return 0;
}

/* Gradient of a real loss through E with respect to L = log psi, rows
 * [row_begin, row_end).  grad_e = dLoss/dRe E + i dLoss/dIm E.  E is
 * holomorphic in L for fixed weights:
 *   dE/dL_y = (1/sum w) [ sum_{x coupled to y} w_x H_xy exp(L_y - L_x) - w_y E_loc(y) ]
 * and grad_L_y = grad_e * conj(dE/dL_y).  With |psi|^2 weights (weights NULL)
 * the weights depend on Re L as well, adding 2 w~_y Re(conj(grad_e)(E_loc(y) - E))
 * to the real part.  H_xy = <x|H|y> is evaluated with the ket y.
 * eloc_rows holds E_loc for the same rows; energy = {Re E, Im E} is needed
 * only for |psi|^2 weights. */
int oracle_adjoint(int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                   const uint64_t* yz, int64_t n_unique, const uint64_t* keys, const double* logpsi,
                   const double* weights, const double* eloc_rows, const double* energy,
                   double grad_re, double grad_im, int64_t row_begin, int64_t row_end,
                   double* grad_out) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, coeff, xy, yz) != 0) return -1;
    table_t T;
    int rc = table_build(&T, H.W, n_unique, keys);
    if (rc != 0) { ham_free(&H); free(T.sorted); return rc; }
    int W = H.W;
    double total;
    double* wt = normalised_weights(n_unique, logpsi, weights, &total);
    double complex ge = grad_re + I * grad_im;
    double complex E = energy ? energy[0] + I * energy[1] : 0.0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t y = row_begin; y < row_end; ++y) {
        const uint64_t* ky = keys + y * W;
        double complex Ly = load_c(logpsi, y);
        double complex s = 0.0;
        uint64_t kx[MAXW] = {0, 0};
        for (int64_t g = 0; g < H.n_groups; ++g) {
            for (int w = 0; w < W; ++w) kx[w] = ky[w] ^ H.grp_xy[g * W + w];
            int64_t x = table_find(&T, kx);
            if (x < 0) continue;
            double complex Hxy = matrix_element(&H, g, ky);   /* ket y */
            s += wt[x] * Hxy * cexp(Ly - load_c(logpsi, x));
        }
        double complex Ey = load_c(eloc_rows, y - row_begin);
        double complex G = s - wt[y] * Ey;
        double complex gr = ge * conj(G);
        double re = creal(gr), im = cimag(gr);
        if (!weights) re += 2.0 * wt[y] * creal(conj(ge) * (Ey - E));
        grad_out[2 * (y - row_begin)] = re;
        grad_out[2 * (y - row_begin) + 1] = im;
    }
    free(wt);
    free(T.sorted);
    ham_free(&H);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Conventional local energy (Eq. local_energy over all x', not only U)     */
/* ---------------------------------------------------------------------- */

/* sum of |h_l| over the terms of group g: the scale of "H_xx' != 0" */
static double group_abs_sum(const ham_t* H, int64_t g) {
    double s = 0.0;
    for (int64_t t = H->grp_begin[g]; t < H->grp_begin[g + 1]; ++t) s += fabs(H->coeff[H->term_of[t]]);
    return s;
}

/* |H_xx'| > tol * sum_{l in P_g} |h_l|: the reading of "H_xx' != 0" that
 * treats strings cancelling in exact arithmetic (hopping strings between
 * particle-number sectors) as zero */
static int coupled_nonzero(const ham_t* H, int64_t g, const uint64_t* xprime, double tol) {
    double complex h = matrix_element(H, g, xprime);
    return cabs(h) > tol * group_abs_sum(H, g);
}

static int key_cmp_desc_words(const void* a, const void* b) {
    const uint64_t* x = (const uint64_t*)a;
    const uint64_t* y = (const uint64_t*)b;
    for (int w = W_cmp - 1; w >= 0; --w) {
        if (x[w] < y[w]) return -1;
        if (x[w] > y[w]) return 1;
    }
    return 0;
}

void oracle_free(void* p) { free(p); }

/* The states outside U that H couples to a sampled state: the x' of the sum
 * of Eq. local_energy that the sample-aware form leaves out,
 *   V = { x' not in U : x' = x ^ XY_g, x in U, |H_xx'| > tol sum_{l in P_g} |h_l| },
 * each once, sorted ascending as W-word integers (most significant word
 * first).  *out receives a malloc'ed [count][W] array (oracle_free).
 * Returns the count, -1 bad input, -2 duplicate keys in U. */
int64_t oracle_find_misses(int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                           const uint64_t* yz, int64_t n_unique, const uint64_t* keys, double tol,
                           uint64_t** out) {
    *out = NULL;
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, coeff, xy, yz) != 0) return -1;
    table_t T;
    int rc = table_build(&T, H.W, n_unique, keys);
    if (rc != 0) { ham_free(&H); free(T.sorted); return rc; }
    const int W = H.W;
    int nthreads = omp_get_max_threads();
    uint64_t** part = (uint64_t**)calloc((size_t)nthreads, sizeof(uint64_t*));
    int64_t* plen = (int64_t*)calloc((size_t)nthreads, sizeof(int64_t));
    int64_t* pcap = (int64_t*)calloc((size_t)nthreads, sizeof(int64_t));
#pragma omp parallel
    {
        const int t = omp_get_thread_num();
        uint64_t xp[MAXW] = {0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n_unique; ++i) {
            const uint64_t* x = keys + i * W;
            for (int64_t g = 0; g < H.n_groups; ++g) {
                for (int w = 0; w < W; ++w) xp[w] = x[w] ^ H.grp_xy[g * W + w];
                if (table_find(&T, xp) >= 0) continue;          /* in U: a pair of E_loc^var */
                if (!coupled_nonzero(&H, g, xp, tol)) continue;
                if (plen[t] == pcap[t]) {
                    pcap[t] = pcap[t] ? 2 * pcap[t] : 1024;
                    part[t] = (uint64_t*)realloc(part[t], sizeof(uint64_t) * (size_t)(pcap[t] * W));
                }
                for (int w = 0; w < W; ++w) part[t][plen[t] * W + w] = xp[w];
                ++plen[t];
            }
        }
    }
    int64_t total = 0;
    for (int t = 0; t < nthreads; ++t) total += plen[t];
    uint64_t* all = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)((total > 0 ? total : 1) * W));
    int64_t pos = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (plen[t]) memcpy(all + pos * W, part[t], sizeof(uint64_t) * (size_t)(plen[t] * W));
        pos += plen[t];
        free(part[t]);
    }
    free(part);
    free(plen);
    free(pcap);
    W_cmp = W;
    qsort(all, (size_t)total, sizeof(uint64_t) * (size_t)W, key_cmp_desc_words);
    int64_t n = 0;
    for (int64_t a = 0; a < total; ++a) {
        if (n > 0 && key_cmp_desc_words(all + a * W, all + (n - 1) * W) == 0) continue;
        if (n != a) memmove(all + n * W, all + a * W, sizeof(uint64_t) * (size_t)W);
        ++n;
    }
    *out = all;
    free(T.sorted);
    ham_free(&H);
    return n;
}

/* Conventional local energy of Eq. local_energy for rows [row_begin,
 * row_end) of U: E_loc(x) = sum over the XY groups g of H_{x x'} psi(x')/psi(x)
 * with x' = x ^ XY_g, the amplitudes taken from U (logpsi) or from the extra
 * states V (keys_v, logpsi_v; V disjoint from U).  A coupled x' found in
 * neither contributes only when |H_xx'| > tol sum |h| (the reading of
 * H_xx' != 0 above), and is then an error: its amplitude is missing.
 * Returns 0, -1 bad input, -2 duplicate keys in U or V, -3 missing state. */
int oracle_local_energy_full(int n_qubits, int64_t n_terms, const double* coeff, const uint64_t* xy,
                             const uint64_t* yz, int64_t n_unique, const uint64_t* keys, const double* logpsi,
                             int64_t n_v, const uint64_t* keys_v, const double* logpsi_v, double tol,
                             int64_t row_begin, int64_t row_end, double* eloc_out) {
    ham_t H;
    if (ham_build(&H, n_qubits, n_terms, coeff, xy, yz) != 0) return -1;
    const int W = H.W;
    /* one ordered table of U followed by V: index < n_unique is a sample of U */
    uint64_t* all = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)((n_unique + n_v) * W + 1));
    memcpy(all, keys, sizeof(uint64_t) * (size_t)(n_unique * W));
    if (n_v) memcpy(all + n_unique * W, keys_v, sizeof(uint64_t) * (size_t)(n_v * W));
    table_t T;
    int rc = table_build(&T, W, n_unique + n_v, all);
    if (rc != 0) { ham_free(&H); free(T.sorted); free(all); return rc; }
    int missing = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : missing)
    for (int64_t i = row_begin; i < row_end; ++i) {
        const uint64_t* x = keys + i * W;
        double complex Li = load_c(logpsi, i);
        double complex e = 0.0;
        uint64_t xp[MAXW] = {0, 0};
        for (int64_t g = 0; g < H.n_groups; ++g) {
            for (int w = 0; w < W; ++w) xp[w] = x[w] ^ H.grp_xy[g * W + w];
            int64_t j = table_find(&T, xp);
            if (j < 0) {
                if (coupled_nonzero(&H, g, xp, tol)) missing = 1;
                continue;
            }
            double complex Lj = j < n_unique ? load_c(logpsi, j) : load_c(logpsi_v, j - n_unique);
            e += matrix_element(&H, g, xp) * cexp(Lj - Li);
        }
        eloc_out[2 * (i - row_begin)] = creal(e);
        eloc_out[2 * (i - row_begin) + 1] = cimag(e);
    }
    free(T.sorted);
    free(all);
    ham_free(&H);
    return missing ? -3 : 0;
}
