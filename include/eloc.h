/*
 * eloc.h - C ABI of the MI355X (gfx950) engine for the sample-aware local
 * energy of arXiv 2408.07625 ("Neural quantum states and peaked molecular
 * wave functions: curse or blessing?").
 *
 * The engine evaluates, for a qubit Hamiltonian H = sum_l h_l P^(l)
 * (Eq. jw_hamiltonian) and a batch U of unique sampled basis vectors,
 *
 *     E_loc^var(x) = sum_{x' in U} H_xx' psi(x') / psi(x)       (x in U)
 *
 * (Eq. local_energy restricted to U, Sec. "Streamlined local energy
 * calculations"), and the weighted energy of Eq. variational_energy.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A Pauli term is (h_l, XY_l, YZ_l) with XY = X|Y and YZ = Y|Z as N-bit
 *    vectors (Sec. "Hamiltonian arithmetic"); Y_l = XY_l & YZ_l.
 *  - Bit vectors are W = ceil(N/64) uint64 words, row-major [count][W]:
 *    qubit q lives in word q/64, bit q%64.  Bits >= N must be zero.
 *    N <= 128 (W <= 2).
 *  - <x|P^(l)|x'> = i^(|Y_l| + 2|x' & YZ_l|) if x ^ x' == XY_l, else 0
 *    (Eq. pauli_melem; the phase is taken on the ket x').
 *  - Two samples are coupled when x ^ x' equals one of the Hamiltonian's
 *    XY masks (the unique-XY set); a coupled pair can have H_xx' == 0.
 *    Coupled pairs are ordered pairs and include x == x' when the
 *    Hamiltonian has a diagonal term.
 *  - The unique-XY set is numbered in first-appearance order of the terms
 *    as passed to eloc_set_hamiltonian ("group id").
 *  - Complex numbers are eloc_c64 = {re, im} doubles (the layout of
 *    complex128).  Log-amplitudes are L = log psi = log|psi| + i phase.
 *  - "DEVICE" pointers are device memory of the context's device; "HOST"
 *    pointers are ordinary host memory.  The caller owns every pointer it
 *    passes; the library copies what it keeps.
 *  - Every call returns an eloc_status (0 = OK, < 0 error) and never
 *    throws.  eloc_last_error() gives the text of the last failure.
 *  - Work is enqueued on the context's stream; calls return before the
 *    GPU finishes unless documented as synchronising.  A context is not
 *    thread-safe; use one per host thread.
 *  - Many problems at once: the eloc_batch_* calls at the end evaluate a
 *    set of (Hamiltonian, U) problems of uneven size in one pipeline
 *    replayed from a HIP graph.
 */
#ifndef ELOC_H
#define ELOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eloc_ctx_s* eloc_ctx;
typedef struct {
    double re, im;
} eloc_c64;

enum eloc_status {
    ELOC_OK = 0,
    ELOC_EINVAL = -1,    /* bad argument (null pointer, size, bits >= N, bad weights) */
    ELOC_EDUP = -2,      /* U contains the same key twice (U must be unique)          */
    ELOC_ENOMEM = -3,    /* device allocation failed                                 */
    ELOC_ECAPACITY = -4, /* caller buffer too small; the required size is returned   */
    ELOC_ERANGE = -5,    /* log-amplitude spread too wide for the FP32 form          */
    ELOC_EHIP = -6,      /* HIP runtime error                                        */
    ELOC_ESTATE = -7,    /* call order: Hamiltonian or samples not set               */
    ELOC_EAGAIN = -8     /* a hash table overflowed and was rebuilt; repeat the call  */
};

/* FindCoupledPairs variants (Sec. "FindCoupledPairs implementations"). */
enum eloc_variant {
    ELOC_TERMS = 0, /* loop over the unique XY set, look x ^ XY up in U (Alg. 2A)   */
    ELOC_BATCH = 1, /* loop over U, look x ^ x' up in the XY set (Alg. 2B)           */
    ELOC_TRIE = 2,  /* walk prefix trees of U and of the XY set together (Alg. 2C)   */
    ELOC_AUTO = 3,  /* ELOC_BATCH if |U| <= |unique XY set|, else ELOC_TERMS         */
    ELOC_STORED = 4 /* forward / adjoint only: the pair list kept by eloc_store_pairs */
};

/* Arithmetic of the ratio accumulation sum_x' H_xx' psi(x')/psi(x). */
enum eloc_precision {
    ELOC_FP64 = 0,  /* complex double throughout                                    */
    ELOC_FP32C = 1  /* FP32 with error-free transforms (hi+lo pairs); FP64 only in
                       the weighted energy / variance reductions                    */
};

/* Create a context on `device` enqueuing on `hip_stream` (a hipStream_t,
 * NULL = the device's null stream).  *out receives the handle. */
int eloc_create(eloc_ctx* out, int device, void* hip_stream);

/* Free the context and every device buffer it owns (synchronises). */
void eloc_destroy(eloc_ctx ctx);

/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char* eloc_last_error(eloc_ctx ctx);

/* Change the stream later work is enqueued on. */
int eloc_set_stream(eloc_ctx ctx, void* hip_stream);

/* Store the Hamiltonian (Sec. "Preparation" of the supplementary GPU notes:
 * the unique XY set with, per XY, its contiguous run of terms).  HOST
 * arrays: coeff[n_terms], xy[n_terms][W], yz[n_terms][W].  Equal Pauli
 * strings may repeat (their coefficients add).  Synchronising.
 * Errors: EINVAL (n_qubits not in 1..128, n_terms < 1, bits >= N),
 * ENOMEM, EHIP. */
int eloc_set_hamiltonian(eloc_ctx ctx, int n_qubits, int64_t n_terms, const double* coeff,
                         const uint64_t* xy, const uint64_t* yz);

/* Number of unique XY masks and of terms of the stored Hamiltonian. */
int eloc_hamiltonian_info(eloc_ctx ctx, int64_t* n_groups, int64_t* n_terms, int* n_qubits);

/* Store the batch U of unique samples (the sampler's output, Sec.
 * "Sampling without replacement"; U holds each sampled basis vector once,
 * Eq. energy_estimator_via_unique).  DEVICE keys_dev[n_unique][W] in any
 * order, copied; sample index i below always means row i of this array.
 * Asynchronous: the copy, the membership table, the duplicate and bit
 * checks and the prefilter parameters of U are all computed on the device.
 * A key that repeats or has bits >= N is reported by the next synchronising
 * call (eloc_check, eloc_count_pairs, eloc_find_pairs, eloc_store_pairs)
 * as EDUP / EINVAL; until then the pair kernels do no work and the outputs
 * of eloc_local_energy / adjoint are unspecified.  eloc_check returns
 * EAGAIN (after rebuilding it) if U's membership table did not settle,
 * which invalidates the calls made since.
 * Errors (immediate): EINVAL (n_unique < 1 or >= 2^24, null keys),
 * ESTATE (no Hamiltonian), ENOMEM, EHIP. */
int eloc_set_samples(eloc_ctx ctx, int64_t n_unique, const uint64_t* keys_dev);

/* Geometry of U's membership table (two-choice cuckoo hashing with a stash):
 * HOST outputs, each optional (NULL skips it): n_unique, table_slots (slot
 * count, a power of two of at least 4 n_unique), table_stash (keys held in
 * the stash, 0..32; reading it synchronises).  Errors: ESTATE (no samples
 * set). */
int eloc_samples_info(eloc_ctx ctx, int64_t* n_unique, int64_t* table_slots, int* table_stash);

/* Forward pass (Eq. local_energy restricted to U: the sample-aware local
 * energy; weighted energy of Eq. variational_energy or
 * Eq. energy_estimator_via_unique).  DEVICE inputs logpsi_dev[n_unique] (complex log psi) and
 * weights_dev[n_unique] or NULL; DEVICE outputs eloc_dev[n_unique] and
 * stats_dev[4].  weights NULL: w = |psi|^2 renormalised over U
 * (Eq. variational_energy); else w >= 0 with sum w > 0, renormalised by
 * its sum (Eq. energy_estimator_via_unique with occurrence counts).
 * stats = {Re E, Im E, Var, sum of raw weights}, E = sum w~ E_loc,
 * Var = sum w~ |E_loc - E|^2.  Asynchronous: invalid weights or an FP32C
 * range failure are reported by the next synchronising call
 * (eloc_check) as EINVAL / ERANGE and the outputs are then unspecified.
 * Re L must be finite with max Re L - min Re L <= 60 for ELOC_FP32C and
 * <= 700 for ELOC_FP64 (exp(L - max Re L) and its inverse stay normal),
 * else ERANGE (deferred).
 * Errors (immediate): EINVAL (variant/precision), ESTATE. */
int eloc_local_energy(eloc_ctx ctx, int variant, int precision, const eloc_c64* logpsi_dev,
                      const double* weights_dev, eloc_c64* eloc_dev, double* stats_dev);

/* The forward pass of eloc_local_energy, allocating nothing: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and deferred errors as eloc_local_energy, bit for bit.  The amplitudes,
 * partial row sums and reduction scratch live in a fixed workspace of
 * 64 MiB per device that the library holds from its first eloc_create on
 * that device until the process ends; about 64 bytes per sample (FP32C) or
 * 32 (FP64) plus 16 per sample and inner-loop chunk must fit (2^18 samples
 * do at the 100-qubit workload; ECAPACITY, with the size needed in
 * eloc_last_error, when they do not).  Every context on a device shares
 * that device's workspace: calls that overlap on one device (several
 * contexts or streams) race.  Variants ELOC_TERMS, ELOC_BATCH, ELOC_AUTO
 * and ELOC_STORED; ELOC_TRIE is EINVAL (its sorted copy of U is built on
 * first use).  U's Bloom filter is not used.  The context's own buffers
 * (Hamiltonian, U's tables) come from eloc_set_hamiltonian and
 * eloc_set_samples, which allocate only when U grows.
 * Errors (immediate): EINVAL, ESTATE, ECAPACITY, EHIP. */
int eloc_local_energy_noalloc(eloc_ctx ctx, int variant, int precision, const eloc_c64* logpsi_dev,
                              const double* weights_dev, eloc_c64* eloc_dev, double* stats_dev);

/* Wait for the context's stream and report a deferred device-side error:
 * first of the current samples (EINVAL, EDUP, EAGAIN as in
 * eloc_set_samples), then of the last eloc_local_energy / adjoint /
 * pair_elements call (EINVAL, ERANGE, ECAPACITY).  A run error is reported
 * once (this call clears it), and eloc_set_samples clears it too.
 * Synchronising. */
int eloc_check(eloc_ctx ctx);

/* Number of coupled ordered pairs (x, x') in U x U, diagonal included:
 * the size of the set that FindCoupledPairs returns (Sec. "Streamlined
 * local energy calculations"; Alg. 2A, 2B and 2C give the same set), which
 * is the number of terms in the sum of Eq. local_energy restricted to U.
 * Synchronising; EDUP / EINVAL if the current samples are invalid. */
int eloc_count_pairs(eloc_ctx ctx, int variant, int64_t* n_pairs_host);

/* The coupled pairs themselves: DEVICE i_dev/j_dev/g_dev[capacity] receive
 * (sample i, sample j, group id of x_i ^ x_j), sorted by (i, j) ascending
 * (the row-major order of the paper's pair arrays, x->U and x'->U).
 * *n_pairs_host receives the pair count; ECAPACITY if it exceeds
 * `capacity` (nothing useful written).  Synchronising. */
int eloc_find_pairs(eloc_ctx ctx, int variant, int64_t capacity, int32_t* i_dev, int32_t* j_dev,
                    int32_t* g_dev, int64_t* n_pairs_host);

/* MatrixElement (supplementary algorithm; Eq. pauli_melem) for n given
 * pairs of samples: DEVICE i_dev/j_dev[n] sample indices, h_dev[n]
 * receives H_{x_i x_j} = sum over the terms l of the group of x_i ^ x_j of
 * h_l i^(k_l), k_l = (|Y_l| + 2 |x_j & YZ_l|) mod 4 (phase on the ket
 * x_j); 0 when x_i ^ x_j is not an XY mask of H.
 * Optional phase exponents (both DEVICE, NULL skips them):
 *   term_offsets_dev[n + 1] receives the exclusive prefix sum of the pairs'
 *     term counts |P_{x_i ^ x_j}| (0 for an uncoupled pair), so that
 *     term_offsets_dev[n] is the total;
 *   k_dev[k_capacity] (needs term_offsets_dev) receives, for pair t at
 *     [term_offsets[t], term_offsets[t + 1]), the exponent k_l in {0,1,2,3}
 *     of every term l of the group in ascending caller index l (the term
 *     set P_XY of Eq. xy_to_yz_set, in the caller's order).  If the total
 *     exceeds k_capacity nothing is written to k_dev and eloc_check
 *     reports ECAPACITY; call once with k_dev NULL to learn the total.
 * EINVAL (deferred, eloc_check) if an index is outside U.  Asynchronous. */
int eloc_pair_elements(eloc_ctx ctx, int64_t n, const int32_t* i_dev, const int32_t* j_dev,
                       eloc_c64* h_dev, int64_t* term_offsets_dev, uint8_t* k_dev, int64_t k_capacity);

/* Adjoint of the forward energy: the derivative of E with respect to the
 * log-amplitudes, which the parameter gradient of Eq. grad_def is built from
 * (the chain rule through log psi(x; theta) is the caller's).  The paper
 * gives no adjoint; this is the derivative of Eq. local_energy restricted to
 * U and of the weighted sum of Eq. variational_energy / counts.  For a real loss with upstream
 * grad_e = dLoss/dRe E + i dLoss/dIm E, writes DEVICE grad_logpsi_dev[n]
 * = dLoss/dRe L + i dLoss/dIm L.  With fixed weights E is holomorphic in L:
 *   dE/dL_y = sum_{x coupled to y} w~_x H_xy psi(y)/psi(x) - w~_y E_loc(y)
 * (H_xy = <x|H|y>, phase on the ket y) and grad_L_y = grad_e conj(dE/dL_y);
 * with |psi|^2 weights (weights_dev NULL) the real part gains
 * 2 w~_y Re(conj(grad_e) (E_loc(y) - E)).  eloc_dev and stats_dev are the
 * forward outputs for the same inputs.  Pairs are found again by the
 * variant's kernels, or read from the stored list (ELOC_STORED).
 * Errors as eloc_local_energy. */
int eloc_local_energy_adjoint(eloc_ctx ctx, int variant, int precision,
                              const eloc_c64* logpsi_dev, const double* weights_dev,
                              const eloc_c64* eloc_dev, const double* stats_dev, eloc_c64 grad_e,
                              eloc_c64* grad_logpsi_dev);

/* The conventional local energy (Eq. local_energy summed over every x',
 * the estimator that Sec. "Streamlined local energy calculations" replaces
 * by the sample-aware sum over U) needs the amplitudes of the states outside
 * U that H couples to U.  eloc_find_misses lists them: every
 * x' = x ^ XY_g (x in U, XY_g a mask of H) that is not in U and whose
 * matrix element is non-zero, read as |H_xx'| > tol * sum_{l in P_g} |h_l|
 * (FP64; strings that cancel exactly, such as hopping strings between
 * particle-number sectors, give no state; tol >= 0, 1e-10 is a good value).
 * DEVICE keys_dev[capacity][W] receives them once each, sorted ascending as
 * W-word integers (word W-1 most significant); *n_misses_host receives
 * their count, ECAPACITY (nothing written) if it exceeds capacity (call with
 * capacity 0 to learn it).  Synchronising; EDUP / EINVAL for invalid
 * samples.  One-word keys of at most 30 qubits are deduplicated in a bitmap
 * over the key space (2^(N-3) bytes of device memory); other keys are
 * listed, sorted and deduplicated, with ECAPACITY beyond 2^31 states before
 * deduplication. */
int eloc_find_misses(eloc_ctx ctx, double tol, int64_t capacity, uint64_t* keys_dev, int64_t* n_misses_host);

/* Conventional local energy of Eq. local_energy for every sample of U:
 * E_loc(x) = sum_{x'} H_xx' psi(x')/psi(x) over U and the extra states V,
 * DEVICE extra_keys_dev[n_extra][W] with extra_logpsi_dev[n_extra] (the
 * list of eloc_find_misses in any order, with the ansatz's log-amplitudes;
 * V must not meet U or repeat a key: EDUP).  A coupled state in neither U
 * nor V is skipped, so V must hold every state with a non-zero matrix
 * element.  DEVICE outputs eloc_dev[n_unique] and stats_dev[4] as in
 * eloc_local_energy (weights over U only).  LoopOverTerms over U's rows
 * with membership in U and V; |U| + n_extra < 2^24.  Synchronising; the
 * deferred errors of eloc_local_energy are returned directly. */
int eloc_local_energy_full(eloc_ctx ctx, int precision, const eloc_c64* logpsi_dev, const double* weights_dev,
                           int64_t n_extra, const uint64_t* extra_keys_dev, const eloc_c64* extra_logpsi_dev,
                           eloc_c64* eloc_dev, double* stats_dev);

/* Stochastic reconfiguration over the highest-probability samples
 * (Sec. "ANQS-tailored stochastic reconfiguration": the quantum geometric
 * tensor of Eq. qgt_definition is estimated only over the N_SR unique
 * samples of highest probability, with their probabilities renormalised
 * over that set).
 *
 * eloc_sr_select: DEVICE idx_dev[n_sr] receives the indices of the n_sr
 * entries of logpsi_dev[n] with the largest Re log psi (largest |psi|),
 * in descending order, ties to the lower index.  Works on any log-amplitude
 * array (no Hamiltonian or samples needed); uses the context's sort scratch.
 * Asynchronous.  Errors: EINVAL (1 <= n_sr <= n < 2^31). */
int eloc_sr_select(eloc_ctx ctx, int64_t n, const eloc_c64* logpsi_dev, int n_sr, int32_t* idx_dev);

/* eloc_sr_solve: the SR-transformed gradient d = (Re S + lambda I)^{-1} F for
 * real parameters theta.  DEVICE inputs: o_re_dev / o_im_dev [n_sr][n_params]
 * row-major, the real and imaginary parts of O_xp = d log psi(x) / d theta_p
 * (d log|psi| and d phase) of the set's samples; logpsi_set_dev[n_sr] their
 * log-amplitudes (weights w_x = |psi_x|^2 / sum over the set); grad_dev
 * [n_params] the energy gradient F (Eq. grad_def); lambda > 0 the diagonal
 * shift.  S_pq = sum_x w_x conj(O_xp - Obar_p)(O_xq - Obar_q), Obar = sum_x
 * w_x O_x.  DEVICE output d_dev[n_params].  The solve runs through the
 * 2 n_sr x 2 n_sr Gram matrix of the centred, weighted rows (no n_params^2
 * matrix is formed).  1 <= n_sr <= 256.  Asynchronous; a shifted matrix
 * that is not positive definite in FP64 is reported by eloc_check as
 * ERANGE.  Scratch: about 8 (2 n_params + 520 (2 n_sr + 16)^2) bytes. */
int eloc_sr_solve(eloc_ctx ctx, int n_sr, int64_t n_params, const double* o_re_dev, const double* o_im_dev,
                  const eloc_c64* logpsi_set_dev, const double* grad_dev, double lambda, double* d_dev);

/* Autoregressive sampling without replacement (Methods, "Autoregressive
 * sampling without replacement", Algorithm ARGumbelTopK): the producer of
 * the unique batch U.  The ansatz is the paper's for the modulus (Methods,
 * "Ansatz architecture", "Grouping qubits into qudits", "Global
 * activation", "Local pruning strategy"): qudit k covers qubits
 * [k D, k D + D_k) (D_k = D except for the last, which takes the rest); its
 * conditional distribution given the earlier qubits comes from a
 * perceptron with two hidden layers of width 64,
 *   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2 + h1),  z = W3 h2 + b3,
 * x_q = +1 / -1 for an earlier qubit set / clear and 0 for the others; z
 * (the qudit's log|psi| per outcome c, bit t of c = qubit kD + t) is
 * shifted by its mean, outcomes that can no longer reach n_up electrons on
 * the even qubits and n_down on the odd ones get probability 0 (n_up < 0:
 * no mask), and log p(c | x_<) = 2 z_c - log sum_allowed exp(2 z_c').
 * The search keeps, qudit by qudit, the K prefixes with the largest
 * conditioned perturbed log-probability; the Gumbel variable of a node
 * (qudit, prefix, outcome) is -log(-log u) with u from the top 53 bits of
 * the SplitMix64 output function chained over (seed + 0x9E3779B97F4A7C15
 * (qudit + 1), prefix words, outcome).  Ties go to the earlier (prefix,
 * outcome).  All DEVICE weights row-major: W1 [Q][64][N], b1 [Q][64],
 * W2 [Q][64][64], b2 [Q][64], W3 [Q][2^D][64] (the last qudit uses the first
 * 2^D_last rows), b3 [Q][2^D]. */
typedef struct {
    int n_qubits;        /* N, 1..128 */
    int qudit;           /* D, 1..6 */
    int hidden;          /* must be 64 */
    int n_up, n_down;    /* electron targets on even / odd qubits, or -1 */
    const double* W1;
    const double* b1;
    const double* W2;
    const double* b2;
    const double* W3;
    const double* b3;
} eloc_ar_model;

/* DEVICE outputs keys_dev[k][W] (W = ceil(N / 64)), logp_dev[k] (log p(x)
 * of each sample) and pert_dev[k] or NULL (the conditioned perturbed
 * log-probability), in descending order of the latter; *n_out_host
 * receives the number produced, min(k, number of allowed states).  The
 * keys are unique by construction.  Synchronising (one host read per qudit).
 * Errors: EINVAL (sizes, hidden != 64, 1 <= k < 2^24), ENOMEM, EHIP. */
int eloc_sample(eloc_ctx ctx, const eloc_ar_model* model, int64_t k, uint64_t seed, uint64_t* keys_dev,
                double* logp_dev, double* pert_dev, int64_t* n_out_host);

/* Store the coupled pairs of the current samples, found with `variant`, as
 * a list by row of (column j, H_ij): afterwards eloc_local_energy and
 * eloc_local_energy_adjoint with ELOC_STORED read it instead of finding the
 * pairs again (one pass over about 20 bytes per pair), until the samples or
 * the Hamiltonian change.  *n_pairs_host receives the pair count.  If the
 * list (with the transient emission buffers: 32 bytes per pair, plus 8 per
 * sample) needs more than budget_bytes of device memory, nothing is stored
 * and ECAPACITY is returned: the caller keeps recomputing (any other
 * variant).  Synchronising. */
int eloc_store_pairs(eloc_ctx ctx, int variant, size_t budget_bytes, int64_t* n_pairs_host);

/* Work count of LoopOverTrie (Alg. 2C): the number of (U tree node, XY tree
 * node) pairs its walk visits over all rows of the current samples and all
 * XY chunk trees - the unit of work of this variant, as the candidates
 * |U| |XY| are for LoopOverTerms and |U|^2 for LoopOverBatch.
 * Synchronising. */
int eloc_trie_visits(eloc_ctx ctx, int64_t* visits_host);

/* Launch geometry of the pair kernels (autotuning, benchmarks).  Results do
 * not depend on these settings beyond the floating-point summation order of
 * the chunk partial sums. */
typedef struct {
    int chunks;          /* split of the loop over the unique XY set (TERMS) or
                            over U (BATCH) of every row; 0 = automatic           */
    int sig_filter;      /* 1: exact TERMS prefilters (U's single (even-qubit,
                            total) popcount signature, U's radius around its
                            majority key); 0: off                               */
    int rows_per_wave;   /* rows one wave owns: 4 or 8 (0 = automatic)          */
    int bloom;           /* 1: TERMS probes first test U's Bloom filter, staged
                            in LDS, when U is small enough to have one; 0: off  */
    int waves_per_block; /* waves sharing a workgroup (and its Bloom filter):
                            1 or 4 (0 = automatic)                              */
    int partition;       /* forward / adjoint LoopOverTerms by partitions of U's
                            membership table, each XCD probing its own
                            partitions one after another, so that its L2 holds
                            the partition it works on: 0 = automatic (tables
                            of 8 MB and more), 1 = on (any size), -1 = off.
                            Takes effect at the next eloc_set_hamiltonian /
                            eloc_set_samples.                                 */
    int partition_count; /* partitions: 8, 16 or 32; 0 = automatic (enough to
                            bring one partition to 1 MB)                      */
    int trie_chunk;      /* XY masks per chunk tree of LoopOverTrie (2..32767);
                            0 = automatic (about 2^25 / n_unique chunks, at
                            least 64 masks each).  The trees are built at the
                            first LoopOverTrie use after eloc_set_samples.   */
} eloc_tuning;
int eloc_set_tuning(eloc_ctx ctx, const eloc_tuning* tuning);
int eloc_get_tuning(eloc_ctx ctx, eloc_tuning* tuning);

/* Stage timing with HIP events on the context's stream (the per-part time
 * breakdown of the paper's Fig. 4: sample preparation, FindCoupledPairs +
 * MatrixElement + accumulation, reductions).  While enabled, every call
 * records a start/end event pair around each of its stages. */
enum eloc_stage {
    ELOC_STAGE_SAMPLES = 0,        /* eloc_set_samples: copy, hash table, checks  */
    ELOC_STAGE_AMPLITUDES = 1,     /* exp(L - max Re L) and its inverse           */
    ELOC_STAGE_PAIRS = 2,          /* fused pair kernel (forward)                  */
    ELOC_STAGE_FINISH = 3,         /* chunk sums times 1/psi(x)                    */
    ELOC_STAGE_ENERGY = 4,         /* weighted energy and variance                 */
    ELOC_STAGE_ADJOINT_PAIRS = 5,  /* fused pair kernel (adjoint)                  */
    ELOC_STAGE_ADJOINT_FINISH = 6, /* adjoint row combination                      */
    ELOC_NSTAGES = 7
};
int eloc_profile_enable(eloc_ctx ctx, int on);

/* Totals since the last read: HOST ms_total[ELOC_NSTAGES] (milliseconds)
 * and count[ELOC_NSTAGES] (number of timed launches).  Synchronising;
 * resets the totals. */
int eloc_profile_read(eloc_ctx ctx, double* ms_total, int64_t* count);


/* ===========================================================================
 * Batched evaluation: many problems (H_k, U_k) of uneven size in one
 * pipeline.  Per problem the result is the forward pass above
 * (E_loc^var over U_k and the weighted statistics); the pair stage of all
 * problems is one kernel per key format over the work items (problem, row
 * tile, chunk of the inner loop) of all problems in the schedule's order, and
 * the whole pipeline (sample tables, amplitudes, pairs, row sums,
 * reductions) is captured once per precision into a HIP graph and replayed
 * by eloc_batch_run.  Every problem uses LoopOverTerms or LoopOverBatch as
 * the schedule decides; pairs and phases are those of the single-problem
 * calls, and E_loc equals the single-problem result with the same chunking
 * and rows per wave bit for bit.
 * ======================================================================== */
typedef struct eloc_batch_s* eloc_batch;

/* One problem.  HOST: coeff[n_terms], xy[n_terms][W_k], yz[n_terms][W_k]
 * with W_k = ceil(n_qubits / 64), read during eloc_batch_create only.
 * DEVICE (read / written by every eloc_batch_run, so they must stay valid
 * and keep their sizes while the batch exists): keys_dev[n_unique][W_k]
 * (unique, any order), logpsi_dev[n_unique], weights_dev[n_unique] or
 * NULL (|psi|^2 weights), outputs eloc_dev[n_unique] and stats_dev[4] as
 * in eloc_local_energy. */
typedef struct {
    int n_qubits;
    int64_t n_terms;
    const double* coeff;
    const uint64_t* xy;
    const uint64_t* yz;
    int64_t n_unique;
    const uint64_t* keys_dev;
    const eloc_c64* logpsi_dev;
    const double* weights_dev;
    eloc_c64* eloc_dev;
    double* stats_dev;
} eloc_problem;

/* Schedule of the batched pair kernel. */
typedef struct {
    int rows_per_wave;       /* 4 or 8 rows owned by one wave per work item        */
    int blocks_per_cu;       /* 0: one workgroup per work item; else that many
                                per compute unit (at most what fits), striding
                                over the items                                     */
    int64_t item_candidates; /* target candidates (row x inner index) per item;
                                sets the chunk length of every problem             */
    int order;               /* 0: problems with most candidates first; 1: as given */
    double batch_ratio;      /* LoopOverBatch for problems with n_unique <=
                                batch_ratio * |unique XY|, else LoopOverTerms      */
} eloc_batch_schedule;

/* Ingest n problems (1..256) on `device`, work enqueued on `hip_stream`.
 * Synchronising.  Errors: EINVAL (as eloc_set_hamiltonian / set_samples,
 * with the problem index in the message), ENOMEM, EHIP.  Unless out is NULL
 * or n / probs are invalid, *out receives a handle even on failure, usable
 * for eloc_batch_last_error and eloc_batch_destroy only. */
int eloc_batch_create(eloc_batch* out, int device, void* hip_stream, int n, const eloc_problem* probs);
void eloc_batch_destroy(eloc_batch batch);
const char* eloc_batch_last_error(eloc_batch batch);
int eloc_batch_set_stream(eloc_batch batch, void* hip_stream);

/* Evaluate every problem from the current contents of its DEVICE inputs.
 * Asynchronous; the first call of a precision captures the graph.  Input
 * errors (bits >= N, duplicate keys, bad weights, FP32C range) are
 * reported by eloc_batch_check. */
int eloc_batch_run(eloc_batch batch, int precision);

/* 1: replay the captured graph (default); 0: launch the same kernels one by
 * one on the stream (for comparison). */
int eloc_batch_set_graph(eloc_batch batch, int on);

/* Stage timing of the batched pipeline with HIP events on the batch's
 * stream (for roofline figures): while enabled, every eloc_batch_run with
 * the graph off records events around its three stages - per-sample
 * preparation, the batched pair kernels, row sums and reductions.
 * eloc_batch_profile_read writes HOST ms_total[3] and count[3] (totals since
 * the last read) and resets them; synchronising.  Graph replays are not
 * timed. */
int eloc_batch_profile_enable(eloc_batch batch, int on);
int eloc_batch_profile_read(eloc_batch batch, double* ms_total, int64_t* count);

/* Wait for the stream and report the first problem (*bad_problem, -1 if
 * none) whose last run failed: EINVAL, EDUP, ERANGE as in the
 * single-problem calls, or EAGAIN when its sample table overflowed (it is
 * rebuilt with a new salt by this call; run again).  Synchronising. */
int eloc_batch_check(eloc_batch batch, int* bad_problem);

/* HOST counts_host[n]: coupled ordered pairs of every problem found by the
 * last run.  Synchronising. */
int eloc_batch_pair_counts(eloc_batch batch, int64_t* counts_host);

/* Per-problem view of the schedule: unique XY count, term count, variant
 * used (ELOC_TERMS / ELOC_BATCH) and chunks per row. */
int eloc_batch_problem_info(eloc_batch batch, int k, int64_t* n_groups, int64_t* n_terms, int* variant,
                            int* chunks);

int eloc_batch_get_schedule(eloc_batch batch, eloc_batch_schedule* schedule);
int eloc_batch_set_schedule(eloc_batch batch, const eloc_batch_schedule* schedule);

/* Autotuner: times the pipeline (eager launches, best of two after a warm
 * run) over a coordinate search of the schedule - rows per wave x
 * candidates per item, then the LoopOverBatch ratio, workgroups per CU and
 * problem order - and keeps the fastest.  The inputs must hold valid data.
 * cache_path (HOST string or NULL): a text file of earlier choices keyed
 * by device, precision and problem sizes; a hit skips the timing
 * (*from_cache = 1), a new choice is written to it.  Synchronising. */
int eloc_batch_tune(eloc_batch batch, int precision, const char* cache_path, int* from_cache);

#ifdef __cplusplus
}
#endif

#endif /* ELOC_H */
