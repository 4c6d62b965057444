/*
 * smp.h - C-ABI of the SMP-PCA hot path for AMD Instinct MI355X (gfx950).
 *
 * SMP-PCA (Wu, Bhojanapalli, Sanghavi, Dimakis, "Single Pass PCA of Matrix
 * Products", arXiv 1610.06656) computes a rank-r approximation U V^T of A^T B
 * for A (d x n1) and B (d x n2) while reading A and B only once (Alg. 1):
 *
 *   1. one pass: Gaussian JL sketches A~ = Pi A, B~ = Pi B with Pi(c,l) ~ N(0,1/k),
 *      and the exact column norms ||A_i||, ||B_j||           (Alg. 1 step 2)
 *   2. sample each (i,j) independently with probability q^_ij = min(1, q_ij),
 *      q_ij = m (||A_i||^2/(2 n2 ||A||_F^2) + ||B_j||^2/(2 n1 ||B||_F^2))
 *                                                         (Eq. (1), Alg. 1 step 3)
 *   3. rescaled-JL estimates M~_ij = ||A_i|| ||B_j|| <A~_i,B~_j>/(||A~_i|| ||B~_j||)
 *      on the sampled set Omega only                     (Eq. (2), Alg. 1 step 4)
 *   4. WAltMin: weighted alternating least squares with weights w_ij = 1/q^_ij,
 *      initialised by the top-r SVD of w .* P_Omega(M~) and a row trim
 *                                                  (Alg. 1 step 5; Appendix A, Alg. 2)
 *
 * Conventions for every call below:
 *  - All matrix/vector pointers are DEVICE pointers on the context's device,
 *    allocated and owned by the caller, unless stated otherwise. The library
 *    never frees caller memory.
 *  - All work is enqueued asynchronously on the context's HIP stream, in call
 *    order. Calls that must return a data-dependent size to the host
 *    (smp_sample) synchronise that stream once.
 *  - Layouts: A is d x n1 row-major with leading dimension lda >= n1
 *    (element (l,i) at A[l*lda + i]), the layout of a contiguous (d, n1) torch
 *    tensor; B likewise. Sketches are stored TRANSPOSED, At (n1 x k) row-major
 *    with At[i*k + c] = A~(c,i), so that each column's sketch A~_i is
 *    contiguous. U (n1 x r) and V (n2 x r) are row-major FP64.
 *  - Arguments are validated before anything is launched; on an error the
 *    outputs are untouched and smp_last_error(ctx) describes the problem.
 *    Device faults surface as SMP_ERR_DEVICE.
 *  - A context is used by one host thread at a time.
 *
 * Random streams: every random draw comes from Philox4x32-10 (Salmon et al.,
 * SC'11) keyed by params.seed. Call (col_block, row, tag) uses the counter
 * (col_block, row mod 2^32, tag, row >> 32) and key (seed mod 2^32, seed >> 32),
 * and serves the four columns 4*col_block..4*col_block+3 of `row`.
 *   Pi(c,l) = Z/sqrt(k), Z = Box-Muller lane (c mod 4) of call (c/4, l, tag 1),
 *     lanes (0,1) from words (w0,w1), lanes (2,3) from (w2,w3), with
 *     u = ((a>>8)+1) 2^-24, phi = (b>>8) 2^-24, Z = sqrt(-2 ln u)(cos 2 pi phi, sin 2 pi phi);
 *   coin(i,j) = word (j mod 4) of call (j/4, i, tag 2);
 *   subset(i,j) (SPLIT mode) = (word (j mod 4) of call (j/4, i, tag 3) * (2T+1)) >> 32.
 */
#ifndef SMP_H_
#define SMP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum smp_status {
  SMP_OK = 0,
  SMP_ERR_INVALID_ARG = 1,  /* a size, pointer or parameter is out of range */
  SMP_ERR_OUT_OF_MEMORY = 2,/* a device allocation of library workspace failed */
  SMP_ERR_DEVICE = 3,       /* a HIP runtime call or kernel failed */
  SMP_ERR_NUMERIC = 4,      /* non-finite input or factorisation failure */
  SMP_ERR_CAPACITY = 5,     /* caller buffer too small; the required size is reported */
  SMP_ERR_STATE = 6,        /* call out of order (e.g. push after end) */
  SMP_ERR_BUSY = 7          /* admission refused: the job cannot start now (smp_server_try_submit) */
} smp_status;

typedef enum smp_precision {
  SMP_PREC_FP32 = 0,        /* sketch GEMM operands FP32 (v_mfma_f32_16x16x4_f32) */
  SMP_PREC_BF16 = 1,        /* Pi and data rounded to bfloat16 (nearest even), FP32 accumulate
                               (v_mfma_f32_16x16x32_bf16); the norms use the unrounded data */
  SMP_PREC_FP8 = 2          /* Pi rounded to FP8 E4M3; data to E4M3 with one power-of-two (E8M0)
                               scale per column and block of 32 rows (the smallest with
                               max|x| <= 448 * scale); FP32 accumulate on the block-scaled
                               v_mfma_scale_f32_16x16x128_f8f6f4; norms from the unrounded data.
                               For k > 416 each window of rows is first quantised once into
                               operand fragments (library scratch of at most about 512 MiB for
                               a window's Pi, fragments, scales and norms), then multiplied.
                               Streaming pushes must start on a multiple of 32 rows and hold a
                               multiple of 32 rows unless they end at row d. */
} smp_precision;

typedef enum smp_omega_mode {
  SMP_OMEGA_REUSE = 0,      /* every WAltMin half-step uses all of Omega */
  SMP_OMEGA_SPLIT = 1       /* Alg. 2 step 3: 2T+1 random subsets, one per step */
} smp_omega_mode;

enum {
  SMP_B_IS_A = 1u,              /* flags: B is A (PCA of A^T A, Section 3 Remark 3) */
  SMP_SAMPLE_MULTINOMIAL = 2u,  /* flags: draw Omega row by row (Appendix D) instead of one coin per entry */
  SMP_SKETCH_SRHT = 4u          /* flags: sketch with the subsampled randomized Hadamard transform (FP32 only) */
};

/* The problem statement of Section 2 (A, B, r, k, m, T) plus the seed. */
typedef struct smp_params {
  int64_t d, n1, n2;  /* A is d x n1, B is d x n2 */
  int32_t k;          /* sketch size, Pi is k x d; 1 <= k <= 4096 */
  int32_t r;          /* target rank; 1 <= r <= min(n1, n2, 32) */
  int32_t T;          /* WAltMin iterations; 0 <= T <= 1000 */
  int32_t prec;       /* smp_precision of the sketch GEMM */
  int32_t omega_mode; /* smp_omega_mode */
  uint32_t flags;     /* SMP_B_IS_A | SMP_SAMPLE_MULTINOMIAL | SMP_SKETCH_SRHT */
  double m;           /* sample-count parameter of Eq. (1); > 0 */
  uint64_t seed;      /* Philox key */
  int32_t init_iters; /* subspace iterations of the WAltMin init; 0 = default (2) */
  int32_t reserved;   /* must be 0 */
} smp_params;

typedef struct smp_ctx smp_ctx;

/* Sampled entry set Omega (Alg. 1 step 3) with weights and estimates, as two
 * sorted listings: CSR (by row i, then column j) and CSC (by column j, then
 * row i). All arrays are caller-owned device buffers of the stated lengths;
 * the per-entry arrays hold `cap` elements. smp_sample fills the index and
 * weight arrays and `nnz`; smp_estimate fills mt_csr and mt_csc. sub_csr and
 * sub_csc may be NULL in REUSE mode. */
typedef struct smp_omega {
  int64_t n1, n2;     /* grid size */
  int64_t cap;        /* capacity of every per-entry array */
  int64_t nnz;        /* |Omega|, written by smp_sample (host value) */
  int64_t *row_ptr;   /* n1+1 CSR offsets */
  int32_t *col_idx;   /* cap: CSR column of each entry */
  double *w_csr;      /* cap: w = 1/q^ (Alg. 2 step 2) */
  double *mt_csr;     /* cap: M~ on the entry (Eq. (2)) */
  uint8_t *sub_csr;   /* cap: subset id in [0, 2T] (SPLIT mode) or NULL */
  int64_t *col_ptr;   /* n2+1 CSC offsets */
  int32_t *row_idx;   /* cap: CSC row of each entry */
  double *w_csc;      /* cap */
  double *mt_csc;     /* cap */
  uint8_t *sub_csc;   /* cap or NULL */
} smp_omega;

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a
 * hipStream_t; NULL = the default stream). The context owns its workspace. */
smp_status smp_create(smp_ctx **ctx, int device, void *hip_stream);
void smp_destroy(smp_ctx *ctx);
const char *smp_status_str(smp_status s);
const char *smp_last_error(const smp_ctx *ctx);
smp_status smp_set_stream(smp_ctx *ctx, void *hip_stream);

/* Validate params (the checks listed with smp_params). */
smp_status smp_check_params(const smp_params *p);

/* Device bytes of library workspace that smp_solve needs for `p`, excluding
 * the caller's inputs and outputs. The Omega part uses the expected size
 * m plus a 6-sigma margin. */
smp_status smp_workspace_size(const smp_params *p, size_t *bytes);

/* ---- a1: the sketching matrix Pi (Alg. 1 step 2) ----------------------------
 * Writes rows l0 .. l0+nrows-1 of Pi^T: out[(l-l0)*k + c] = Pi(c, l) (FP32,
 * N(0,1/k), the same values the sketch pass uses). For inspection and tests.
 * The sketch pass never holds all of Pi: the FP32 pass regenerates each
 * block of Pi inside the workgroup that multiplies it; the BF16 and FP8
 * passes draw Pi (already rounded, in the matrix-core operand order) one
 * window of data rows at a time into library scratch of at most 128 MiB
 * (smp_workspace_size does not grow with d through Pi) and multiply that
 * window before drawing the next; the FP8 pass at k > 416 shares its window
 * with the quantised data (512 MiB in all). */
smp_status smp_pi_fill(smp_ctx *ctx, const smp_params *p, int64_t l0, int64_t nrows, float *out);

/* ---- a2+a3: the single pass (Alg. 1 step 2; Section 2 "Step 1") -------------
 * At = (Pi A)^T (n1 x k), Bt = (Pi B)^T (n2 x k), na2[i] = ||A_i||^2 (n1),
 * nb2[j] = ||B_j||^2 (n2), all FP32. With SMP_B_IS_A, B/ldb are ignored and Bt,
 * nb2 receive copies of At, na2 (they may also be NULL). Squared norms use
 * compensated FP32 sums per lane and an FP64 combine. */
smp_status smp_sketch(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                      int64_t ldb, float *At, float *Bt, float *na2, float *nb2);
/* With SMP_SKETCH_SRHT in p->flags (and p->prec == SMP_PREC_FP32) the pass
 * sketches with the subsampled randomized Hadamard transform instead of the
 * Gaussian Pi (Section 4: the Spark implementation's choice):
 * Pi[c,l] = sigma_l (-1)^popcount(rho_c & l) / sqrt(k), with sigma_l = +-1 from
 * bit 0 of the Philox word of (row 0, column l) under tag 7 and rho_c < D (D the
 * smallest power of two >= d) the low log2 D bits of the word of (row 0,
 * column c) under tag 8 (rows of the Hadamard matrix drawn with replacement).
 * Computed by length-512 fast Walsh-Hadamard transforms of row chunks in FP32
 * (O(d n log 512 + d n k / 512) additions, no Gaussian draws); every other
 * call (streaming pushes in any order, sampling, estimates, WAltMin, solve)
 * works unchanged on its sketches. */

/* Streaming form of the same pass: rows may be pushed in any order and any
 * block sizes (each row exactly once). The state holds O(k (n1+n2)) partial
 * sums; rows row0 .. row0+nrows-1 of A are A_rows[0 .. nrows-1] (leading
 * dimension lda). smp_sketch_end writes the same outputs as smp_sketch and
 * frees nothing; smp_sketch_free releases the state. */
typedef struct smp_sketch_state smp_sketch_state;
smp_status smp_sketch_begin(smp_ctx *ctx, const smp_params *p, smp_sketch_state **st);
smp_status smp_sketch_push(smp_ctx *ctx, smp_sketch_state *st, const float *A_rows, int64_t lda,
                           const float *B_rows, int64_t ldb, int64_t row0, int64_t nrows);
smp_status smp_sketch_end(smp_ctx *ctx, smp_sketch_state *st, float *At, float *Bt, float *na2, float *nb2);
void smp_sketch_free(smp_sketch_state *st);

/* ---- entries in any order (Section 1: the entries of A and B may arrive in an
 * arbitrary order, as in streaming logs; Section 3 "Computation Complexity":
 * the sketch costs O(nnz(A) k + nnz(B) k)) ----------------------------------
 * Add the entries (l, i, v) of A (which = SMP_MAT_A) or B (SMP_MAT_B) to a
 * streaming state: A~[:, i] += v Pi[:, l], ||A_i||^2 += v^2, i.e. the state
 * then holds the sketch of the matrix the entries describe (entries not
 * given are zero). Every (l, i) may occur at most once over the whole stream
 * of a matrix; a pair repeated inside one push is rejected, a pair repeated
 * across pushes is the caller's error (its square would enter the norm
 * twice). Entry pushes and dense row pushes (smp_sketch_push) may be mixed,
 * each entry of the matrix given once in all.
 *
 * The result does not depend on the order of the entries in a push: they are
 * grouped by (column, row) with a stable radix sort and every sum runs in a
 * fixed order. Pi is the state's sketching matrix: the Gaussian Pi regenerated
 * from the counter per entry (FP32 products; with SMP_PREC_BF16 both Pi and v
 * rounded to bfloat16, exact products, FP32 sums) or, with SMP_SKETCH_SRHT, the
 * SRHT's +-1/sqrt(k). SMP_PREC_FP8 states refuse entry pushes
 * (SMP_ERR_INVALID_ARG: its scales need whole 32-row blocks of a column).
 *
 * COO: rows[e] (int64, in [0, d)), cols[e] (int32, in [0, n)), vals[e] (FP32),
 * e < nnz, device arrays, any order. CSR: rows row0 .. row0 + nrows - 1 of the
 * matrix (row0 + nrows <= d), row_ptr (nrows + 1 int64, row_ptr[0] = 0,
 * row_ptr[nrows] = nnz, non-decreasing), cols and vals as for COO.
 * 0 <= nnz < 2^31 per push; d * (n + 1) < 2^64.
 *
 * Each push synchronises the stream once, after validating the entries on
 * the device: an index out of range, a repeated pair or an invalid row_ptr
 * gives SMP_ERR_INVALID_ARG and leaves the state as it was. The context holds
 * a device scratch of about 28 B per entry plus 64 B per column plus
 * 4 k B per 256 entries (grown to the largest push; SMP_ERR_OUT_OF_MEMORY if
 * that fails), released by smp_destroy. With SMP_B_IS_A only SMP_MAT_A is
 * accepted. */
enum { SMP_MAT_A = 0, SMP_MAT_B = 1 };
smp_status smp_sketch_push_coo(smp_ctx *ctx, smp_sketch_state *st, int which, const int64_t *rows,
                               const int32_t *cols, const float *vals, int64_t nnz);
smp_status smp_sketch_push_csr(smp_ctx *ctx, smp_sketch_state *st, int which, int64_t row0, int64_t nrows,
                               const int64_t *row_ptr, const int32_t *cols, const float *vals, int64_t nnz);

/* Alg. 1 steps 3-5 (sampling, estimates, WAltMin) from sketches and squared
 * norms already formed, e.g. by smp_sketch_end after streaming or entry
 * pushes: the same outputs and errors as smp_solve, whose remaining stages it
 * runs. At (n1 x k), Bt (n2 x k), na2 (n1), nb2 (n2) as smp_sketch writes
 * them; with SMP_B_IS_A in p->flags, Bt and nb2 may be NULL (At and na2 are
 * used). Synchronises the stream. */
smp_status smp_solve_sketched(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt,
                              const float *na2, const float *nb2, double *U, double *V, double *sigma);

/* ---- a4: sampling (Eq. (1); Alg. 1 step 3; Alg. 2 steps 2-3) ---------------
 * From the FP32 squared norms na2 (n1) and nb2 (n2), draws Omega and writes
 * both listings and the weights into `om` (om->n1, n2, cap and the pointers
 * set by the caller). q^ is evaluated in FP64 in a fixed order (F_A summed
 * sequentially in blocks of 256, then over the blocks; den = (2 n2) F_A;
 * alpha_i = na2_i/den; q = m (alpha_i + beta_j); q^ = min(1,q)); (i,j) is kept
 * iff coin(i,j) < floor(q^ 2^32). Synchronises the stream once. If |Omega| >
 * cap, returns SMP_ERR_CAPACITY with om->nnz = |Omega| and no entries written.
 * If ||A||_F^2 or ||B||_F^2 (the sums of na2, nb2) is not finite - a NaN or
 * Inf in A or B, or a squared norm beyond the FP32 range - returns
 * SMP_ERR_NUMERIC and writes no entries.
 *
 * With SMP_SAMPLE_MULTINOMIAL in p->flags, Omega is drawn row by row instead
 * (Appendix D, "Sampling"): row i makes c_i draws with replacement, c_i the
 * randomised rounding of m_i = m (||A_i||^2/(2||A||_F^2) + 1/(2 n1)), each
 * from q_ij / m_i by binary search over an integer CDF (52-bit fixed-point
 * weights a_i = floor(alpha_i 2^52), b_j = floor(beta_j 2^52) of the same
 * binary64 marginals; CDF_i(j) = (j+1) a_i + b_0 + ... + b_j). An entry drawn
 * N_ij times is listed once with w = N_ij / q_ij, q_ij = m (a_i + b_j) 2^-52.
 * O(n1 + n2 + m log(n1 n2)) work instead of O(n1 n2); the sort of the draws
 * is deterministic, so Omega is the same on every run. |Omega| <= m + n1 + 16. */
smp_status smp_sample(smp_ctx *ctx, const smp_params *p, const float *na2, const float *nb2, smp_omega *om);

/* ---- a3 (rescale) + a5: estimates on Omega (Eq. (2)) -------------------------
 * Fills om->mt_csr and om->mt_csc from the transposed sketches At (n1 x k),
 * Bt (n2 x k) and the squared norms. cos is clamped to [-1,1]; M~ = 0 when any
 * of the four norms is 0. */
smp_status smp_estimate(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt,
                        const float *na2, const float *nb2, smp_omega *om);

/* Allocation-free form of smp_estimate, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, layouts and results (bit for bit),
 * but the FP64 column-norm scratch lives in a file-scope device array of
 * 16 MiB that the library holds on every device it runs on until the process
 * ends; no call allocates or frees anything. Limit: n1 + n2 <= 1,048,576,
 * else SMP_ERR_CAPACITY (nothing launched). All calls on one GPU share that
 * GPU's array: calls that overlap on one GPU (different streams, threads or
 * contexts) race and must be serialised by the caller. */
smp_status smp_estimate_noalloc(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt,
                                const float *na2, const float *nb2, smp_omega *om);

/* ---- comparison methods (Section 1 footnote; Section 4) ----------------------
 * SVD(A~^T B~): the top-r SVD of the product of the sketches At (n1 x k),
 * Bt (n2 x k) written by smp_sketch, without the rescaling of Eq. (2). Block
 * subspace iteration on X = At Bt^T (p = min(r + 10, 64, n1, n2, k) columns,
 * p->init_iters rounds, 0 = 8; Philox-seeded start) and a Rayleigh-Ritz step,
 * all FP64 (the FP32 sketches widened exactly); output in the canonical form
 * of smp_waltmin (orthonormal U, V, sigma descending; sigma NULL folds it into
 * U). Needs r <= k. smp_solve_svd_sketch runs the sketch pass first (the same
 * Pi as smp_solve) and synchronises at its end. */
smp_status smp_svd_sketch(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt, double *U, double *V,
                          double *sigma);
smp_status smp_solve_svd_sketch(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                                int64_t ldb, double *U, double *V, double *sigma);

/* LELA, the two-pass method (Section 4, "Comparison of SMP-PCA and LELA"):
 * smp_column_norms is its first pass (na2[i] = ||A_i||^2, nb2 likewise; FP64
 * partial sums over row blocks added in a fixed order, stored as FP32; with
 * SMP_B_IS_A, B is ignored and nb2 receives a copy or may be NULL);
 * smp_exact_entries its second (om->mt_csr and mt_csc receive the exact
 * (A^T B)_ij on Omega: the plain GEMM A^T B by rocBLAS SGEMM over chunks of
 * 65,536 rows, each chunk's FP32 product added into an FP64 accumulator, then
 * gathered; n1 n2 x 12 bytes of library workspace). smp_lela runs the whole
 * method: norms, the sample of Eq. (1) (p->flags selects the sampler as for
 * smp_sample), exact entries, WAltMin and the canonical form, as smp_solve
 * does after its sketch pass; it synchronises at its end. */
smp_status smp_column_norms(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                            int64_t ldb, float *na2, float *nb2);
smp_status smp_exact_entries(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                             int64_t ldb, smp_omega *om);
smp_status smp_lela(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B, int64_t ldb,
                    double *U, double *V, double *sigma);

/* ---- a6-a8: WAltMin (Appendix A, Alg. 2) and the canonical output -----------
 * Init: top-r left/right singular subspace of R = w .* P_Omega0(M~) by block
 * subspace iteration; rows of U0 with ||U0_i|| > 8 sqrt(r) sqrt(na2_i / F_A)
 * are zeroed (trim). T alternating steps: V_j = argmin sum_i w_ij (q_i^T v - M~_ij)^2
 * with q the rows of U, then the same for U against V. The fixed factor is
 * used as it is; orthonormalising it first would change only the basis of
 * the solution, not U V^T (when the fixed factor has full rank r), so V is
 * orthonormalised once, before the last step; every r x r system
 * is solved by FP64 Cholesky (pivot <= 1e-12 max diag:
 * retry on G + 1e-9 tr(G)/r I; else 0). Output in canonical form
 * U V^T -> U diag(sigma) V^T with U (n1 x r), V (n2 x r) orthonormal and
 * sigma (r, descending; may be NULL, then sigma is folded into U). */
smp_status smp_waltmin(smp_ctx *ctx, const smp_params *p, const smp_omega *om, const float *na2, double *U,
                       double *V, double *sigma);

/* WAltMin for a group of jobs resident at once (batching and serving): job j
 * is exactly smp_waltmin(ctx, &p[j], &om[j], na2[j], U[j], V[j], sigma[j])
 * (sigma may be NULL, or sigma[j] NULL, as there), bit for bit. The jobs'
 * launch sequences are recorded on the host and grouped by sequence (the same
 * r, T, init_iters, omega_mode and block-width class give the same kernels in
 * the same order); each group then runs as one launch per step over all its
 * jobs, each kernel finding its job's arguments in a device table (blockIdx.y
 * = job), and with graph != 0 as one HIP graph per group (captured, launched
 * once and released; the table is copied before the capture, so the graph
 * holds kernel nodes only). The context keeps one workspace for all jobs
 * (their WAltMin workspaces plus the tables). Synchronises the stream. */
smp_status smp_waltmin_group(smp_ctx *ctx, int njobs, const smp_params *p, const smp_omega *om,
                             const float *const *na2, double *const *U, double *const *V, double *const *sigma,
                             int graph);

/* Sketches of a group of independent BF16 jobs in grouped launches (Alg. 1
 * step 2 for every job; batching many jobs at once). Job j computes what
 * smp_sketch(ctx, &p[j], A[j], lda[j], B[j], ldb[j], At[j], Bt[j], na2[j],
 * nb2[j]) computes, with the same meaning of every argument (SMP_B_IS_A in
 * p[j].flags: B[j] ignored, Bt[j] and nb2[j] receive copies or may be NULL),
 * but through the regenerating BF16 pass of its own k: Pi is drawn inside
 * each tile and never stored, and the jobs whose launches use the same
 * kernel run as one launch (blockIdx.y = job, each job's arguments from a
 * device table, each job's work decoded over a grid of its own so that it
 * still spreads over all XCDs), then one launch for all their tails, then
 * each job's reduction. Results are the BF16 sketch as the oracle defines it
 * (the split-K partial sums may be added in another order than smp_sketch's,
 * so the last FP32 bits can differ). Every p[j].prec must be SMP_PREC_BF16
 * (else SMP_ERR_INVALID_ARG); njobs <= 65535. Pointers are device pointers
 * except the arrays themselves and p, which are host arrays of njobs entries
 * each. The context keeps the jobs' partials and the device job table in its
 * workspace. Synchronises the stream once (after copying the job table). */
smp_status smp_sketch_group(smp_ctx *ctx, int njobs, const smp_params *p, const float *const *A,
                            const int64_t *lda, const float *const *B, const int64_t *ldb, float *const *At,
                            float *const *Bt, float *const *na2, float *const *nb2);

/* ---- sketch launch-shape tuning (batching and serving) -------------------------
 * The sketch pass has two free launch parameters: the number of row splits
 * (split-K workgroups per column tile) and, for the BF16 stored-Pi pass, the
 * sketch-row chunk (13 or 16 m-tiles of 16 rows per workgroup). By default a
 * cost model picks them. smp_tune_sketch times every candidate on the first
 * rows of the given A and B that four launches of this shape cover (a launch
 * covers one stored-Pi window, else all d rows; device pointers, layouts as
 * smp_sketch; one warm-up and five timed passes per candidate, each costed per
 * launch, with the reduction of the partials spread over the launches of a
 * whole pass; Gaussian passes only,
 * SMP_ERR_INVALID_ARG for the SRHT) and keeps the fastest in a table shared by every context of the
 * process, keyed by (prec, k, n1, n2 or 0 when SMP_B_IS_A, rows per launch):
 * every later sketch of that shape, in any context, uses it. It writes the
 * choice (cap 0: the plan's own chunk) and its median cost per launch in ms. Running it
 * while other threads sketch the same shape is allowed (they use the table as
 * it stands); it synchronises the stream, and leaves the context's stage
 * timing level as it was (the recorded stages are forgotten).
 * smp_tune_save writes the table as JSON ({"format": "smp-sketch-tuning",
 * "version": 1, "entries": [{"prec", "srht", "k", "n1", "n2", "rows", "cap",
 * "splits", "ms"}, ...]}); smp_tune_load merges such a file into the table
 * (SMP_ERR_INVALID_ARG for anything else, the table unchanged); the first
 * smp_create of a process loads the file named by the environment variable
 * SMP_TUNE_FILE, if set. smp_tune_lookup reports the stored choice for a
 * parameter set (splits 0: none stored); smp_tune_clear empties the table. */
smp_status smp_tune_sketch(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                           int64_t ldb, int32_t *cap, int32_t *splits, double *ms);
smp_status smp_tune_lookup(const smp_params *p, int32_t *cap, int32_t *splits);
smp_status smp_tune_save(const char *path);
smp_status smp_tune_load(const char *path);
void smp_tune_clear(void);

/* ---- stage timing ------------------------------------------------------------
 * With timing enabled, smp_solve (and smp_sketch) record HIP events on the
 * context's stream around each stage; smp_stage_times writes the durations (ms)
 * of the last call (an entry push records [0]: its accumulation kernels,
 * after the sort): [0] sketch kernel, [1] sketch reduction, [2] sampling,
 * [3] estimate, [4] WAltMin (init + iterations + canonical form). Stages that
 * did not run report 0. n is the capacity of ms (up to 5 are written).
 * enable: 0 off, 1 every stage, 2 the sketch stage only (the others report 0);
 * other values are SMP_ERR_INVALID_ARG. Changing the level forgets the stages
 * recorded before. Each timed stage costs one event pair on the stream (about
 * 10 us of idle GPU at each stage boundary); it does not synchronise more. */
smp_status smp_set_timing(smp_ctx *ctx, int enable);
smp_status smp_stage_times(smp_ctx *ctx, float *ms, int n);

/* ---- the whole of Alg. 1 -----------------------------------------------------
 * smp_sketch -> smp_sample -> smp_estimate -> smp_waltmin with library-owned
 * intermediates. Outputs as smp_waltmin. B may equal A (or SMP_B_IS_A).
 * Non-finite input: SMP_ERR_NUMERIC (see smp_sample), U and V untouched. */
smp_status smp_solve(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B, int64_t ldb,
                     double *U, double *V, double *sigma);

/* ---- batching and serving: many independent jobs on one GPU ------------------
 * A server runs jobs (each one smp_solve) on `workers` threads, each with its
 * own context, HIP stream and workspace, so the kernels of different jobs
 * overlap on the device (continuous batching: a job submitted while others
 * run starts as soon as a worker is free and the HBM budget allows). Jobs are
 * admitted in submission order while the device memory in use stays within
 * `hbm_budget` bytes. Memory in use = the workspace every worker's context
 * holds (a worker keeps its buffers between jobs; while it runs a job, at
 * least that job's smp_workspace_size) + the inputs and outputs of the
 * running jobs (d*lda*4 + d*ldb*4 unless B is A, + (n1+n2+1)*r*8). A job
 * larger than the budget runs when nothing else does, and its worker then
 * releases its workspace. 0 means no budget (workers keep their buffers).
 * The caller owns every job's inputs and outputs (device memory of the
 * server's device) and keeps them alive and untouched until the job is
 * waited for. Results are the same as smp_solve of the job alone.
 * smp_server_destroy runs the jobs still queued to completion first. */
typedef struct smp_server smp_server;

typedef struct smp_job_result {
  int32_t status;    /* smp_status of the job's smp_solve */
  int32_t worker;    /* index of the worker that ran it */
  double queue_ms;   /* submission -> start */
  double run_ms;     /* start -> completion (includes the final stream synchronisation) */
} smp_job_result;

typedef struct smp_server_stats {
  int64_t submitted, completed, failed;
  int32_t max_running;        /* most jobs running at once */
  int32_t workers;
  int64_t max_budget_in_use;  /* largest memory in use at an admission (bytes, as defined above) */
  int64_t refused;            /* smp_server_try_submit calls answered SMP_ERR_BUSY */
} smp_server_stats;

/* workers in [1, 16]. Creates the worker threads and their contexts. */
smp_status smp_server_create(int device, int workers, size_t hbm_budget, smp_server **out);
/* Validates p (as smp_check_params) and the pointers, queues the job and
 * returns its id. Does not block on the GPU. */
smp_status smp_server_submit(smp_server *s, const smp_params *p, const float *A, int64_t lda, const float *B,
                             int64_t ldb, double *U, double *V, double *sigma, uint64_t *job_id);
/* Admission without queueing, for callers that would rather retry or route
 * the job elsewhere than wait: queues the job (as smp_server_submit) only if
 * it can start at once - no job waits ahead of it, a worker is free, and
 * either nothing runs or the memory in use with it stays within the budget -
 * else returns SMP_ERR_BUSY and queues nothing (stats.refused counts these).
 * Argument checks as smp_server_submit. */
smp_status smp_server_try_submit(smp_server *s, const smp_params *p, const float *A, int64_t lda, const float *B,
                                 int64_t ldb, double *U, double *V, double *sigma, uint64_t *job_id);
/* Blocks until the job has finished; fills *res (may be NULL) and forgets the
 * job. SMP_ERR_INVALID_ARG for an unknown or already waited id. Each id is
 * waited for once, by one thread (different ids may be waited for from
 * different threads). The job's own status is res->status; its error text,
 * when it failed, is returned by smp_server_last_error until the next wait. */
smp_status smp_server_wait(smp_server *s, uint64_t job_id, smp_job_result *res);
const char *smp_server_last_error(const smp_server *s);
smp_status smp_server_get_stats(smp_server *s, smp_server_stats *st);
void smp_server_destroy(smp_server *s);

/* Runs njobs jobs through a temporary server (workers, hbm_budget as above)
 * and waits for all. Arrays have njobs entries; res may be NULL. Returns
 * SMP_OK when every job succeeded, else the status of the first failed job. */
smp_status smp_solve_batch(int device, int njobs, const smp_params *p, const float *const *A, const int64_t *lda,
                           const float *const *B, const int64_t *ldb, double *const *U, double *const *V,
                           double *const *sigma, int workers, size_t hbm_budget, smp_job_result *res);

/* The same batch in two phases: `workers` threads (1..32), each with its own
 * context and stream, run the sketch pass, the sample and the estimates of
 * one job after another (each job's sample and estimates kept in memory of
 * its own); then WAltMin runs for all jobs at once through smp_waltmin_group
 * (graph != 0: one HIP graph per group of jobs with the same launch
 * sequence). Each job's U, V, sigma are bit for bit those of smp_solve. The
 * batch holds every job's sample until the end (about 40 B per sampled entry
 * plus 4 n1 B per job); res[j].queue_ms is the wait before the job's first
 * phase, run_ms from its start to the end of the grouped phase. Returns
 * SMP_OK when every job succeeded, else the status of the first failed job. */
smp_status smp_solve_batch_group(int device, int njobs, const smp_params *p, const float *const *A,
                                 const int64_t *lda, const float *const *B, const int64_t *ldb, double *const *U,
                                 double *const *V, double *const *sigma, int workers, int graph,
                                 smp_job_result *res);

#ifdef __cplusplus
}
#endif

#endif /* SMP_H_ */
