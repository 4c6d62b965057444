// Host-side internals shared by the C-ABI implementation files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/smp.h"

struct smp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // growable library workspace (device), reused across calls
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // small pinned host buffer for the few readbacks
  int64_t *host_pinned = nullptr;
  // stage timing: events[2*s] / events[2*s+1] bracket stage s; timing is
  // 0 (off), 1 (every stage) or 2 (the sketch stage only)
  int timing = 0;
  hipEvent_t events[10] = {};
  bool recorded[5] = {};
  // rocBLAS handle of the LELA baseline's exact entries (created on first use)
  void *blas = nullptr;
};

namespace smp {

// Device bytes of library workspace a context holds now (its growable
// buffers), and their release (after the context's stream has drained).
size_t ctx_workspace_bytes(const smp_ctx *ctx);
void ctx_release_workspace(smp_ctx *ctx);

// ---- sketch --------------------------------------------------------------------
struct SketchPlan {
  int prec;       // smp_precision of the MFMA operands
  int mt_total;   // ceil(k/16) m-tiles of 16 sketch rows
  int kt;         // WG chunks along k
  int mt;         // m-tiles per chunk
  int nv;         // adjacent columns per lane: a wave covers 16*nv columns
  int waves;      // waves per workgroup, sharing one Pi block
  int kc;         // data rows per Pi block (the streaming chunk)
  int ncol_tile;  // columns per WG = waves * 16 * nv
  int kpad;       // mt_total * 16
  void *kernel;         // the instantiated kernel for this shape
  void *kernel_clamp;   // BF16, FP8: variant for partial blocks (the tail launch), else null
  void *kernel_scalar;  // BF16, FP8: variant with guarded scalar loads (unaligned or ragged inputs), else null
  int pi_stored;        // 1: Pi is drawn window by window into a buffer that the pass streams
  int pi_rows;          // stored Pi: data rows per fragment block (32 BF16, 128 FP8)
  int pi_frag_bytes;    // stored Pi: bytes of one fragment (one MFMA A operand: 1024 BF16, 2048 FP8)
  int vec_elems = 0;    // vector loads: the alignment (elements) of base, leading dimension and column count
                        // they need (0: nv)
  void *kernel_v2 = nullptr;        // vec_elems > nv: the variants with one nv-wide load per row, for
  void *kernel_v2_clamp = nullptr;  // inputs aligned to nv but not to vec_elems
  int frag = 0;         // FP8: the data is first quantised, window by window, into MFMA B-operand fragments
  int64_t ntot = 0;     // frag: n1 + n2 (the columns its fragment windows are sized for)
  int srht = 0;         // 1: the SRHT pass (sketch_srht.hip); mt holds its accumulators per thread
  int64_t d = 0;        // SRHT: rows of A and B (the Hadamard size is the next power of two)
};

// The SRHT pass (Section 4's Spark sketch): plan, splits and one push.
SketchPlan sketch_plan_srht(int k);
int srht_splits(const SketchPlan &pl, int64_t d, int64_t n1, int64_t n2);
hipError_t srht_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                     int64_t n2, int64_t d, int64_t row0, int64_t rows, int k, uint64_t seed, int S, bool accumulate,
                     float *part, double *npart, hipStream_t st);

// Partial-sketch slots a pass with S splits writes: S, plus one for the rows
// the BF16 / FP8 main launch leaves to its tail launch.
inline int sketch_slots_total(const SketchPlan &pl, int S) { return pl.prec == SMP_PREC_FP32 || pl.frag ? S : S + 1; }

// Tile plan for sketch size k and operand precision prec.
SketchPlan sketch_plan(int k, int prec);
SketchPlan sketch_plan_bf16(int k, int cap = 0);   // cap: m-tiles per chunk of the stored-Pi pass (0: default)
SketchPlan sketch_plan_fp8(int k);

// Stored-Pi passes draw Pi one window at a time into a buffer of at most
// kPiWindowBytes (the window: pi_window_rows(pl) data rows, a whole number of
// blocks), so the buffer does not grow with d.
constexpr int64_t kPiWindowBytes = 128ll << 20;
int64_t pi_window_rows(const SketchPlan &pl);

// Bytes of the stored-Pi buffer a push of `rows` rows needs (0 unless
// pl.pi_stored; at most one window), and the kernel that fills it for rows
// [r0, r0 + rows).
size_t sketch_pi_bytes(const SketchPlan &pl, int64_t rows);
hipError_t pi_store(const SketchPlan &pl, uint64_t seed, int64_t r0, int64_t rows, int k, void *buf, hipStream_t st);
hipError_t pi_store_bf16(const SketchPlan &pl, uint64_t seed, int64_t r0, int64_t rows, int k, void *buf,
                         hipStream_t st);
hipError_t pi_store_fp8(const SketchPlan &pl, uint64_t seed, int64_t r0, int64_t rows, int k, void *buf,
                        hipStream_t st);

// FP8 fragment pass (pl.frag): per window of fp8_frag_window_rows(pl) rows the
// Pi fragments, the data quantised into MFMA B operands with their scales
// and squared norms, then the GEMM; fp8_frag_bytes(pl, rows) bytes of scratch
// (at most about kFragWindowBytes, independent of d). Same contract as
// sketch_push; all S slots are written, there is no tail slot.
constexpr int64_t kFragWindowBytes = 512ll << 20;
int64_t fp8_frag_window_rows(const SketchPlan &pl);
size_t fp8_frag_bytes(const SketchPlan &pl, int64_t rows);
hipError_t fp8_frag_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                         int64_t n2, int64_t rows, int k, uint64_t seed, int64_t row0, int S, bool accumulate,
                         float *part, double *npart, void *buf, hipStream_t st);

// Workgroups of the plan's kernel that the device runs at once
// (CUs x resident workgroups per CU).
int sketch_slots(const SketchPlan &pl);


// Pass over rows [row0, row0+rows) of A (and B). part: [S][n1+n2][kpad] FP32,
// npart: [S][n1+n2] FP64. accumulate: add into the partials (zeroed by the
// caller before the first push); otherwise store them (a single push covering
// all rows). pi_buf: sketch_pi_bytes(pl, rows) bytes of scratch (may be null
// when that is 0); the pass draws Pi into it window by window.
hipError_t sketch_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                       int64_t n2, int64_t row0, int64_t rows, int k, uint64_t seed, int S, bool accumulate,
                       float *part, double *npart, void *pi_buf, hipStream_t st);

// Reduce the S partials into At (n1 x k), Bt (n2 x k), na2, nb2 (Bt/nb2 may be null).
hipError_t sketch_finish(const SketchPlan &pl, const float *part, const double *npart, int S, int64_t n1,
                         int64_t n2, int k, float *At, float *Bt, float *na2, float *nb2, hipStream_t st);

hipError_t pi_fill(int64_t l0, int64_t nrows, int k, uint64_t seed, float *out, hipStream_t st);

// Grouped BF16 sketch of many independent jobs (each the whole pass of its own
// d x n1 A and d x n2 B; B null: B = A, n2 is then A's). Every job runs the
// regenerating BF16 pass of its own k (Pi drawn inside each tile, never
// stored); the main launches of all jobs with the same kernel go out as one
// launch, then their tail launches, then each job's finish. scratch holds the
// jobs' split-K partials and the device job table:
// bf16_group_scratch_bytes(jobs, n) bytes.
struct GroupSketchJob {
  const float *A, *B;
  int64_t lda, ldb, n1, n2, d;
  int k;
  uint64_t seed;
  float *At, *Bt, *na2, *nb2;   // Bt and nb2 receive copies of At and na2 when B = A (may be null then)
};
size_t bf16_group_scratch_bytes(const GroupSketchJob *jobs, int njobs);
hipError_t bf16_sketch_group(const GroupSketchJob *jobs, int njobs, void *scratch, size_t scratch_bytes,
                             hipStream_t st);

// ---- sampling ------------------------------------------------------------------
struct SampleWs {
  double *stats;     // [8]: F_A, F_B, den_A, den_B, non-finite flag (1.0 when F_A or F_B is not finite)
  double *alpha;     // n1
  double *beta;      // n2
  double *blocks;    // max(n1, n2)/256 + 1
  int64_t *cnt;      // max(n1, n2) + 1
};
hipError_t sample_prepare(const float *na2, const float *nb2, int64_t n1, int64_t n2, SampleWs &ws,
                          hipStream_t st);
hipError_t sample_count(const SampleWs &ws, int64_t n1, int64_t n2, double m, uint64_t seed, int64_t *row_ptr,
                        int64_t *col_ptr, int64_t *scan_tmp, hipStream_t st);
hipError_t sample_fill(const SampleWs &ws, int64_t n1, int64_t n2, double m, uint64_t seed, int T, int split,
                       const smp_omega &om, hipStream_t st);

// ---- scans and radix sort (sort_scan.hip) --------------------------------------
// Exclusive scans of int64 counts (out[0..n], out[n] = total) and a stable LSD
// radix sort of uint64 keys, 8 bits per pass, with an optional uint32 payload.
struct SortWs {
  int64_t nmax = 0, ntiles = 0;                   // key capacity, radix tiles
  int64_t scan_n = 0;                             // the longest scan the chunk buffers allow
  uint64_t *keys0 = nullptr, *keys1 = nullptr;    // nmax each
  uint32_t *vals0 = nullptr, *vals1 = nullptr;    // nmax each, or null: keys only
  int64_t *hist = nullptr, *hoff = nullptr;       // 256 ntiles, + 1
  int64_t *csum = nullptr, *coff = nullptr;       // scan chunk sums / offsets
};
int64_t radix_tiles(int64_t nmax);
size_t sort_ws_bytes(int64_t nmax, bool payload, int64_t scan_n);
void *sort_ws_carve(void *base, int64_t nmax, bool payload, int64_t scan_n, SortWs &w);   // returns the end
hipError_t scan_exclusive(const SortWs &w, const int64_t *in, int64_t n, int64_t *out, hipStream_t st);
// Sorts (keys0, vals0)[0 .. min(*n_dev, nmax)) by the low `bits` bits of the
// keys. The result is in keys0/vals0 after an even number of 8-bit passes,
// else in keys1/vals1 (radix_result).
hipError_t radix_sort(const SortWs &w, const int64_t *n_dev, int bits, hipStream_t st);
inline const uint64_t *radix_result(const SortWs &w, int bits) { return ((bits + 7) / 8) % 2 ? w.keys1 : w.keys0; }
inline const uint32_t *radix_payload(const SortWs &w, int bits) { return ((bits + 7) / 8) % 2 ? w.vals1 : w.vals0; }

// ---- launch-shape table of the sketch pass (tune.cpp) -------------------------
// rows: the rows one launch covers (one stored-Pi window, else d); n2 = 0
// when B is A; cap 0 keeps the plan's own chunk cap.
struct TuneKey {
  int prec, srht, k;
  int64_t n1, n2, rows;
};
struct TuneChoice {
  int cap, splits;
  double ms;
};
bool tune_lookup(const TuneKey &k, TuneChoice &out);
void tune_store(const TuneKey &k, const TuneChoice &c);
void tune_clear();
size_t tune_count();
std::string tune_save(const char *path);   // "" on success, else the problem
std::string tune_load(const char *path);

// ---- entry-wise sketch (sketch_sparse.hip) ----------------------------------
// One push of triples (l, i, v) of one matrix (COO: rows; CSR: row_ptr over
// rows row0 .. row0 + nrows - 1) into the streaming state's partial slot 0.
struct SparseIn {
  const int64_t *rows = nullptr;      // COO row of each entry, or null
  const int64_t *row_ptr = nullptr;   // CSR offsets (nrows + 1), or null
  int64_t row0 = 0, nrows = 0;
  const int32_t *cols = nullptr;
  const float *vals = nullptr;
  int64_t nnz = 0;
};
// Flags and counts of a push, read back once before anything is added.
struct SpStatus {
  int64_t nnz, nseg, nms, nlong;
  int32_t bad_index, bad_ptr, dup, pad;
};
size_t sparse_ws_bytes(int64_t nnz, int64_t n, int kpad);
bool sparse_key_fits(int64_t d, int64_t n);
// Two phases of a push. prepare: keys, sort, column offsets and segments, then
// one readback into *result (synchronises the stream); nothing is added to
// the state. accumulate (only when prepare set no flag): the segment sketch
// and the long-column reduction into part, npart (slot 0 of this matrix's
// first column), with the same workspace.
hipError_t sparse_prepare(const SketchPlan &pl, const SparseIn &in, int64_t d, int64_t n, void *ws, SpStatus *result,
                          hipStream_t st);
hipError_t sparse_accumulate(const SketchPlan &pl, const SparseIn &in, int64_t d, int64_t n, int k, uint64_t seed,
                             float *part, double *npart, void *ws, const SpStatus &prep, hipStream_t st);

// Row-wise multinomial sampler (Appendix D): device scratch and the two
// passes (count: draws, sort, distinct entries per row -> row_ptr; fill: the
// CSR entries, then the CSC listing).
struct MnWs {
  int64_t dmax = 0;     // bound on the number of draws (buffers' size)
  uint64_t *a = nullptr, *tot = nullptr;          // n1 each
  int64_t *cnt = nullptr, *dcnt = nullptr;        // n1 each
  int64_t *doff = nullptr;                        // n1 + 1
  int64_t *b = nullptr;                           // n2
  int64_t *bptr = nullptr;                        // n2 + 1
  SortWs srt;                                     // dmax draw keys, scans of up to max(n1, n2) counts
};
int64_t mn_draw_bound(int64_t n1, double m);
size_t mn_ws_bytes(int64_t n1, int64_t n2, double m);
void mn_ws_carve(void *base, int64_t n1, int64_t n2, double m, MnWs &w);
hipError_t mn_count(const SampleWs &ws, const MnWs &w, int64_t n1, int64_t n2, double m, uint64_t seed,
                    int64_t *row_ptr, hipStream_t st);
hipError_t mn_fill(const SampleWs &ws, const MnWs &w, int64_t n1, int64_t n2, double m, uint64_t seed, int T,
                   int split, const smp_omega &om, hipStream_t st);

// ---- estimate ------------------------------------------------------------------
// na/nb: sketch-column norms, sa/sb: data-column norms (FP64 scratch, n1 / n2)
hipError_t estimate_run(const float *At, const float *Bt, const float *na2, const float *nb2, int64_t n1,
                        int64_t n2, int k, double *na, double *nb, double *sa, double *sb, const smp_omega &om,
                        hipStream_t st);

// ---- WAltMin -------------------------------------------------------------------
size_t waltmin_ws_bytes(int64_t n1, int64_t n2, int r, int64_t nnz);
// A group of jobs (see waltmin.hip): table_ws holds waltmin_group_table_bytes;
// fa null (or fa[j] null): F_A summed from na2 per job; graph: one HIP graph per
// bucket of jobs with the same launch sequence. Synchronises the stream.
size_t waltmin_group_table_bytes(int njobs, const smp_params *prm, const smp_omega *om);
hipError_t waltmin_group_run(int njobs, const smp_params *prm, const smp_omega *om, const float *const *na2,
                             double *const *Uout, double *const *Vout, double *const *sigma, void *const *wsbase,
                             const double *const *fa, void *table_ws, int graph, hipStream_t st);
hipError_t waltmin_run(const smp_params &p, const smp_omega &om, const float *na2, double *U, double *V,
                       double *sigma, void *ws, hipStream_t st,
                       const double *fa_in);   // F_A on the device, or null to sum it from na2

// ---- comparison methods (Section 4) ----------------------------------------------
// SVD(A~^T B~): top-r SVD of At Bt^T (At n1 x k, Bt n2 x k) by block subspace
// iteration (`iters` rounds) and Rayleigh-Ritz, canonical output.
size_t svd_sketch_ws_bytes(int64_t n1, int64_t n2, int k, int r);
hipError_t svd_sketch_run(const float *At, const float *Bt, int64_t n1, int64_t n2, int k, int r, int iters,
                          uint64_t seed, double *Uout, double *Vout, double *sigma, void *ws, hipStream_t st);
// LELA: column norms (FP64 partials, `part` holds norms_ws_bytes), exact
// entries A_i^T B_j on Omega (rocBLAS SGEMM chunks into an FP64 accumulator).
size_t norms_ws_bytes(int64_t n1, int64_t n2);
hipError_t column_norms(const float *X, int64_t ld, int64_t d, int64_t n, float *out, double *part, hipStream_t st);
size_t exact_entries_ws_bytes(int64_t n1, int64_t n2);
hipError_t exact_entries(void *blas, const float *A, int64_t lda, const float *B, int64_t ldb, int64_t d, int64_t n1,
                         int64_t n2, const smp_omega &om, void *ws, hipStream_t st);
hipError_t blas_create(void **blas);
void blas_destroy(void *blas);

}  // namespace smp
