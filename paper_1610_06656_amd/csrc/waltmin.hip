// WAltMin (Appendix A, Alg. 2) in FP64 on the GPU, plus the canonical output form.
//
// Init (Alg. 2 steps 4-6): the top-r singular subspace of R = w .* P_Omega0(M~)
// by block subspace iteration (Halko, Martinsson, Tropp 2011, Alg. 4.4) on a
// block of p = r + 5 columns: Y <- orth(R^T orth(R Y)), then a Rayleigh-Ritz
// step on R Y gives U0, S0, V0; rows of U0 with ||U0_i|| > 8 sqrt(r) ||A_i||/||A||_F
// are zeroed (the trim of step 6, with the row-norm bound the paper states
// for the trimmed initial iterate in the proof of its initialisation lemma).
//
// Iterations (Alg. 2 steps 7-10): each half-step is one weighted least-squares
// problem per output row, min_v sum_e w_e (q_e^T v - M~_e)^2 over the row's
// sampled entries, with q the rows of the fixed factor. The
// normal equations G = sum w q q^T, h = sum w M~ q are accumulated on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: four sampled entries per instruction,
// operand A = w q^T, operand B = [q | M~]), copied to LDS, and solved there by
// a right-looking Cholesky with the pivot rule: a pivot <= 1e-12 max diag(G)
// fails, the factorisation is retried once on G + 1e-9 trace(G)/r I, and a row
// that still fails or has no samples gets 0. One wave owns one row.
//
// Orthonormalisation is CholeskyQR (Fukaya et al. 2014): Gram X^T X (fixed
// reduction order), LDS Cholesky, X <- X L^-T. A pivot below 1e-13 of the
// largest diagonal entry drops that direction (its column becomes 0). The
// inner subspace iterations take one pass (only the span matters there);
// factors that must be orthonormal (the final V, the last block of the init)
// take two (CholeskyQR2). The fixed factor of a half-step is not
// orthonormalised (see waltmin_run).
// Small symmetric eigenproblems use a parallel cyclic Jacobi method
// (round-robin ordering, one wave).
//
// Canonical output: with V orthonormal, U V^T = P diag(sigma) (V W)^T where
// U^T U = W diag(sigma^2) W^T and P = U W diag(1/sigma); each component's sign
// makes the largest-magnitude entry of its V column positive.
#include <algorithm>
#include <cmath>
#include <vector>

#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {

typedef double v4d __attribute__((ext_vector_type(4)));

hipError_t fixed_total(const float *x, int64_t n, double *blocks, double *out, hipStream_t st);

namespace {

constexpr int kMaxP = 64;       // largest block width handled by the small kernels
constexpr int kInitOversample = 5;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)std::max<int64_t>(1, (a + b - 1) / b); }

// Lane `src`'s value of v, in every lane.
// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2, each of which squares the relative error (a
// shorter dependent chain than a correctly rounded square root and division).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = __builtin_fma(-(x * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
  }
  return y;
}

__device__ __forceinline__ double readlane_f64(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------- launches
// Every kernel below is a device body taking one argument struct, launched
// either for one job (k_one: the struct by value) or for a group of jobs
// (k_group: blockIdx.y picks the job's struct in a device table). The host
// code issues its launches through an Exec: it launches them on a stream, or
// records them (kernel, grid, the job's struct) so that the same sequence,
// recorded for every job of a group, runs as one launch per step with
// grid.x the largest of the jobs' grids (blocks past a job's own grid find
// nothing to do) and grid.y the number of jobs.
template <class A, void (*F)(const A &), int LB, int MINB>
__global__ __launch_bounds__(LB, MINB) void k_one(A a) {
  F(a);
}
template <class A, void (*F)(const A &), int LB, int MINB>
__global__ __launch_bounds__(LB, MINB) void k_group(const A *__restrict__ table) {
  F(table[blockIdx.y]);
}

struct Op {
  const void *id;   // the group kernel: recordings of different jobs must agree step by step
  dim3 grid, block;
  std::vector<char> arg;
  void (*launch)(const void *table, dim3 grid, dim3 block, hipStream_t st);
};

class Exec {
 public:
  explicit Exec(hipStream_t st) : st_(st) {}
  explicit Exec(std::vector<Op> *rec) : rec_(rec) {}
  hipStream_t stream() const { return st_; }
  bool recording() const { return rec_ != nullptr; }
  template <class A, void (*F)(const A &), int LB, int MINB = 1>
  void run(dim3 grid, dim3 block, const A &a) {
    if (!rec_) {
      hipLaunchKernelGGL((k_one<A, F, LB, MINB>), grid, block, 0, st_, a);
      return;
    }
    Op o;
    o.id = reinterpret_cast<const void *>(&k_group<A, F, LB, MINB>);
    o.grid = grid;
    o.block = block;
    o.arg.assign(reinterpret_cast<const char *>(&a), reinterpret_cast<const char *>(&a) + sizeof(A));
    o.launch = [](const void *table, dim3 g, dim3 b, hipStream_t s) {
      hipLaunchKernelGGL((k_group<A, F, LB, MINB>), g, b, 0, s, static_cast<const A *>(table));
    };
    rec_->push_back(std::move(o));
  }

 private:
  hipStream_t st_ = nullptr;
  std::vector<Op> *rec_ = nullptr;
};

// ---------------------------------------------------------------- Gram
// part[b][a*p + c] = sum over the rows of block b of X[i][a] X[i][c], on the
// FP64 matrix cores: wave w of the block takes the row quads w, w + 4, ...
// (four at a time); lane (c, e) = (lane % 16, lane / 16) loads
// X[4 quad + e][16 tt + c], which is both the A and the B fragment of
// v_mfma_f64_16x16x4f64 for the RT x RT tiles of the result. Rows past the
// block and columns past p load a clamped in-range element and are masked to
// zero afterwards (unconditional loads keep several quads in flight). The four
// waves' tiles are summed in LDS in a fixed order (wave 3, then 2, 1, 0).
struct GramArgs {
  const double *X;
  int64_t n;
  int p;
  int64_t rows_per_block;
  double *part;
};
template <int RT>
__device__ __forceinline__ void gram_partial_body(const GramArgs &a_) {
  const double *__restrict__ X = a_.X;
  const int64_t n = a_.n, rows_per_block = a_.rows_per_block;
  const int p = a_.p;
  double *__restrict__ part = a_.part;
  constexpr int D = 16 * RT;
  constexpr int B = 4;
  __shared__ double S[D * D];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int c = lane & 15, e = lane >> 4;
  const int64_t r0 = blockIdx.x * rows_per_block;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_block);
  v4d acc[RT][RT];
#pragma unroll
  for (int ta = 0; ta < RT; ++ta)
#pragma unroll
    for (int tb = 0; tb < RT; ++tb) acc[ta][tb] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t nq = (r1 - r0 + 3) / 4;
  for (int64_t q0 = wave; q0 < nq; q0 += 4 * B) {
    double x[B][RT];
#pragma unroll
    for (int bq = 0; bq < B; ++bq) {
      const int64_t row = r0 + 4 * (q0 + 4 * bq) + e;
      const int64_t rc = row < r1 ? row : r1 - 1;
#pragma unroll
      for (int tt = 0; tt < RT; ++tt) {
        const int col = 16 * tt + c;
        x[bq][tt] = X[rc * p + (col < p ? col : p - 1)];
      }
    }
#pragma unroll
    for (int bq = 0; bq < B; ++bq) {
      const bool live = r0 + 4 * (q0 + 4 * bq) + e < r1;
#pragma unroll
      for (int tt = 0; tt < RT; ++tt) x[bq][tt] = (live && 16 * tt + c < p) ? x[bq][tt] : 0.0;
#pragma unroll
      for (int ta = 0; ta < RT; ++ta)
#pragma unroll
        for (int tb = 0; tb < RT; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[bq][ta], x[bq][tb], acc[ta][tb], 0, 0, 0);
    }
  }
  // register j of lane (c, e) holds entry (16 ta + 4 j + e, 16 tb + c)
  for (int w = 3; w >= 0; --w) {
    if (wave == w) {
#pragma unroll
      for (int ta = 0; ta < RT; ++ta)
#pragma unroll
        for (int tb = 0; tb < RT; ++tb)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            double *q = S + (16 * ta + 4 * j + e) * D + 16 * tb + c;
            *q = w == 3 ? acc[ta][tb][j] : *q + acc[ta][tb][j];
          }
    }
    __syncthreads();
  }
  const int pp = p * p;
  for (int idx = t; idx < pp; idx += 256) part[(int64_t)blockIdx.x * pp + idx] = S[(idx / p) * D + idx % p];
}

// Entry idx of the sum of the nblk Gram partials, in block order; the loads of
// 16 blocks are issued together (the partials were just written by another
// kernel, so each round trip goes to memory).
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nblk, int pp, int idx) {
  double sum = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = part[(int64_t)(b0 + u < nblk ? b0 + u : nblk - 1) * pp + idx];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (b0 + u < nblk) sum += v[u];
  }
  return sum;
}

// ---------------------------------------------------------------- Cholesky -> L^-T
// One workgroup: sums the nblk Gram partials (fixed order) into G, adds
// shift_rel * trace/p to the diagonal when shift_rel > 0, factors G = L L^T
// (right-looking; a pivot <= 1e-13 of the largest diagonal entry drops that
// direction), inverts L by forward substitution (one column per thread) and
// writes M = L^-T, so that X M has orthonormal columns when X^T X = G.
// With D > 0 (p <= D <= 32) the factorisation and the inverse run on one wave
// in registers: lane i holds row i of G (then of L), pivots and entries are
// broadcast with v_readlane, the same operations in the same order; lane t
// then computes column t of L^-1 and writes row t of M.
struct CholArgs {
  const double *part;
  int nblk, p;
  double shift_rel;
  double *M;
};
template <int D>
__device__ __forceinline__ void chol_inv_body(const CholArgs &a_) {
  const double *__restrict__ part = a_.part;
  const int nblk = a_.nblk, p = a_.p;
  const double shift_rel = a_.shift_rel;
  double *__restrict__ M = a_.M;
  __shared__ double L[kMaxP * kMaxP];
  __shared__ double Y[kMaxP * kMaxP];
  __shared__ double dinv[kMaxP];
  const int t = threadIdx.x;
  const int pp = p * p;
  for (int idx = t; idx < pp; idx += 256) L[idx] = sum_partials(part, nblk, pp, idx);
  __syncthreads();
  if constexpr (D > 0) {
    if (t >= 64) return;
    double tr = 0.0, mx = 0.0;
    for (int a = 0; a < p; ++a) {
      tr += L[a * p + a];
      mx = fmax(mx, L[a * p + a]);
    }
    const double shift = shift_rel > 0.0 ? shift_rel * tr / p : 0.0;
    const double tol = 1e-13 * (mx + shift);
    double l[D], dv[D], y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) l[k] = (t < p && k < p) ? L[t * p + k] + (k == t ? shift : 0.0) : 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      dv[j] = 0.0;
      if (j < p) {
        const double piv = readlane_f64(l[j], j);
        const bool ok = piv > tol && mx > 0.0;
        const double d = ok ? sqrt(piv) : 0.0;
        dv[j] = ok ? 1.0 / d : 0.0;
        l[j] = t == j ? d : (t > j ? l[j] * dv[j] : l[j]);
#pragma unroll
        for (int k = j + 1; k < D; ++k)
          if (k < p) l[k] -= l[j] * readlane_f64(l[j], k);   // only k <= t is kept in lane t
      }
    }
    // y = column t of L^-1 (entries above t stay 0)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      y[i] = 0.0;
      if (i < p) {
        double sum = (i == t) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) sum -= readlane_f64(l[k], i) * y[k];
        y[i] = sum * dv[i];
      }
    }
    if (t < p) {
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (a < p) M[t * p + a] = y[a];
    }
    return;
  }
  double tr = 0.0, mx = 0.0;
  for (int a = 0; a < p; ++a) {
    tr += L[a * p + a];
    mx = fmax(mx, L[a * p + a]);
  }
  const double shift = shift_rel > 0.0 ? shift_rel * tr / p : 0.0;
  __syncthreads();
  if (t < p) L[t * p + t] += shift;
  __syncthreads();
  const double tol = 1e-13 * (mx + shift);
  for (int j = 0; j < p; ++j) {
    const double piv = L[j * p + j];
    const bool ok = piv > tol && mx > 0.0;
    const double d = ok ? sqrt(piv) : 0.0;
    __syncthreads();
    if (t == 0) {
      L[j * p + j] = d;
      dinv[j] = ok ? 1.0 / d : 0.0;
    }
    for (int i = j + 1 + t; i < p; i += 256) L[i * p + j] = ok ? L[i * p + j] / d : 0.0;
    __syncthreads();
    const int m = p - j - 1;
    for (int e = t; e < m * m; e += 256) {
      const int i = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= i) L[i * p + c] -= L[i * p + j] * L[c * p + j];
    }
    __syncthreads();
  }
  // Y = L^-1, column t by thread t: Y[i][t] = (delta_it - sum_{t<=k<i} L[i][k] Y[k][t]) / L[i][i]
  if (t < p) {
    for (int i = 0; i < t; ++i) Y[i * p + t] = 0.0;
    for (int i = t; i < p; ++i) {
      double s = (i == t) ? 1.0 : 0.0;
      for (int k = t; k < i; ++k) s -= L[i * p + k] * Y[k * p + t];
      Y[i * p + t] = s * dinv[i];
    }
  }
  __syncthreads();
  // M[b][a] = Y[a][b]
  for (int idx = t; idx < pp; idx += 256) {
    const int b = idx / p, a = idx % p;
    M[idx] = Y[a * p + b];
  }
}

// Two products in one launch: Xo1 = X1 M1 (n1 rows; blocks 0 .. nb1-1) and
// Xo2 = X2 M2 (n2 rows), each n x pin times pin x pout, one wave per row. When
// na2 is given, rows of Xo1 whose norm exceeds 8 sqrt(pout) sqrt(na2_i / FA)
// are set to zero (the trim of Alg. 2 step 6; the squared norm is summed in
// column order).
struct Apply2Args {
  const double *X1;
  int64_t n1;
  const double *M1;
  double *Xo1;
  const float *na2;
  const double *FA;
  const double *X2;
  int64_t n2;
  const double *M2;
  double *Xo2;
  int pin, pout;
  int64_t nb1;
};
__device__ __forceinline__ void apply2_body(const Apply2Args &a_) {
  const double *__restrict__ X1 = a_.X1, *__restrict__ M1 = a_.M1, *__restrict__ FA = a_.FA;
  const double *__restrict__ X2 = a_.X2, *__restrict__ M2 = a_.M2;
  double *__restrict__ Xo1 = a_.Xo1, *__restrict__ Xo2 = a_.Xo2;
  const float *__restrict__ na2 = a_.na2;
  const int64_t n1 = a_.n1, n2 = a_.n2, nb1 = a_.nb1;
  const int pin = a_.pin, pout = a_.pout;
  const int lane = threadIdx.x & 63;
  const bool first = blockIdx.x < nb1;
  const int64_t i = (first ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - nb1) * 4 + (threadIdx.x >> 6);
  if (i >= (first ? n1 : n2)) return;
  const double *row = (first ? X1 : X2) + i * pin;
  const double *M = first ? M1 : M2;
  double s = 0.0;
  if (lane < pout)
    for (int b = 0; b < pin; ++b) s = fma(row[b], M[b * pout + lane], s);
  if (first && na2) {
    double ss = 0.0;
    for (int a = 0; a < pout; ++a) {
      const double v = readlane_f64(s, a);
      ss += v * v;
    }
    const double fa = FA[0];
    const double thr = fa > 0.0 ? 8.0 * sqrt((double)pout) * sqrt((double)na2[i] / fa) : 0.0;
    if (sqrt(ss) > thr) s = 0.0;
  }
  if (lane < pout) (first ? Xo1 : Xo2)[i * pout + lane] = s;
}

// Xout (n x pout) = X (n x pin) * M (pin x pout), row-major. One wave per row,
// lane a computes output column a; every lane reads the whole input row before
// any lane writes, so Xout may alias X when pin == pout.
struct ApplyArgs {
  const double *X;
  int64_t n;
  int pin;
  const double *M;
  int pout;
  double *Xout;
};
__device__ __forceinline__ void apply_body(const ApplyArgs &a_) {
  const double *X = a_.X;   // may alias Xout
  const int64_t n = a_.n;
  const int pin = a_.pin, pout = a_.pout;
  const double *__restrict__ M = a_.M;
  double *Xout = a_.Xout;
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double *row = X + i * pin;
  double s = 0.0;
  if (lane < pout)
    for (int b = 0; b < pin; ++b) s = fma(row[b], M[b * pout + lane], s);
  __builtin_amdgcn_wave_barrier();
  if (lane < pout) Xout[i * pout + lane] = s;
}

// ---------------------------------------------------------------- Jacobi eigen
// G = the sum of the nblk Gram partials (p x p, symmetrised) -> its
// eigenpairs, sorted by descending eigenvalue, and from the top r of them the
// maps Mu, Mv (p x r) and sigma of the Rayleigh-Ritz and canonical steps.
// One workgroup; cyclic Jacobi with the round-robin pairing so the p/2
// rotations of a round are disjoint.
// An off-diagonal entry is negligible when it is at most 1e-15 of the geometric
// mean of its two diagonal entries or 1e-17 of the largest diagonal magnitude;
// negligible entries are not rotated, and the iteration stops at the first
// sweep that finds none left (at most 40 sweeps). A test on the total
// off-diagonal mass alone can stall when the eigenvalues span several decades:
// every rotation leaves rounding errors of eps times the largest eigenvalue in
// entries that only the small diagonal entries would have to outgrow.
__device__ __forceinline__ bool jacobi_negligible(double apq, double app, double aqq, double dmax) {
  const double a = fabs(apq);
  return a * a <= 1e-30 * fabs(app * aqq) || a <= 1e-17 * dmax;   // squared: no sqrt on the rotation's path
}

// Pair k of round rd of the round-robin schedule over m + 1 players (m odd):
// (m, rd) and (rd + k, rd - k) mod m, lower index first.
__device__ __forceinline__ void jacobi_pair(int rd, int k, int m, int &P, int &Q) {
  if (k == 0) {
    P = m;
    Q = rd;
  } else {
    P = rd + k;
    if (P >= m) P -= m;
    Q = rd - k;
    if (Q < 0) Q += m;
  }
  if (P > Q) {
    const int tmp = P;
    P = Q;
    Q = tmp;
  }
}

struct JacobiArgs {
  const double *part;
  int nblk, p, r;
  double *Mu, *Mv, *sigma;
};
template <int NT>
__device__ __forceinline__ void jacobi_eig_body(const JacobiArgs &a_) {
  const double *__restrict__ part = a_.part;
  const int nblk = a_.nblk, p = a_.p, r = a_.r;
  double *__restrict__ Mu = a_.Mu, *__restrict__ Mv = a_.Mv, *__restrict__ sigma = a_.sigma;
  __shared__ double A[kMaxP * kMaxP];
  __shared__ double V[kMaxP * kMaxP];
  __shared__ double cs[kMaxP / 2][2];
  __shared__ double lam[kMaxP];
  __shared__ double red[64];
  __shared__ int any_left;
  const int t = threadIdx.x;
  const int pp = p * p;
  for (int e = t; e < pp; e += NT) V[e] = sum_partials(part, nblk, pp, e);   // G, summed in block order
  __syncthreads();
  for (int e = t; e < pp; e += NT) A[e] = 0.5 * (V[e] + V[(e % p) * p + e / p]);
  __syncthreads();
  for (int e = t; e < pp; e += NT) V[e] = (e / p == e % p) ? 1.0 : 0.0;
  __syncthreads();
  const int pe = (p + 1) & ~1;   // even number of players; index p is a dummy when p is odd
  const int half = pe / 2, m = pe - 1;
  // this thread's (pair, index) tasks of the update phases; half * p <= 2 NT
  // for the sizes each NT is launched for
  int upi[2], ui[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = t + u * NT;
    upi[u] = e < half * p ? e / p : -1;
    ui[u] = e < half * p ? e % p : 0;
  }
  for (int sweep = 0; sweep < 40 && p > 1; ++sweep) {
    double dmax = 0.0;
    for (int a = 0; a < p; ++a) dmax = fmax(dmax, fabs(A[a * p + a]));
    if (t == 0) any_left = 0;
    __syncthreads();
    for (int e = t; e < p * p; e += NT) {
      const int i = e / p, j = e % p;
      if (i < j && !jacobi_negligible(A[e], A[i * p + i], A[j * p + j], dmax)) any_left = 1;
    }
    __syncthreads();
    if (any_left == 0) break;
    for (int rd = 0; rd < m; ++rd) {
      if (t < half) {
        int P, Q;
        jacobi_pair(rd, t, m, P, Q);
        double c = 1.0, s = 0.0;
        if (Q < p) {
          const double apq = A[P * p + Q], app = A[P * p + P], aqq = A[Q * p + Q];
          if (!jacobi_negligible(apq, app, aqq, dmax)) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        cs[t][0] = c;
        cs[t][1] = s;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int pi = upi[u], i = ui[u];
        if (pi >= 0) {
          int P, Q;
          jacobi_pair(rd, pi, m, P, Q);
          if (Q < p) {
            const double c = cs[pi][0], s = cs[pi][1];
            const double aip = A[i * p + P], aiq = A[i * p + Q];
            A[i * p + P] = c * aip - s * aiq;
            A[i * p + Q] = s * aip + c * aiq;
            const double vip = V[i * p + P], viq = V[i * p + Q];
            V[i * p + P] = c * vip - s * viq;
            V[i * p + Q] = s * vip + c * viq;
          }
        }
      }
      __syncthreads();
      // rows: A <- J^T A
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int pi = upi[u], j = ui[u];
        if (pi >= 0) {
          int P, Q;
          jacobi_pair(rd, pi, m, P, Q);
          if (Q < p) {
            const double c = cs[pi][0], s = cs[pi][1];
            const double apj = A[P * p + j], aqj = A[Q * p + j];
            A[P * p + j] = c * apj - s * aqj;
            A[Q * p + j] = s * apj + c * aqj;
          }
        }
      }
      __syncthreads();
    }
  }
  // descending order: eigenvalue a goes to position rank(a) (ties by index)
  if (t < p) {
    const double la = A[t * p + t];
    int rank = 0;
    for (int b = 0; b < p; ++b) {
      const double lb = A[b * p + b];
      rank += (lb > la || (lb == la && b < t)) ? 1 : 0;
    }
    lam[rank] = la;
    red[rank] = (double)t;
  }
  __syncthreads();
  // Rayleigh-Ritz / canonical maps of the top r pairs (eigenvector a is
  // column red[a] of V): Mu = W_r diag(1/sqrt(lam)), Mv = W_r, sigma =
  // sqrt(lam), with components of lam <= 1e-28 lam_max set to 0
  const double lmax = lam[0];
  for (int e = t; e < p * r; e += NT) {
    const int b = e / r, a = e % r;
    const double l = lam[a];
    const bool ok = l > 1e-28 * lmax && l > 0.0;
    const double wv = V[b * p + (int)red[a]];
    Mu[e] = ok ? wv / sqrt(l) : 0.0;
    Mv[e] = wv;
  }
  if (t < r) {
    const double l = lam[t];
    sigma[t] = (l > 1e-28 * lmax && l > 0.0) ? sqrt(l) : 0.0;
  }
}

// The rounds are latency-bound chains (rotation, then the column and row
// updates); more threads shorten the update phases of the larger problems.
void jacobi_eig(Exec &ex, const double *part, int nblk, int p, int r, double *Mu, double *Mv, double *sigma) {
  const JacobiArgs a{part, nblk, p, r, Mu, Mv, sigma};
  if (p <= 10)
    ex.run<JacobiArgs, jacobi_eig_body<64>, 64>(dim3(1), dim3(64), a);
  else if (p <= 32)
    ex.run<JacobiArgs, jacobi_eig_body<256>, 256>(dim3(1), dim3(256), a);
  else
    ex.run<JacobiArgs, jacobi_eig_body<1024>, 1024>(dim3(1), dim3(1024), a);
}

// ---------------------------------------------------------------- sparse products
// Xout[o][a] = sum over the entries e of row o (those of subset sel when sub
// is given) of w_e M~_e Y[idx_e][a]. One workgroup (4 waves) per output row;
// each wave takes every fourth chunk of 64 entries, loads the chunk's metadata
// one entry per lane, and lets groups of G lanes (G >= p) take one entry each
// and load its row of Y, 16 entries in flight per group. The loads are
// unconditional (clamped indices, values masked afterwards) and the wave's
// next chunk's metadata is requested after the first batch of rows, so that
// one memory round trip serves both. Partial sums are combined with shuffles
// within a wave and through LDS across waves.
struct SpmmArgs {
  const int64_t *ptr;
  const int32_t *idx;
  const double *w, *mt;
  const uint8_t *sub;
  int sel;
  const double *Y;
  int p;
  int64_t n_out;
  const double *Mpost;
  double *Xout;
};
template <int G>
__device__ __forceinline__ void spmm_body(const SpmmArgs &a_) {
  const int64_t *__restrict__ ptr = a_.ptr;
  const int32_t *__restrict__ idx = a_.idx;
  const double *__restrict__ w = a_.w, *__restrict__ mt = a_.mt, *__restrict__ Y = a_.Y;
  const double *__restrict__ Mpost = a_.Mpost;
  const uint8_t *__restrict__ sub = a_.sub;
  const int sel = a_.sel, p = a_.p;
  const int64_t n_out = a_.n_out;
  double *__restrict__ Xout = a_.Xout;
  constexpr int NG = 64 / G;
  __shared__ double red[4 * 64];
  __shared__ double xs[64];
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int g = lane / G, a = lane % G;
  const int64_t o = blockIdx.x;
  if (o >= n_out) return;
  const int64_t e0 = ptr[o], e1 = ptr[o + 1];
  const uint8_t *subp = sub ? sub : reinterpret_cast<const uint8_t *>(idx);   // any valid bytes when unused
  constexpr int BATCH = 16;
  double acc = 0.0;
  int64_t eb = e0 + 64 * wave;
  if (eb < e1) {
    int32_t cj;
    double cw, cm;
    uint8_t cs;
    bool cin;
    auto issue_meta = [&](int64_t ebx) {   // requires e1 > e0
      const int64_t me = ebx + lane;
      const int64_t mc = me < e1 ? me : e1 - 1;
      cin = me < e1;
      cj = idx[mc];
      cw = w[mc];
      cm = mt[mc];
      cs = subp[mc];
    };
    issue_meta(eb);
    for (; eb < e1; eb += 256) {
      const bool ok = cin && (!sub || cs == sel);
      const int32_t mj = ok ? cj : 0;
      const double mv = ok ? cw * cm : 0.0;
      // group g takes entries g, g + NG, g + 2 NG, ... of the chunk (G of them)
      for (int u0 = 0; u0 < G; u0 += BATCH) {
        double y[BATCH];
#pragma unroll
        for (int s8 = 0; s8 < BATCH; ++s8) {
          const int j = __shfl(mj, ((u0 + s8) * NG + g) & 63, 64);
          y[s8] = Y[(int64_t)j * p + (a < p ? a : p - 1)];
        }
        if (u0 == 0) issue_meta(eb + 256);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s8 = 0; s8 < BATCH; ++s8) {
          const double v = __shfl(mv, ((u0 + s8) * NG + g) & 63, 64);
          acc = fma(v, (a < p && v != 0.0) ? y[s8] : 0.0, acc);
        }
      }
    }
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  red[wave * 64 + lane] = acc;
  __syncthreads();
  if (wave != 0) return;
  const double x = (g == 0 && a < p) ? ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane] : 0.0;
  if (!Mpost) {
    if (g == 0 && a < p) Xout[o * p + a] = x;
    return;
  }
  // Xout row = (sum of the rows) Mpost: the factor's CholeskyQR map, applied
  // here instead of to the factor before the product (R (Y M) = (R Y) M)
  if (g == 0 && a < p) xs[a] = x;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (g == 0 && a < p) {
    double y = 0.0;
    for (int b = 0; b < p; ++b) y = fma(xs[b], Mpost[b * p + a], y);
    Xout[o * p + a] = y;
  }
}

struct GaussArgs {
  int64_t n;
  int p;
  uint64_t seed;
  double *Y;
};
__device__ __forceinline__ void gaussian_block_body(const GaussArgs &a_) {
  const int64_t n = a_.n;
  const int p = a_.p;
  const uint64_t seed = a_.seed;
  double *__restrict__ Y = a_.Y;
  const int nb4 = (p + 3) / 4;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * nb4; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nb4;
    const int cb = (int)(e - i * nb4);
    const float4 z = normals4(stream_call(seed, kTagInit, (uint64_t)i, (uint32_t)cb));
    const float zz[4] = {z.x, z.y, z.z, z.w};
    for (int u = 0; u < 4; ++u)
      if (cb * 4 + u < p) Y[i * p + cb * 4 + u] = (double)zz[u];
  }
}

// ---------------------------------------------------------------- scale, sign
struct ScaleArgs {
  double *U;
  int64_t n;
  int r;
  const double *s;
};
__device__ __forceinline__ void scale_cols_body(const ScaleArgs &a_) {
  double *__restrict__ U = a_.U;
  const int64_t n = a_.n;
  const int r = a_.r;
  const double *__restrict__ s = a_.s;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * r; e += (int64_t)gridDim.x * blockDim.x)
    U[e] *= s[e % r];
}

// One workgroup per component c: sign of the largest-magnitude entry of V[:, c]
// (first index on ties); flips U[:, c] and V[:, c] when it is negative.
struct SignArgs {
  double *U;
  int64_t n1;
  double *V;
  int64_t n2;
  int r;
};
__device__ __forceinline__ void sign_fix_body(const SignArgs &a_) {
  double *__restrict__ U = a_.U, *__restrict__ V = a_.V;
  const int64_t n1 = a_.n1, n2 = a_.n2;
  const int r = a_.r;
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t j = t; j < n2; j += 256) {
    const double a = fabs(V[j * r + c]);
    if (a > best) { best = a; bidx = j; }
  }
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      if (bv[t + off] > bv[t] || (bv[t + off] == bv[t] && bi[t + off] < bi[t])) {
        bv[t] = bv[t + off];
        bi[t] = bi[t + off];
      }
    }
    __syncthreads();
  }
  const bool flip = V[bi[0] * r + c] < 0.0;
  __syncthreads();
  if (!flip) return;
  for (int64_t j = t; j < n2; j += 256) V[j * r + c] = -V[j * r + c];
  for (int64_t i = t; i < n1; i += 256) U[i * r + c] = -U[i * r + c];
}

// ---------------------------------------------------------------- weighted LS solves
// One workgroup (4 waves) per output row o; RT = ceil((r+1)/16) MFMA tiles per
// side. Each wave takes every fourth chunk of 64 entries: the chunk's metadata
// is loaded one entry per lane, then BATCH groups of four entries have their
// rows of the fixed factor loaded together before their MFMAs (a whole chunk
// at once when RT = 1); the wave's next chunk's metadata is requested right
// after the first batch of rows, so that the two loads overlap. The four waves'
// Gram tiles are summed in LDS and the r x r system is solved there.
// R > 0: the register solve's row count (RT = 1: r = R; RT = 2: r <= R, padded);
// R = 0: any r of the tile width (RT = 3, the solve in LDS).
struct LsArgs {
  const int64_t *ptr;
  const int32_t *idx;
  const double *w, *mt;
  const uint8_t *sub;
  int sel;
  const double *Q;
  int r;
  int64_t n_out;
  double *Xout;
};
template <int RT, int R>
__device__ __forceinline__ void ls_solve_body(const LsArgs &a_) {
  const int64_t *__restrict__ ptr = a_.ptr;
  const int32_t *__restrict__ idx = a_.idx;
  const double *__restrict__ w = a_.w, *__restrict__ mt = a_.mt, *__restrict__ Q = a_.Q;
  const uint8_t *__restrict__ sub = a_.sub;
  const int sel = a_.sel, r = a_.r;
  const int64_t n_out = a_.n_out;
  double *__restrict__ Xout = a_.Xout;
  static_assert(RT != 1 || R > 0, "the one-tile kernel is instantiated per r");
  constexpr int D = RT * 16;
  constexpr int BATCH = RT == 1 ? 16 : (RT == 2 ? 8 : 4);
  __shared__ double Gw[4 * D * D];
  const int64_t o = blockIdx.x;
  if (o >= n_out) return;
  const int t = threadIdx.x;
  const int wave = t >> 6, lt = t & 63;
  const int col = lt & 15, ent = lt >> 4;
  v4d acc[RT][RT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t e0 = ptr[o], e1 = ptr[o + 1];
  // Every load below is unconditional (indices clamped into the row, values
  // masked afterwards): with loads under conditions the compiler cannot count
  // the ones in flight and waits for all of them, which would serialise the
  // metadata prefetch with the rows.
  const uint8_t *subp = sub ? sub : reinterpret_cast<const uint8_t *>(idx);   // any valid bytes when unused
  struct Meta {
    int32_t row;
    double w, m;
    uint8_t sb;
    bool in;
  };
  auto issue_meta = [&](int64_t eb, Meta &x) {   // requires e1 > e0
    const int64_t me = eb + lt;
    const int64_t mc = me < e1 ? me : e1 - 1;
    x.in = me < e1;
    x.row = idx[mc];
    x.w = w[mc];
    x.m = mt[mc];
    x.sb = subp[mc];
  };
  // Rows of the fixed factor for the four-entry groups s0 .. s0 + BATCH - 1:
  // the loads only (raw values); `multiply` masks them and runs the products.
  struct Batch {
    double qv[BATCH][RT];
  };
  auto gather = [&](int s0, int32_t mrow, Batch &bt) {
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int32_t row = __shfl(mrow, (4 * (s0 + q) + ent) & 63, 64);
#pragma unroll
      for (int tt = 0; tt < RT; ++tt) {
        const int a = tt * 16 + col;
        bt.qv[q][tt] = Q[(int64_t)row * r + (a < r ? a : r - 1)];
      }
    }
  };
  auto multiply = [&](int s0, int nsteps, double mw, double mm, const Batch &bt) {
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int src = (4 * (s0 + q) + ent) & 63;
      const double we = __shfl(mw, src, 64);
      const double me_ = __shfl(mm, src, 64);
      const bool live = s0 + q < nsteps && we != 0.0;
      double af[RT], bf[RT];
#pragma unroll
      for (int tt = 0; tt < RT; ++tt) {
        const int a = tt * 16 + col;
        const double x = live ? (a < r ? bt.qv[q][tt] : (a == r ? me_ : 0.0)) : 0.0;
        bf[tt] = x;
        af[tt] = a < r ? we * x : 0.0;
      }
      // G is symmetric: the tiles below the diagonal are never formed (the
      // solve reads the upper triangle); the right-hand side sits in column r
#pragma unroll
      for (int ta = 0; ta < RT; ++ta)
#pragma unroll
        for (int tb = ta; tb < RT; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ta], bf[tb], acc[ta][tb], 0, 0, 0);
    }
  };
  int64_t eb = e0 + 64 * wave;
  if (eb < e1) {
    Meta cur;
    issue_meta(eb, cur);
    for (; eb < e1; eb += 256) {
      const bool ok = cur.in && (!sub || cur.sb == sel);
      const int32_t mrow = ok ? cur.row : 0;
      const double mw = ok ? cur.w : 0.0, mm = ok ? cur.m : 0.0;
      const int nsteps = (int)std::min<int64_t>(16, (e1 - eb + 3) / 4);
      Batch bt;
      gather(0, mrow, bt);
      issue_meta(eb + 256, cur);   // the wave's next chunk, requested after this chunk's first rows
      __builtin_amdgcn_sched_barrier(0);   // all of the batch's loads in flight before the first product
      multiply(0, nsteps, mw, mm, bt);
      for (int s0 = BATCH; s0 < nsteps; s0 += BATCH) {
        gather(s0, mrow, bt);
        __builtin_amdgcn_sched_barrier(0);
        multiply(s0, nsteps, mw, mm, bt);
      }
    }
  }
  // v_mfma_f64_16x16x4f64 leaves D[4*j + t/16][t%16] in register j of lane t
  double *Gme = Gw + wave * D * D;
#pragma unroll
  for (int ta = 0; ta < RT; ++ta)
#pragma unroll
    for (int tb = ta; tb < RT; ++tb)
#pragma unroll
      for (int j = 0; j < 4; ++j) Gme[(ta * 16 + 4 * j + ent) * D + tb * 16 + col] = acc[ta][tb][j];
  __syncthreads();
  for (int e = t; e < D * D; e += 256) Gw[e] = ((Gw[e] + Gw[D * D + e]) + Gw[2 * D * D + e]) + Gw[3 * D * D + e];
  __syncthreads();
  const double *G = Gw;
  // The r x r solve is serial in r: one wave runs it, ordering its LDS
  // accesses with wavefront-scope fences instead of workgroup barriers.
  if (wave != 0) return;
  auto wsync = [] { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); };

  double mx = 0.0, tr = 0.0;
  for (int a = 0; a < r; ++a) {
    mx = fmax(mx, G[a * D + a]);
    tr += G[a * D + a];
  }
  if constexpr (RT <= 2) {
    // r <= 31: the same steps with row i of the system in the registers of
    // lane i (pivots and solution entries broadcast with v_readlane); the
    // back substitution reads the columns of L through LDS once. Each pivot's
    // reciprocal is taken once and multiplied (one division per column). The
    // kernel is instantiated for R rows (every bound below is a compile-time
    // constant): R = r for r <= 15; for 16 <= r <= 31, R is r rounded up to a
    // multiple of 4 and the system is padded to R rows with an identity block
    // (diagonal max(G) so that its pivots pass the test; zero right-hand
    // side), which leaves rows < r as they are.
    constexpr int RR = R > 0 ? R : D;
    double l[RR];
    bool solved = false;
    double x = 0.0;
    for (int attempt = 0; attempt < 2 && mx > 0.0 && !solved; ++attempt) {
      const double shift = attempt == 0 ? 0.0 : 1e-9 * tr / r;
      const double tol = 1e-12 * (mx + shift);
      const double pad = mx + shift;
#pragma unroll
      for (int k = 0; k < RR; ++k)
        l[k] = (t < r && k < r) ? G[(t < k ? t : k) * D + (t < k ? k : t)] + (k == t ? shift : 0.0)
                                : (t == k && t < RR ? pad : 0.0);
      double y = t < r ? G[t * D + r] : 0.0;
      double dv = 0.0;   // lane j: the reciprocal of pivot j
      bool ok = true;
#pragma unroll
      for (int j = 0; j < RR; ++j) {
        if (ok) {
          const double piv = readlane_f64(l[j], j);
          if (!(piv > tol)) {
            ok = false;
          } else {
            const double dj = rsqrt_nr(piv);
            const double d = piv * dj;
            dv = t == j ? dj : dv;
            l[j] = t == j ? d : (t > j ? l[j] * dj : l[j]);
#pragma unroll
            for (int k = j + 1; k < RR; ++k) l[k] -= l[j] * readlane_f64(l[j], k);   // only k <= t is kept in lane t
          }
        }
      }
      if (!ok) continue;
      // forward: L y = h
#pragma unroll
      for (int k = 0; k < RR; ++k) {
        const double yk = readlane_f64(y, k) * readlane_f64(dv, k);
        y = t == k ? yk : (t > k ? y - l[k] * yk : y);
      }
      // backward: L^T x = y; lane t reads column t of L from LDS (the second
      // wave's Gram area, free once the four partial Grams are summed)
      double *Lr = Gw + D * D;
#pragma unroll
      for (int k = 0; k < RR; ++k)
        if (t < RR && k <= t) Lr[t * RR + k] = l[k];
      wsync();
#pragma unroll
      for (int k = RR - 1; k >= 0; --k) {
        const double xk = readlane_f64(y, k) * readlane_f64(dv, k);
        y = t == k ? xk : (t < k ? y - Lr[k * RR + (t < k ? t : 0)] * xk : y);
      }
      x = y;
      solved = true;
    }
    if (t < r) Xout[o * r + t] = solved ? x : 0.0;
  } else {
  // r = 32: the same steps on the system in LDS
  __shared__ double L[32 * 32];
  __shared__ double hv[32];
  bool solved = false;
  for (int attempt = 0; attempt < 2 && mx > 0.0 && !solved; ++attempt) {
    const double shift = attempt == 0 ? 0.0 : 1e-9 * tr / r;
    const double tol = 1e-12 * (mx + shift);
    for (int e = t; e < r * r; e += 64) {   // G from its upper triangle (the tiles formed)
      const int i = e / r, c = e % r;
      L[i * 32 + c] = G[(i < c ? i : c) * D + (i < c ? c : i)] + ((i == c) ? shift : 0.0);
    }
    if (t < r) hv[t] = G[t * D + r];
    wsync();
    bool ok = true;
    for (int j = 0; j < r; ++j) {
      const double piv = L[j * 32 + j];
      if (!(piv > tol)) { ok = false; break; }
      const double d = sqrt(piv);
      wsync();
      if (t == 0) L[j * 32 + j] = d;
      for (int i = j + 1 + t; i < r; i += 64) L[i * 32 + j] /= d;
      wsync();
      const int m = r - j - 1;
      for (int e = t; e < m * m; e += 64) {
        const int i = j + 1 + e / m, c = j + 1 + e % m;
        if (c <= i) L[i * 32 + c] -= L[i * 32 + j] * L[c * 32 + j];
      }
      wsync();
    }
    if (!ok) {
      wsync();
      continue;
    }
    // forward: L y = h (column-oriented, updates in index order)
    for (int i = 0; i < r; ++i) {
      wsync();
      const double yi = hv[i] / L[i * 32 + i];
      wsync();
      if (t == 0) hv[i] = yi;
      for (int k = i + 1 + t; k < r; k += 64) hv[k] -= L[k * 32 + i] * yi;
    }
    // backward: L^T x = y
    for (int i = r - 1; i >= 0; --i) {
      wsync();
      const double xi = hv[i] / L[i * 32 + i];
      wsync();
      if (t == 0) hv[i] = xi;
      for (int k = t; k < i; k += 64) hv[k] -= L[i * 32 + k] * xi;
    }
    wsync();
    solved = true;
  }
  if (t < r) Xout[o * r + t] = solved ? hv[t] : 0.0;
  }
}

// ---------------------------------------------------------------- host helpers
struct Ws {
  double *FA;       // [1]
  double *blocks;   // n1/256 + 1
  double *X, *Y;     // n1*p, n2*p
  double *part;     // gram partials
  double *M, *Mu, *Mv, *sig;
  double *U, *V;    // n1*r, n2*r iterates
};

// ---- the dense low-rank operator X = S1 S2^T of the SVD(A~^T B~) baseline -----
// S (n x k, FP32, row-major) times a block: the sketches enter as they are
// (widened exactly to FP64), the products are FP64.

// part[b][c][j] = sum over the rows i of block b of S[i][c] Y[i][j]. Thread
// (c mod 64, j group g) keeps the columns j = g, g + 4, ... of one c.
template <int JPT>
__global__ __launch_bounds__(256) void tmul_partial_kernel(const float *__restrict__ S, int64_t n, int k,
                                                           const double *__restrict__ Y, int p, int64_t rpb,
                                                           double *__restrict__ part) {
  const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const int64_t i0 = (int64_t)blockIdx.y * rpb, i1 = i0 + rpb < n ? i0 + rpb : n;
  double acc[JPT];
#pragma unroll
  for (int u = 0; u < JPT; ++u) acc[u] = 0.0;
  const int cc = c < k ? c : k - 1;
  for (int64_t i = i0; i < i1; ++i) {
    const double sv = c < k ? (double)S[i * k + cc] : 0.0;
    const double *y = Y + i * p;
#pragma unroll
    for (int u = 0; u < JPT; ++u) {
      const int j = g + 4 * u;
      acc[u] = fma(sv, y[j < p ? j : p - 1], acc[u]);
    }
  }
  if (c < k) {
#pragma unroll
    for (int u = 0; u < JPT; ++u) {
      const int j = g + 4 * u;
      if (j < p) part[((int64_t)blockIdx.y * k + c) * p + j] = acc[u];
    }
  }
}

// T[c][j] = sum of the partials in block order.
__global__ void tmul_reduce_kernel(const double *__restrict__ part, int nblk, int64_t kp, double *__restrict__ T) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < kp; x += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * kp + x];
    T[x] = s;
  }
}

// X[i][j] = sum_c S[i][c] T[c][j]: one wave per row, lane j; four
// accumulators over c mod 4, added in a fixed order.
__global__ __launch_bounds__(256) void smul_kernel(const float *__restrict__ S, int64_t n, int k,
                                                   const double *__restrict__ T, int p, double *__restrict__ X) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const float *row = S + i * k;
  const int j = lane < p ? lane : p - 1;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int c = 0;
  for (; c + 4 <= k; c += 4) {
    a0 = fma((double)row[c], T[(int64_t)c * p + j], a0);
    a1 = fma((double)row[c + 1], T[(int64_t)(c + 1) * p + j], a1);
    a2 = fma((double)row[c + 2], T[(int64_t)(c + 2) * p + j], a2);
    a3 = fma((double)row[c + 3], T[(int64_t)(c + 3) * p + j], a3);
  }
  for (; c < k; ++c) a0 = fma((double)row[c], T[(int64_t)c * p + j], a0);
  if (lane < p) X[i * p + lane] = (a0 + a1) + (a2 + a3);
}

constexpr int kGramBlocks = 64;

template <typename T>
T *carve(char *&p, size_t count) {
  T *out = reinterpret_cast<T *>(p);
  p += (count * sizeof(T) + 255) / 256 * 256;
  return out;
}

Ws carve_ws(void *base, int64_t n1, int64_t n2, int p, int r) {
  char *c = static_cast<char *>(base);
  Ws w;
  w.FA = carve<double>(c, 4);
  w.blocks = carve<double>(c, n1 / 256 + 2);
  w.X = carve<double>(c, n1 * p);
  w.Y = carve<double>(c, n2 * p);
  w.part = carve<double>(c, (size_t)kGramBlocks * kMaxP * kMaxP);
  w.M = carve<double>(c, kMaxP * kMaxP);
  w.Mu = carve<double>(c, kMaxP * kMaxP);
  w.Mv = carve<double>(c, kMaxP * kMaxP);
  w.sig = carve<double>(c, kMaxP);
  w.U = carve<double>(c, n1 * r);
  w.V = carve<double>(c, n2 * r);
  return w;
}

size_t carve_bytes(int64_t n1, int64_t n2, int p, int r) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t s = 0;
  s += al(4 * 8) + al((n1 / 256 + 2) * 8) + al(n1 * p * 8) + al(n2 * p * 8);
  s += al((size_t)kGramBlocks * kMaxP * kMaxP * 8) + al(kMaxP * kMaxP * 8);
  s += 2 * al(kMaxP * kMaxP * 8) + al(kMaxP * 8) + al(n1 * r * 8) + al(n2 * r * 8);
  return s;
}

int gram(Exec &ex, const Ws &w, const double *X, int64_t n, int p) {
  const int nblk = (int)std::min<int64_t>(kGramBlocks, std::max<int64_t>(1, (n + 127) / 128));
  const int64_t rpb = (n + nblk - 1) / nblk;
  const dim3 grid((unsigned)nblk), blk(256);
  const GramArgs a{X, n, p, rpb, w.part};
  if (p <= 16)
    ex.run<GramArgs, gram_partial_body<1>, 256>(grid, blk, a);
  else if (p <= 32)
    ex.run<GramArgs, gram_partial_body<2>, 256>(grid, blk, a);
  else if (p <= 48)
    ex.run<GramArgs, gram_partial_body<3>, 256>(grid, blk, a);
  else
    ex.run<GramArgs, gram_partial_body<4>, 256>(grid, blk, a);
  return nblk;
}

void apply2(Exec &ex, const double *X1, int64_t n1, const double *M1, double *Xo1, const float *na2, const double *FA,
            const double *X2, int64_t n2, const double *M2, double *Xo2, int pin, int pout) {
  const int64_t nb1 = cdiv(n1, 4), nb2 = cdiv(n2, 4);
  ex.run<Apply2Args, apply2_body, 256>(dim3((unsigned)(nb1 + nb2)), dim3(256),
                                       Apply2Args{X1, n1, M1, Xo1, na2, FA, X2, n2, M2, Xo2, pin, pout, nb1});
}

void apply(Exec &ex, const double *X, int64_t n, int pin, const double *M, int pout, double *Xout) {
  ex.run<ApplyArgs, apply_body, 256>(dim3(cdiv(n, 4)), dim3(256), ApplyArgs{X, n, pin, M, pout, Xout});
}

void chol_inv(Exec &ex, const Ws &w, int nblk, int p, double shift_rel) {
  const CholArgs a{w.part, nblk, p, shift_rel, w.M};
  if (p <= 16)
    ex.run<CholArgs, chol_inv_body<16>, 256>(dim3(1), dim3(256), a);
  else if (p <= 32)
    ex.run<CholArgs, chol_inv_body<32>, 256>(dim3(1), dim3(256), a);
  else
    ex.run<CholArgs, chol_inv_body<0>, 256>(dim3(1), dim3(256), a);
}

// X (n x p) <- X L^-T for X^T X (+ a tiny shift) = L L^T: one CholeskyQR pass,
// span preserved; twice gives orthonormal columns to working precision.
void cholqr_pass(Exec &ex, const Ws &w, const double *X, int64_t n, int p, double shift_rel, double *Xout) {
  chol_inv(ex, w, gram(ex, w, X, n, p), p, shift_rel);
  apply(ex, X, n, p, w.M, p, Xout);
}

// X (n x p) <- orthonormal basis of its span (CholeskyQR2, in place).
void orth(Exec &ex, const Ws &w, double *X, int64_t n, int p) {
  cholqr_pass(ex, w, X, n, p, 1e-14, X);
  cholqr_pass(ex, w, X, n, p, 0.0, X);
}

// The map of one shifted CholeskyQR pass (X^T X + shift = L L^T, w.M = L^-T),
// without applying it: the next sparse product multiplies its output by w.M
// (span kept; X w.M has orthonormal columns up to O(eps cond(X)^2), enough to
// condition the next product).
void orth1_map(Exec &ex, const Ws &w, const double *X, int64_t n, int p) {
  chol_inv(ex, w, gram(ex, w, X, n, p), p, 1e-14);
}

// Xout = R Y (CSR side) or R^T Y (CSC side), times Mpost (p x p) when given.
void spmm(Exec &ex, const int64_t *ptr, const int32_t *idx, const double *wt, const double *mt, const uint8_t *sub,
          int sel, const double *Y, int p, int64_t n_out, const double *Mpost, double *Xout) {
  const dim3 grid((unsigned)std::max<int64_t>(1, n_out)), blk(256);
  const SpmmArgs a{ptr, idx, wt, mt, sub, sel, Y, p, n_out, Mpost, Xout};
  if (p <= 16)
    ex.run<SpmmArgs, spmm_body<16>, 256>(grid, blk, a);
  else if (p <= 32)
    ex.run<SpmmArgs, spmm_body<32>, 256>(grid, blk, a);
  else
    ex.run<SpmmArgs, spmm_body<64>, 256>(grid, blk, a);
}

template <int R>
void ls_solve_r(Exec &ex, const LsArgs &a) {
  ex.run<LsArgs, ls_solve_body<1, R>, 256, 5>(dim3((unsigned)std::max<int64_t>(1, a.n_out)), dim3(256), a);
}

typedef void (*LsLaunch)(Exec &, const LsArgs &);
const LsLaunch kLsByR[16] = {nullptr,       ls_solve_r<1>,  ls_solve_r<2>,  ls_solve_r<3>,  ls_solve_r<4>,
                             ls_solve_r<5>,  ls_solve_r<6>,  ls_solve_r<7>,  ls_solve_r<8>,  ls_solve_r<9>,
                             ls_solve_r<10>, ls_solve_r<11>, ls_solve_r<12>, ls_solve_r<13>, ls_solve_r<14>,
                             ls_solve_r<15>};

void ls_solve(Exec &ex, const int64_t *ptr, const int32_t *idx, const double *wt, const double *mt,
              const uint8_t *sub, int sel, const double *Q, int r, int64_t n_out, double *Xout) {
  const int rt = (r + 1 + 15) / 16;
  const dim3 grid((unsigned)std::max<int64_t>(1, n_out));
  const LsArgs a{ptr, idx, wt, mt, sub, sel, Q, r, n_out, Xout};
  if (rt == 1)
    kLsByR[r](ex, a);
  else if (rt == 2) {   // the register solve padded to the next multiple of 4 rows
    if (r <= 20)
      ex.run<LsArgs, ls_solve_body<2, 20>, 256, 4>(grid, dim3(256), a);
    else if (r <= 24)
      ex.run<LsArgs, ls_solve_body<2, 24>, 256, 4>(grid, dim3(256), a);
    else if (r <= 28)
      ex.run<LsArgs, ls_solve_body<2, 28>, 256, 4>(grid, dim3(256), a);
    else
      ex.run<LsArgs, ls_solve_body<2, 32>, 256, 4>(grid, dim3(256), a);
  } else
    ex.run<LsArgs, ls_solve_body<3, 0>, 256, 1>(grid, dim3(256), a);
}

void gaussian_block(Exec &ex, int64_t n, int p, uint64_t seed, double *Y) {
  ex.run<GaussArgs, gaussian_block_body, 256>(dim3(cdiv(n * ((p + 3) / 4), 256)), dim3(256), GaussArgs{n, p, seed, Y});
}

void scale_cols(Exec &ex, double *U, int64_t n, int r, const double *s) {
  ex.run<ScaleArgs, scale_cols_body, 256>(dim3(cdiv(n * r, 256)), dim3(256), ScaleArgs{U, n, r, s});
}

// U (n1 x r), V (n2 x r, orthonormal columns) -> canonical Uc, sigma, Vc
// (U V^T = Uc diag(sigma) Vc^T). Uc written to Uout, Vc to Vout.
void canonical(Exec &ex, const Ws &w, const double *U, int64_t n1, const double *V, int64_t n2, int r, double *Uout,
               double *Vout, double *sigma) {
  jacobi_eig(ex, w.part, gram(ex, w, U, n1, r), r, r, w.Mu, w.Mv, sigma);
  apply2(ex, U, n1, w.Mu, Uout, nullptr, nullptr, V, n2, w.Mv, Vout, r, r);
  ex.run<SignArgs, sign_fix_body, 256>(dim3(r), dim3(256), SignArgs{Uout, n1, Vout, n2, r});
}

}  // namespace

// ---- SVD(A~^T B~): the top-r SVD of the product of the sketches ---------------
constexpr int kSvdOversample = 10;
constexpr int kTmulBlocks = 32;

static int svd_p(int64_t n1, int64_t n2, int k, int r) {
  const int64_t lim = std::min<int64_t>(std::min(n1, n2), k);
  return std::max(r, std::min<int>(kMaxP, (int)std::min<int64_t>(lim, r + kSvdOversample)));
}

size_t svd_sketch_ws_bytes(int64_t n1, int64_t n2, int k, int r) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const int p = svd_p(n1, n2, k, r);
  return carve_bytes(n1, n2, p, r) + al((size_t)k * p * 8) + al((size_t)kTmulBlocks * k * p * 8);
}

// out (n_out x p) = S_out (S_in^T Y) with S_in n_in x k, S_out n_out x k.
static void lowrank_apply(const float *S_in, int64_t n_in, const float *S_out, int64_t n_out, int k, const double *Y,
                          int p, double *T, double *tpart, double *out, hipStream_t st) {
  const int nblk = (int)std::min<int64_t>(kTmulBlocks, std::max<int64_t>(1, (n_in + 255) / 256));
  const int64_t rpb = (n_in + nblk - 1) / nblk;
  const dim3 grid((unsigned)((k + 63) / 64), (unsigned)nblk);
  if (p <= 16)
    hipLaunchKernelGGL(tmul_partial_kernel<4>, grid, dim3(256), 0, st, S_in, n_in, k, Y, p, rpb, tpart);
  else if (p <= 32)
    hipLaunchKernelGGL(tmul_partial_kernel<8>, grid, dim3(256), 0, st, S_in, n_in, k, Y, p, rpb, tpart);
  else
    hipLaunchKernelGGL(tmul_partial_kernel<16>, grid, dim3(256), 0, st, S_in, n_in, k, Y, p, rpb, tpart);
  hipLaunchKernelGGL(tmul_reduce_kernel, dim3(cdiv((int64_t)k * p, 256)), dim3(256), 0, st, tpart, nblk,
                     (int64_t)k * p, T);
  hipLaunchKernelGGL(smul_kernel, dim3(cdiv(n_out, 4)), dim3(256), 0, st, S_out, n_out, k, T, p, out);
}

hipError_t svd_sketch_run(const float *At, const float *Bt, int64_t n1, int64_t n2, int k, int r, int iters,
                          uint64_t seed, double *Uout, double *Vout, double *sigma, void *wsbase, hipStream_t st) {
  const int p = svd_p(n1, n2, k, r);
  Ws w = carve_ws(wsbase, n1, n2, p, r);
  char *c = static_cast<char *>(wsbase) + carve_bytes(n1, n2, p, r);
  double *T = reinterpret_cast<double *>(c);
  double *tpart = reinterpret_cast<double *>(c + ((size_t)k * p * 8 + 255) / 256 * 256);
  Exec ex(st);
  // block subspace iteration on X = At Bt^T (n1 x n2) from a Philox-seeded start
  gaussian_block(ex, n2, p, seed, w.Y);
  orth(ex, w, w.Y, n2, p);
  for (int it = 0; it < iters; ++it) {
    lowrank_apply(Bt, n2, At, n1, k, w.Y, p, T, tpart, w.X, st);   // X = At (Bt^T Y)
    orth(ex, w, w.X, n1, p);
    lowrank_apply(At, n1, Bt, n2, k, w.X, p, T, tpart, w.Y, st);   // Y = Bt (At^T X)
    orth(ex, w, w.Y, n2, p);
  }
  lowrank_apply(Bt, n2, At, n1, k, w.Y, p, T, tpart, w.X, st);
  // Rayleigh-Ritz: X^T X = W diag(lam) W^T; U = X W_r lam^-1/2, V = Y W_r, sigma = lam^1/2
  jacobi_eig(ex, w.part, gram(ex, w, w.X, n1, p), p, r, w.Mu, w.Mv, w.sig);
  apply2(ex, w.X, n1, w.Mu, w.U, nullptr, nullptr, w.Y, n2, w.Mv, w.V, p, r);
  scale_cols(ex, w.U, n1, r, w.sig);
  double *sig_out = sigma ? sigma : w.sig;
  canonical(ex, w, w.U, n1, w.V, n2, r, Uout, Vout, sig_out);
  if (!sigma) scale_cols(ex, Uout, n1, r, sig_out);
  return hipGetLastError();
}

size_t waltmin_ws_bytes(int64_t n1, int64_t n2, int r, int64_t /*nnz*/) {
  const int p = std::min<int>(kMaxP, (int)std::min<int64_t>(std::min(n1, n2), r + kInitOversample));
  return carve_bytes(n1, n2, std::max(p, r), r);
}

static int waltmin_p(int64_t n1, int64_t n2, int r) {
  return std::max(r, std::min<int>(kMaxP, (int)std::min<int64_t>(std::min(n1, n2), r + kInitOversample)));
}

// Alg. 2 on one job's sample, its launches issued through `ex`; FA on the device.
static void waltmin_body(Exec &ex, const smp_params &prm, const smp_omega &om, const float *na2, double *Uout,
                         double *Vout, double *sigma, const Ws &w, const double *FA) {
  const int64_t n1 = om.n1, n2 = om.n2;
  const int r = prm.r, T = prm.T;
  const int p = waltmin_p(n1, n2, r);
  const int iters = prm.init_iters > 0 ? prm.init_iters : 2;
  const bool split = prm.omega_mode == SMP_OMEGA_SPLIT;
  const uint8_t *scsr = split ? om.sub_csr : nullptr;
  const uint8_t *scsc = split ? om.sub_csc : nullptr;

  // ---- init: subspace iteration on R = w .* P_Omega0(M~)
  gaussian_block(ex, n2, p, prm.seed, w.Y);
  // each sparse product applies the CholeskyQR map of its input (orth1_map)
  orth1_map(ex, w, w.Y, n2, p);
  for (int it = 0; it < iters; ++it) {
    spmm(ex, om.row_ptr, om.col_idx, om.w_csr, om.mt_csr, scsr, 0, w.Y, p, n1, w.M, w.X);
    orth1_map(ex, w, w.X, n1, p);
    spmm(ex, om.col_ptr, om.row_idx, om.w_csc, om.mt_csc, scsc, 0, w.X, p, n2, w.M, w.Y);
    if (it + 1 < iters) orth1_map(ex, w, w.Y, n2, p);
  }
  orth(ex, w, w.Y, n2, p);
  spmm(ex, om.row_ptr, om.col_idx, om.w_csr, om.mt_csr, scsr, 0, w.Y, p, n1, nullptr, w.X);
  // Rayleigh-Ritz: X = R Y; X^T X = W diag(lam) W^T; U0 = X W_r lam^-1/2, V0 = Y W_r
  jacobi_eig(ex, w.part, gram(ex, w, w.X, n1, p), p, r, w.Mu, w.Mv, w.sig);
  apply2(ex, w.X, n1, w.Mu, w.U, na2, FA, w.Y, n2, w.Mv, w.V, p, r);   // U0 (trimmed), V0

  if (T == 0) {
    scale_cols(ex, w.U, n1, r, w.sig);
  } else {
    // Alg. 2 orthonormalises the fixed factor before each half-step. The
    // least-squares solution for the other factor only changes basis with it
    // (U -> U R gives V -> V R^-T), so U V^T is the same; the factors are
    // orthonormalised once, before the last half-step, which also gives the
    // orthonormal V that the canonical form needs.
    for (int t = 0; t < T; ++t) {
      ls_solve(ex, om.col_ptr, om.row_idx, om.w_csc, om.mt_csc, scsc, 2 * t + 1, w.U, r, n2, w.V);
      if (t + 1 == T) orth(ex, w, w.V, n2, r);   // Q_V
      ls_solve(ex, om.row_ptr, om.col_idx, om.w_csr, om.mt_csr, scsr, 2 * t + 2, w.V, r, n1, w.U);
    }
  }
  double *sig_out = sigma ? sigma : w.sig;
  canonical(ex, w, w.U, n1, w.V, n2, r, Uout, Vout, sig_out);
  if (!sigma) scale_cols(ex, Uout, n1, r, sig_out);
}

hipError_t waltmin_run(const smp_params &prm, const smp_omega &om, const float *na2, double *Uout, double *Vout,
                       double *sigma, void *wsbase, hipStream_t st, const double *fa_in) {
  const Ws w = carve_ws(wsbase, om.n1, om.n2, waltmin_p(om.n1, om.n2, prm.r), prm.r);
  // F_A (the squared Frobenius norm of A in the sampler's fixed order): given, or summed here
  const double *FA = fa_in;
  if (!FA) {
    fixed_total(na2, om.n1, w.blocks, w.FA, st);
    FA = w.FA;
  }
  Exec ex(st);
  waltmin_body(ex, prm, om, na2, Uout, Vout, sigma, w, FA);
  return hipGetLastError();
}

// A group of WAltMin jobs: each job's launch sequence is recorded, the jobs
// are bucketed by sequence (same kernels in the same order: same r, T,
// initial iterations, subset mode and block-width class), and each bucket runs
// as one launch per step over all its jobs, from per-step argument tables
// copied to the device once (table_ws, waltmin_group_table_bytes bytes).
// With graph != 0 the bucket's launches are captured into one HIP graph and
// replayed once. Every job computes exactly what waltmin_run computes.
size_t waltmin_group_table_bytes(int njobs, const smp_params *prm, const smp_omega *om) {
  size_t total = 0;
  for (int j = 0; j < njobs; ++j) {
    std::vector<Op> ops;
    Exec rec(&ops);
    Ws w{};   // addresses are not used while recording sizes
    smp_omega o = om[j];
    waltmin_body(rec, prm[j], o, nullptr, nullptr, nullptr, nullptr, w, nullptr);
    for (const Op &op : ops) total += (op.arg.size() + 15) / 16 * 16;
  }
  return total + 256;
}

hipError_t waltmin_group_run(int njobs, const smp_params *prm, const smp_omega *om, const float *const *na2,
                             double *const *Uout, double *const *Vout, double *const *sigma, void *const *wsbase,
                             const double *const *fa, void *table_ws, int graph, hipStream_t st) {
  std::vector<std::vector<Op>> rec(njobs);
  for (int j = 0; j < njobs; ++j) {
    const Ws w = carve_ws(wsbase[j], om[j].n1, om[j].n2, waltmin_p(om[j].n1, om[j].n2, prm[j].r), prm[j].r);
    const double *FA = fa ? fa[j] : nullptr;
    if (!FA) {   // F_A in the sampler's fixed order, one small launch per job before the group runs
      fixed_total(na2[j], om[j].n1, w.blocks, w.FA, st);
      FA = w.FA;
    }
    Exec ex(&rec[j]);
    waltmin_body(ex, prm[j], om[j], na2[j], Uout[j], Vout[j], sigma ? sigma[j] : nullptr, w, FA);
  }
  // buckets of jobs with the same sequence of kernels
  std::vector<std::vector<int>> buckets;
  for (int j = 0; j < njobs; ++j) {
    bool placed = false;
    for (auto &b : buckets) {
      const std::vector<Op> &a = rec[b[0]], &c = rec[j];
      bool same = a.size() == c.size();
      for (size_t i = 0; same && i < a.size(); ++i)
        same = a[i].id == c[i].id && a[i].block.x == c[i].block.x && a[i].arg.size() == c[i].arg.size();
      if (same) {
        b.push_back(j);
        placed = true;
        break;
      }
    }
    if (!placed) buckets.push_back({j});
  }
  // argument tables: bucket by bucket, step by step, job by job
  std::vector<char> host;
  std::vector<std::vector<size_t>> offs(buckets.size());
  for (size_t bi = 0; bi < buckets.size(); ++bi) {
    const auto &b = buckets[bi];
    for (size_t i = 0; i < rec[b[0]].size(); ++i) {
      offs[bi].push_back(host.size());
      for (int j : b) host.insert(host.end(), rec[j][i].arg.begin(), rec[j][i].arg.end());
      host.resize((host.size() + 15) / 16 * 16);
    }
  }
  hipError_t e = hipMemcpyAsync(table_ws, host.data(), host.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;   // the host tables are freed on return
  char *dev = static_cast<char *>(table_ws);
  // a graph is captured on a stream of its own when the caller's is the null stream
  hipStream_t cs = st;
  if (graph && !st && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return e;
  for (size_t bi = 0; bi < buckets.size() && e == hipSuccess; ++bi) {
    const auto &b = buckets[bi];
    const std::vector<Op> &ops = rec[b[0]];
    if (graph && (e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) break;
    for (size_t i = 0; i < ops.size(); ++i) {
      unsigned gx = 1;
      for (int j : b) gx = std::max(gx, rec[j][i].grid.x);
      ops[i].launch(dev + offs[bi][i], dim3(gx, (unsigned)b.size()), ops[i].block, graph ? cs : st);
    }
    if (graph) {
      hipGraph_t g = nullptr;
      if ((e = hipStreamEndCapture(cs, &g)) != hipSuccess) break;
      hipGraphExec_t ge = nullptr;
      e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (e == hipSuccess) e = hipGraphLaunch(ge, cs);
      const hipError_t e2 = hipStreamSynchronize(cs);
      if (ge) hipGraphExecDestroy(ge);
      hipGraphDestroy(g);
      if (e == hipSuccess) e = e2;
    }
  }
  if (cs != st) hipStreamDestroy(cs);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace smp
