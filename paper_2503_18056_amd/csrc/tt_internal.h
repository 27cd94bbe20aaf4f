// Internal declarations of the MI355X tensor-train S_N library.
//
// Ranks are data dependent (tolerance-driven truncation), so every size a
// kernel needs at run time lives in a small int32 table on the device (the
// "dims" table below).  Launch grids are sized for the rank capacities and
// blocks beyond the live sizes exit early; no step needs a host round trip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tt {

// ---- device dims table ----------------------------------------------------
enum DimIndex : int {
  D_R1 = 0,      // state rank r1
  D_R2,          // state rank r2
  D_RC1,         // concatenated rank R1 (bond 1)
  D_RC2,         // concatenated rank R2 (bond 2)
  D_KA1,         // kept Gram eigenpairs, bond 1, left side (A = X_cat)
  D_KB1,         // kept, bond 1, right side (B_1)
  D_KM1,         // number of singular values of M at bond 1 = min(kA, kB)
  D_SIDE1,       // 0: kA <= kB (left vectors of M computed); 1: right vectors
  D_R1N,         // truncated rank r1'
  D_KEA1,        // effective inner size for P1 (0 when the tensor is zero)
  D_KEB1,        // effective inner size for M_upd1
  D_KA2, D_KB2, D_KM2, D_SIDE2, D_R2N, D_KEA2, D_KEB2,
  D_FLAG,        // error bits (FLAG_*)
  D_REPLAY1,     // replayed rank, bond 1 (<= 0: rule)
  D_REPLAY2,     // replayed rank, bond 2
  D_KC1,         // singular vectors computed for M, bond 1
  D_KC2,
  D_R1NT,        // r1' * ntheta
  D_ZERO1,       // 1 when bond 1 found a zero tensor
  D_ZERO2,
  D_TGK1,        // order 2 min(kA, kB) of the Golub-Kahan tridiagonal, bond 1
  D_TGK2,
  D_HSLOT,       // next rank-history slot (steps recorded since the cores were set)
  D_SCHEDPOS,    // next entry of the replayed rank schedule
  D_JAC_MAXSW,   // cap on the one-sided Jacobi SVD's sweeps (<= 0: its own limit)
  D_NDIMS = 64
};

enum : int {
  FLAG_NONFINITE = 1,
  FLAG_NEWTON = 2,
  FLAG_EIG = 4,
  FLAG_BARRIER = 8,  // a grid barrier of a multi-block eigensolver timed out
  FLAG_NOCONV = 16,  // the one-sided Jacobi SVD ran out of sweeps
  FLAG_CHOL = 32,    // a Cholesky factor of a sketch Gram met a non-positive pivot
};

// diagnostics (double table)
enum DiagIndex : int {
  G_NORM2 = 0, G_DELTA2, G_KA1, G_KB1, G_KA2, G_KB2, G_R1N, G_R2N,
  G_TAIL1, G_TAIL2, G_S1, G_SR1, G_SR1P, G_SR2, G_SR2P, G_RC1, G_NDIAG = 32
};

// A size evaluated on the device: (idx >= 0 ? dims[idx] : 0) * mul + add.
struct DimExpr {
  int idx, mul, add;
};
__host__ __device__ inline DimExpr dimc(int v) { return DimExpr{-1, 0, v}; }
__host__ __device__ inline DimExpr dimv(int idx, int mul = 1, int add = 0) {
  return DimExpr{idx, mul, add};
}
__device__ inline int eval_dim(const int* dims, DimExpr e) {
  return (e.idx >= 0 ? dims[e.idx] : 0) * e.mul + e.add;
}

// ---- generic FP64 GEMM ----------------------------------------------------
// C[m x n] = alpha * rs(i) * sum_l op(A)[i,l] ks(l) op(B)[l,j] * cs(j) + beta*C
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int lda, ldb, ldc;
  long long sA, sB, sC;      // batch strides (blockIdx.z)
  int transA, transB;
  DimExpr m, n, k;
  double alpha, beta;
  const double* rowscale;    // length m or null
  const double* colscale;    // length n or null
  const double* kscale;      // length k or null
  int cond_idx, cond_val;    // run only if dims[cond_idx] == cond_val (idx < 0: always)
  // per-batch live size: with bclip_idx >= 0, batch z uses
  // lim = dims[bclip_idx] - z * bclip_mul; it is skipped when lim <= bclip_min
  // and m, n, k are clipped to lim.
  int bclip_idx, bclip_mul, bclip_min;
  // ksplit > 0: split-K, batch z contracts l in [z ksplit, min((z+1) ksplit, k))
  // (A, B, kscale offset along k in the kernel; sA, sB unused); a batch past
  // the end writes zeros, so its partial slot is defined
  int ksplit;
};
void gemm(const GemmDesc& g, int mcap, int ncap, int batch, const int* dims, hipStream_t s);
// out[i][j] = sum_{z < nz} part[z][i][j] (fixed order) + beta out[i][j],
// i < m, j < n (dynamic).
void sum_partials(const double* part, long long zstride, int nz, double* out, int ldo, int ldp,
                  DimExpr m, DimExpr n, int mcap, int ncap, const int* dims, hipStream_t s,
                  double beta = 0.0);

// ---- tall Gram on MFMA: G = A^T A, A is K x n (row-major, lda), n <= ncap
struct GramPlan {
  int K, ncap, lda;
  // above 384 columns (FP64 and the sliced FP32 form): 128-column tile
  // pairs, wslices row slices of wkslice rows
  int wtiles, wpairs, wslices, wkslice;
  // row-slice form (ncap <= 384): nblk blocks of rows_per_blk rows, up to
  // ntask_cap upper-triangular 32x32 tasks each
  bool rows_mode;
  int nblk, rows_per_blk, ntask_cap;
};
GramPlan gram_plan(int K, int ncap, int lda);
size_t gram_partial_doubles(const GramPlan& p);
void gram_tall(const GramPlan& p, const double* A, DimExpr n, double* partial, double* G,
               int ldg, const int* dims, hipStream_t s);
void gram_tall_partial(const GramPlan& p, const double* A, DimExpr n, double* partial,
                       const int* dims, hipStream_t s);
void gram_tall_reduce(const GramPlan& p, DimExpr n, const double* partial, double* G, int ldg,
                      const int* dims, hipStream_t s);

// ---- FP32-mixed form: sliced (error-free) Gram of an FP32 matrix on FP32
// MFMA into partial tiles (reduce with gram_split_reduce); colmax is scratch
// of ncap words; slices: 11-bit slices per entry (1 .. 6; others give 4).
constexpr int GRAM_SLICES_DEFAULT = 4;
void gram_split_partial(const GramPlan& p, const float* A, DimExpr n, unsigned* colmax,
                        double* partial, const int* dims, hipStream_t s,
                        int slices = GRAM_SLICES_DEFAULT);
void gram_split_reduce(const GramPlan& p, DimExpr n, const double* partial, double* G, int ldg,
                       const int* dims, hipStream_t s);
// C (FP32) = A (FP32) * B (FP64, split hi/lo) on FP32 MFMA.
void gemm_tall_f32(int K, const float* A, int lda, const double* B, int ldb, float* C, int ldc,
                   DimExpr kdim, DimExpr ndim, int ncap, const int* dims, hipStream_t s);

// ---- tall GEMM on MFMA: C[K x n] = A[K x k] * B[k x n], k, n dynamic
void gemm_tall(int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
               DimExpr kdim, DimExpr ndim, int kcap, int ncap, const int* dims, hipStream_t s);

// ---- symmetric eigensolver (batched, one job per matrix) ------------------
// A (n x n, lda) is destroyed.  Outputs: lam (n, descending), V (n x n, ldv,
// columns = eigenvectors in descending order, only the kept ones are
// computed), sq / isq (sqrt and 1/sqrt of kept eigenvalues), dims[kept_idx]
// = number kept: lambda > clip * n * u * lambda_max and lambda > 0.
struct EigJob {
  double* A;
  int lda;
  int n_idx;        // dims index holding n
  double* lam;
  double* V;
  int ldv;
  double* sq;
  double* isq;
  int kept_idx;     // dims index receiving the kept count
  double clip;      // clip factor (1: Gram clip rule; 0: keep all lambda > 0)
  double* work;     // eig_work_doubles(ncap)
};
size_t eig_work_doubles(int ncap);
void eig_batched(const EigJob* jobs, int njobs, int ncap, int* dims, hipStream_t s);

// ---- small SVD (one matrix) -------------------------------------------------
// M is a x b (row-major, ldm), a = dims[a_idx], b = dims[b_idx], side =
// dims[side_idx] (0 when a <= b).  Golub-Kahan bidiagonalisation of the
// taller orientation, then the eigenpairs of the order-2q Golub-Kahan
// tridiagonal (q = min(a, b); eigenvalues +-sigma) by the same divide and
// conquer, so singular values carry absolute error ~ u sigma_1 rather than
// the u sigma_1^2 / sigma of an eigensolve of M M^T.  Outputs in the job:
// lam = sigma (q, descending), V = singular vectors of the short side
// (side 0: left vectors of M, a x q; side 1: right vectors, b x q), each
// column sign-fixed (largest |entry| positive), sq = sigma, isq = 1/sigma,
// dims[kept_idx] = number with sigma > 2q u sigma_1.  J.A is a work matrix
// of at least max(a,b) x min(a,b) (row-major, J.lda); dims[J.n_idx]
// receives 2q.  2 q_max <= ncap2 <= 2048, J.work holds eig_work_doubles(ncap2);
// max(a, b) <= pcap <= 1024.
void svd_short_side(const double* M, int ldm, int a_idx, int b_idx, int side_idx,
                    const EigJob& job, int ncap2, int pcap, int* dims, hipStream_t s);

// Largest static + dynamic LDS (bytes) of the launches of eig_batched at
// capacity N, and of svd_short_side at Golub-Kahan capacity ncap2 and longer
// side pcap; `which` (may be null) names that kernel.  runtime: take the
// static sizes from the HIP runtime where it reports more.  lds_fits: within
// the 160 KiB of one CU.
size_t eig_lds_bytes(int N, bool runtime, const char** which);
size_t svd_lds_bytes(int ncap2, int pcap, bool runtime, const char** which);
bool lds_fits(size_t bytes);

}  // namespace tt
