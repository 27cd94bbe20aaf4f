// Randomized TT rounding to fixed target ranks (App. A.3, eqs. randfinal and
// randprojection), over the two bonds from left to right.
//
// Bond k holds the TT as A_k B_k^T.  With the caller's Gaussian test matrix
// Omega_k (its column count is the target rank), the sketch of the small
// factor W = B_k^T Omega_k is formed first, then Y = A_k W, an orthonormal
// basis Q of range(Y), A_k' = Q and M_upd = Q^T A_k carried into the next
// core (reading: the QR that the text attaches to W can only be of A_k W,
// whose rows are A_k's).  Bond 1: A_1 = X (N_s x r1), B_1^T = (Theta x Phi)
// unfolded to r1 x (N_theta N_phi).  Bond 2: A_2 = (M_upd1 Theta) unfolded
// to (k1 N_theta) x r2, B_2^T = Phi.
//
// The orthonormal basis follows the shifted CholeskyQR3 of Fukaya, Kannan,
// Nakatsukasa, Yamamoto and Yanagisawa (2020): a Gram with a diagonal shift
// s = 11 (m n + n (n + 1)) u ||Y||^2 (the trace bounds ||Y||_2^2), its upper
// Cholesky factor R and Q = Y R^{-1}, then plain CholeskyQR passes on Q;
// with one more shifted pass (cholqr) it also covers a sketch of lower
// numerical rank than its width.  Every pass is a k x k Gram of the tall
// sketch and a tall product on the FP64 MFMA kernels, and M_upd = Q^T A_k
// one split-K product over the rows: the N_s-long work is N_s r k for the
// sketch and for M_upd plus ten N_s k^2 products, against N_s R^2 for the
// Gram route.  No eigensolver runs.
#include <math.h>

#include <algorithm>

#include "tt_ctx.h"

namespace tt {

namespace {

constexpr double UNIT_ROUNDOFF = 1.1102230246251565e-16;  // 2^-53

// Upper Cholesky factor R of a k x k Gram G (G = R^T R; only G's upper
// triangle is read), with s added to the diagonal first when shift_rows > 0,
// and R^{-1}, in one block.  R and Ri are k x k (ld ldr) with zero lower
// parts.  A pivot that is not positive raises FLAG_CHOL (its row then
// continues with pivot 1 so that the kernel ends normally).
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ G, int ldg, int k,
                                                  long long shift_rows, double* __restrict__ R,
                                                  double* __restrict__ Ri, int ldr,
                                                  int* __restrict__ dims) {
  __shared__ double red[256];
  __shared__ double sdiag;
  const int t = threadIdx.x;
  double shift = 0.0;
  if (shift_rows > 0) {
    double a = 0.0;
    for (int i = t; i < k; i += 256) a += G[(long long)i * ldg + i];
    red[t] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) red[t] += red[t + o];
      __syncthreads();
    }
    shift = 11.0 * ((double)shift_rows * k + (double)k * (k + 1)) * UNIT_ROUNDOFF * red[0];
  }
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      double d = G[(long long)j * ldg + j] + shift;
      for (int i = 0; i < j; ++i) d -= R[(long long)i * ldr + j] * R[(long long)i * ldr + j];
      sdiag = d;
    }
    __syncthreads();
    const double d = sdiag;
    const bool bad = !(d > 0.0);
    const double rjj = bad ? 1.0 : sqrt(d);
    if (bad && t == 0) atomicOr(&dims[D_FLAG], FLAG_CHOL);
    for (int l = j + t; l < k; l += 256) {
      double v = rjj;
      if (l > j) {
        v = G[(long long)j * ldg + l];
        for (int i = 0; i < j; ++i) v -= R[(long long)i * ldr + j] * R[(long long)i * ldr + l];
        v /= rjj;
      }
      R[(long long)j * ldr + l] = v;
    }
    for (int l = t; l < j; l += 256) R[(long long)j * ldr + l] = 0.0;
    __syncthreads();
  }
  // column c of R^{-1} solves R x = e_c by back substitution (a thread each)
  for (int cc = t; cc < k; cc += 256) {
    for (int i = k - 1; i > cc; --i) Ri[(long long)i * ldr + cc] = 0.0;
    Ri[(long long)cc * ldr + cc] = 1.0 / R[(long long)cc * ldr + cc];
    for (int i = cc - 1; i >= 0; --i) {
      double v = 0.0;
      for (int l = i + 1; l <= cc; ++l) v += R[(long long)i * ldr + l] * Ri[(long long)l * ldr + cc];
      Ri[(long long)i * ldr + cc] = -v / R[(long long)i * ldr + i];
    }
  }
}

// The same for k <= CHOL_LDS_K, LDS-resident (k (k + 1) doubles of dynamic LDS):
// right-looking Cholesky (per pivot: scale its row, update the trailing
// upper triangle), then R^{-1} in place column by column (column j from the
// inverted leading block and R's column j), so that every step is parallel
// over rows and the serial chain is k steps of LDS work.
constexpr int CHOL_LDS_K = 128;

__global__ __launch_bounds__(256) void k_chol_inv_lds(const double* __restrict__ G, int ldg, int k,
                                                      long long shift_rows, double* __restrict__ R,
                                                      double* __restrict__ Ri, int ldr,
                                                      int* __restrict__ dims) {
  extern __shared__ double A[];  // k x k, ld lk = k + 1 (odd: rows in distinct banks)
  __shared__ double red[256];
  const int t = threadIdx.x, lk = k + 1;
  double a = 0.0;
  for (int i = t; i < k; i += 256) a += G[(long long)i * ldg + i];
  red[t] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double shift =
      shift_rows > 0 ? 11.0 * ((double)shift_rows * k + (double)k * (k + 1)) * UNIT_ROUNDOFF * red[0] : 0.0;
  for (int e = t; e < k * k; e += 256) {
    const int i = e / k, l = e % k;
    A[i * lk + l] = l >= i ? G[(long long)i * ldg + l] + (l == i ? shift : 0.0) : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    __syncthreads();  // the previous pivot's trailing update is complete
    const double d = A[j * lk + j];
    const bool bad = !(d > 0.0);
    const double rjj = bad ? 1.0 : sqrt(d);
    if (bad && t == 0) atomicOr(&dims[D_FLAG], FLAG_CHOL);
    __syncthreads();
    const double inv = 1.0 / rjj;
    for (int l = j + t; l < k; l += 256) A[j * lk + l] = l == j ? rjj : A[j * lk + l] * inv;
    __syncthreads();
    for (int i = j + 1 + (t >> 4); i < k; i += 16) {
      const double rji = A[j * lk + i];
      for (int l = i + (t & 15); l < k; l += 16) A[i * lk + l] -= rji * A[j * lk + l];
    }
  }
  __syncthreads();
  for (int e = t; e < k * k; e += 256) {
    const int i = e / k, l = e % k;
    R[(long long)i * ldr + l] = l >= i ? A[i * lk + l] : 0.0;
  }
  // in place: after column j, A[0:j+1, 0:j+1] holds the leading block of
  // R^{-1}; row i's dot product for column j is split between threads i and
  // i + 128 (halves of l in [i, j)), each with four independent partial sums
  const int ri = t & 127, half = t >> 7;
  for (int j = 0; j < k; ++j) {
    const double ajj = 1.0 / A[j * lk + j];
    double v = 0.0;
    if (ri < j) {
      const int mid = (ri + j) >> 1;
      const int l0 = half ? mid : ri, l1 = half ? j : mid;
      double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
      int l = l0;
      for (; l + 3 < l1; l += 4) {
        v0 += A[ri * lk + l] * A[l * lk + j];
        v1 += A[ri * lk + l + 1] * A[(l + 1) * lk + j];
        v2 += A[ri * lk + l + 2] * A[(l + 2) * lk + j];
        v3 += A[ri * lk + l + 3] * A[(l + 3) * lk + j];
      }
      for (; l < l1; ++l) v0 += A[ri * lk + l] * A[l * lk + j];
      v = (v0 + v1) + (v2 + v3);
    }
    red[t] = v;
    __syncthreads();
    if (t < j) A[t * lk + j] = -(red[t] + red[t + 128]) * ajj;
    if (t == 0) A[j * lk + j] = ajj;
    __syncthreads();
  }
  for (int e = t; e < k * k; e += 256) {
    const int i = e / k, l = e % k;
    Ri[(long long)i * ldr + l] = l >= i ? A[i * lk + l] : 0.0;
  }
}

// One factorisation: the LDS kernel when k fits, else the global one.
void chol_inv(const double* G, int ldg, int k, long long shift_rows, double* R, double* Ri, int ldr,
              int* dims, hipStream_t s) {
  if (k <= CHOL_LDS_K)
    k_chol_inv_lds<<<1, 256, (size_t)k * (k + 1) * sizeof(double), s>>>(G, ldg, k, shift_rows, R, Ri, ldr,
                                                                          dims);
  else
    k_chol_inv<<<1, 256, 0, s>>>(G, ldg, k, shift_rows, R, Ri, ldr, dims);
}

__global__ void k_set_ranks(int* __restrict__ dims, int r1, int r2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dims[D_R1] = r1;
    dims[D_R2] = r2;
  }
}

int ru8(int x) { return (x + 7) / 8 * 8; }

#define RCHK(ctx, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ctx_fail(ctx, TT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// M (m x n, ld ldm) = Q^T A over K rows (Q: K x m, A: K x n), split over
// row slices into per-slice partials (gpart) summed in a fixed order.
void contract_tall(tt_ctx* c, const double* Q, int ldq, const double* A, int lda, int K, int m, int n,
                   double* M, int ldm) {
  const long long tile = (long long)m * n;
  const long long avail = (long long)c->nt * c->R1c * c->R1c;  // gpart holds at least this
  const int zmax = (int)std::max<long long>(1, std::min<long long>(avail / tile, 128));
  int ks = (K + zmax - 1) / zmax;
  ks = std::max(64, (ks + 15) / 16 * 16);
  const int nz = (K + ks - 1) / ks;
  GemmDesc g = gd(Q, ldq, 1, A, lda, 0, c->gpart, n, dimc(m), dimc(n), dimc(K));
  g.ksplit = ks;
  g.sC = tile;
  gemm(g, m, n, nz, c->dims, c->st);
  sum_partials(c->gpart, tile, nz, M, ldm, n, dimc(m), dimc(n), m, n, c->dims, c->st);
}

// The Gram of columns [off, off + n) of Z (K rows, ld ldz) into G (ld N):
// the tall MFMA Gram for the spatial bond, the generic product for bond 2.
struct Tall {
  int K;
  double* Z;
  int ldz;
  bool spatial;
};

void gram_cols(tt_ctx* c, const Tall& t, int off, int n, double* G, int ldg, const GramPlan* p) {
  if (t.spatial) {
    gram_tall(*p, t.Z + off, dimc(n), c->gpart, G, ldg, c->dims, c->st);
  } else {
    contract_tall(c, t.Z + off, t.ldz, t.Z + off, t.ldz, t.K, n, n, G, ldg);
  }
}

// C (K x n, ld ldc) = Z[:, off : off + kk] B (kk x n, ld ldb).
void tall_product(tt_ctx* c, const Tall& t, int off, int kk, const double* B, int ldb, double* C,
                  int ldc, int n) {
  if (t.spatial) {
    gemm_tall(t.K, t.Z + off, t.ldz, B, ldb, C, ldc, dimc(kk), dimc(n), kk, n, c->dims, c->st);
  } else {
    GemmDesc g = gd(t.Z + off, t.ldz, 0, B, ldb, 0, C, ldc, dimc(t.K), dimc(n), dimc(kk));
    gemm(g, t.K, n, 1, c->dims, c->st);
  }
}

// Orthonormal basis of Y = Z[:, 0 : k] (slot b at column o1 >= k) into
// Qout (K x k, ld ldq): three shifted CholeskyQR passes, then two plain
// ones (shifted CholeskyQR3 with two more shifted passes).  A
// well-conditioned Y needs only the first shift; the others lift directions
// that Y holds at rounding level (a target rank past the numerical rank) by
// 1/sqrt(s) each (at least about 30x at K k^2 <= 1e9 rows x columns^2), so
// that the plain passes, which need cond < u^{-1/2}, finish them
// orthonormal as a Householder QR would.  Each pass: the k x k Gram of its slot, the
// Cholesky factor and inverse, and the product into the other slot (the last
// into Qout).  Scratch: three N x N eigen slots.
constexpr int CHOLQR_PASSES = 5, CHOLQR_SHIFTED = 3;

void cholqr(tt_ctx* c, const Tall& t, int k, int o1, double* Qout, int ldq, const GramPlan* p) {
  const int N = c->N;
  double *G = c->E[0].V, *R = c->E[1].V, *Ri = c->E[2].V;
  hipStream_t s = c->st;
  int from = 0, to = o1;
  for (int pass = 0; pass < CHOLQR_PASSES; ++pass) {
    gram_cols(c, t, from, k, G, N, p);
    chol_inv(G, N, k, pass < CHOLQR_SHIFTED ? (long long)t.K : 0, R, Ri, N, c->dims, s);
    if (pass == CHOLQR_PASSES - 1) tall_product(c, t, from, k, Ri, N, Qout, ldq, k);
    else tall_product(c, t, from, k, Ri, N, t.Z + to, t.ldz, k);
    std::swap(from, to);
  }
}


}  // namespace

}  // namespace tt

using namespace tt;

extern "C" tt_status tt_round_randomized(tt_ctx* c, const double* omega1, int32_t k1,
                                         const double* omega2, int32_t k2, int32_t ranks_out[2]) {
  if (!c) return ctx_fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (c->poisoned) return ctx_fail(c, TT_ERR_STATE, "context poisoned");
  if (!omega1 || !omega2) return ctx_fail(c, TT_ERR_INVALID_ARG, "null test matrix");
  if (c->mixed) return ctx_fail(c, TT_ERR_INVALID_ARG, "randomized rounding needs a TT_FP64 context");
  hipStream_t s = c->st;
  int r[2];
  RCHK(c, hipMemcpyAsync(r, c->dims, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  RCHK(c, hipStreamSynchronize(s));
  const int r1 = r[0], r2 = r[1], nt = c->nt, np = c->np, ns = c->ns, N = c->N;
  if (k1 < 1 || k2 < 1 || k1 > r1 || k2 > r2 || k1 > nt * np || k2 > np || k2 > k1 * nt)
    return ctx_fail(c, TT_ERR_INVALID_ARG,
                    "target ranks must satisfy 1 <= k1 <= min(r1, N_theta N_phi) and "
                    "1 <= k2 <= min(r2, N_phi, k1 N_theta)");
  // two 8-column-aligned slots per tall factor: [Y / Q'' | Q']
  const int o1 = ru8(k1), q1 = ru8(k2);
  if (o1 + k1 > std::min(c->R1c, c->ldC) || q1 + k2 > c->R2c)
    return ctx_fail(c, TT_ERR_INVALID_ARG, "rank capacity too small for the sketch slots");
  if (c->gb.on && c->nhist > 0) c->gb.stale = true;
  const int r2c = c->r2c, R1c = c->R1c, R2c = c->R2c;
  // ---- bond 1 ---------------------------------------------------------------
  // E_l = Phi Omega1_l (r2 x k1 per theta ordinate l; rows (l, b) of T1)
  GemmDesc e = gd(c->Ph, np, 0, omega1, k1, 0, c->T1, k1, dimc(r2), dimc(k1), dimc(np));
  e.sB = (long long)np * k1;
  e.sC = (long long)r2 * k1;
  gemm(e, r2, k1, nt, c->dims, s);
  // W1 = sum_l Theta_l E_l (r1 x k1): per-l partials, summed in a fixed order
  GemmDesc w = gd(c->Th, nt * r2c, 0, c->T1, k1, 0, c->gpart, k1, dimc(r1), dimc(k1), dimc(r2));
  w.sA = r2c;
  w.sB = (long long)r2 * k1;
  w.sC = (long long)r1 * k1;
  gemm(w, r1, k1, nt, c->dims, s);
  double* W1 = c->M1;
  sum_partials(c->gpart, (long long)r1 * k1, nt, W1, k1, k1, dimc(r1), dimc(k1), r1, k1, c->dims, s);
  double* Z = c->Xcat;
  const int ldz = c->ldC;
  gemm_tall(ns, c->X, c->ldX, W1, k1, Z, ldz, dimc(r1), dimc(k1), r1, k1, c->dims, s);
  // the sketch's k1 columns (row-slice form up to 384), when its partial
  // tiles fit the Gram partial buffer (sized at creation as below)
  GramPlan p1 = gram_plan(ns, k1, ldz);
  const size_t gpart_doubles =
      std::max(std::max(gram_partial_doubles(gram_plan(ns, R1c, ldz)),
                        gram_partial_doubles(gram_plan(ns, c->r1c, c->ldX))),
               std::max((size_t)nt * R1c * R1c, (size_t)nt * R2c * R2c));
  if (gram_partial_doubles(p1) > gpart_doubles) p1 = gram_plan(ns, R1c, ldz);
  cholqr(c, Tall{ns, Z, ldz, true}, k1, o1, c->Xn, c->ldX, &p1);
  double* M1 = c->Mupd1;  // k1 x r1 = Q1^T X, ld R1c
  contract_tall(c, c->Xn, c->ldX, c->X, c->ldX, ns, k1, r1, M1, R1c);
  // ---- bond 2 ---------------------------------------------------------------
  // A2 = M1 Theta: rows (i, l) of T1 with ld r2c (columns past r2 unused)
  GemmDesc a = gd(M1, R1c, 0, c->Th, nt * r2c, 0, c->T1, nt * r2c, dimc(k1), dimc(nt * r2c), dimc(r1));
  gemm(a, k1, nt * r2c, 1, c->dims, s);
  // W2 = Phi Omega2 (r2 x k2)
  double* W2 = c->E[4].V;  // r2 x k2
  GemmDesc w2 = gd(c->Ph, np, 0, omega2, k2, 0, W2, k2, dimc(r2), dimc(k2), dimc(np));
  gemm(w2, r2, k2, 1, c->dims, s);
  const int K2 = k1 * nt;
  double* Z2 = c->Thcat;
  GemmDesc y2 = gd(c->T1, r2c, 0, W2, k2, 0, Z2, R2c, dimc(K2), dimc(k2), dimc(r2));
  gemm(y2, K2, k2, 1, c->dims, s);
  // Theta' = Q2 reshaped: rows (i, l) of the state's Theta (ld r2c)
  cholqr(c, Tall{K2, Z2, R2c, false}, k2, q1, c->Th, r2c, nullptr);
  double* M2 = c->E[3].V;  // k2 x r2 = Q2^T A2, ld N
  contract_tall(c, c->Th, r2c, c->T1, r2c, K2, k2, r2, M2, N);
  // Phi' = M2 Phi (k2 x N_phi), through Phi_cat
  GemmDesc ph = gd(M2, N, 0, c->Ph, np, 0, c->Phcat, np, dimc(k2), dimc(np), dimc(r2));
  gemm(ph, k2, np, 1, c->dims, s);
  RCHK(c, hipMemcpyAsync(c->Ph, c->Phcat, (size_t)k2 * np * 8, hipMemcpyDeviceToDevice, s));
  k_set_ranks<<<1, 64, 0, s>>>(c->dims, k1, k2);
  RCHK(c, hipGetLastError());
  std::swap(c->X, c->Xn);
  int flag = 0;
  RCHK(c, hipMemcpyAsync(&flag, c->dims + D_FLAG, sizeof(int), hipMemcpyDeviceToHost, s));
  RCHK(c, hipStreamSynchronize(s));
  if (flag) {
    c->poisoned = true;
    return ctx_fail(c, TT_ERR_NUMERIC,
                    flag & FLAG_CHOL ? "numerical failure: a sketch Gram lost definiteness"
                                     : "numerical failure");
  }
  if (ranks_out) {
    ranks_out[0] = k1;
    ranks_out[1] = k2;
  }
  return TT_OK;
}
