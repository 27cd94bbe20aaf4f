// Dense FP64 contractions: a generic LDS-tiled GEMM for the rank-sized
// products, and MFMA kernels for the two N_s-long contractions of the step:
// the left Gram of the spatial core (G = X_cat^T X_cat, App. A.2 G_A = A^T A)
// and the spatial core update (X' = X_cat P, App. A.2 A' = A V_A S_A^-1 U).
#include "tt_internal.h"

namespace tt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Generic GEMM (vector FP64, 64x64 tiles, 16-deep K slabs staged in LDS).
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gemm(GemmDesc g, const int* __restrict__ dims) {
  if (g.cond_idx >= 0 && dims[g.cond_idx] != g.cond_val) return;
  int m = eval_dim(dims, g.m), n = eval_dim(dims, g.n), k = eval_dim(dims, g.k);
  if (g.bclip_idx >= 0) {
    const int lim = dims[g.bclip_idx] - (int)blockIdx.z * g.bclip_mul;
    if (lim <= g.bclip_min) return;
    m = min(m, lim);
    n = min(n, lim);
    k = min(k, lim);
  }
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  if (i0 >= m || j0 >= n) return;
  const double* A = g.A + (long long)blockIdx.z * g.sA;
  const double* B = g.B + (long long)blockIdx.z * g.sB;
  double* C = g.C + (long long)blockIdx.z * g.sC;
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int l0 = 0; l0 < k; l0 += 16) {
#pragma unroll
    for (int e = tid; e < 1024; e += 256) {
      int i, l;
      if (TA == 0) { i = e >> 4; l = e & 15; } else { l = e >> 6; i = e & 63; }
      const int gi = i0 + i, gl = l0 + l;
      double v = 0.0;
      if (gi < m && gl < k) {
        v = TA == 0 ? A[(long long)gi * g.lda + gl] : A[(long long)gl * g.lda + gi];
        if (g.kscale) v *= g.kscale[gl];
      }
      As[l][i] = v;
    }
#pragma unroll
    for (int e = tid; e < 1024; e += 256) {
      int j, l;
      if (TB == 0) { l = e >> 6; j = e & 63; } else { j = e >> 4; l = e & 15; }
      const int gj = j0 + j, gl = l0 + l;
      double v = 0.0;
      if (gj < n && gl < k)
        v = TB == 0 ? B[(long long)gl * g.ldb + gj] : B[(long long)gj * g.ldb + gl];
      Bs[l][j] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int l = 0; l < 16; ++l) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[l][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[l][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty + 16 * r;
    if (i >= m) continue;
    const double rs = g.rowscale ? g.rowscale[i] : 1.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx + 16 * c;
      if (j >= n) continue;
      double v = g.alpha * acc[r][c] * rs * (g.colscale ? g.colscale[j] : 1.0);
      double* dst = C + (long long)i * g.ldc + j;
      *dst = g.beta == 0.0 ? v : v + g.beta * *dst;
    }
  }
}

__global__ void k_sum_partials(const double* __restrict__ part, long long zstride, int nz,
                               double* __restrict__ out, int ldo, int ldp, DimExpr mdim,
                               DimExpr ndim, const int* __restrict__ dims) {
  const int m = eval_dim(dims, mdim), n = eval_dim(dims, ndim);
  const long long tot = (long long)m * n;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e % n);
    double acc = 0.0;
    for (int z = 0; z < nz; ++z) acc += part[z * zstride + (long long)i * ldp + j];
    out[(long long)i * ldo + j] = acc;
  }
}

void sum_partials(const double* part, long long zstride, int nz, double* out, int ldo, int ldp,
                  DimExpr m, DimExpr n, int mcap, int ncap, const int* dims, hipStream_t s) {
  long long tot = (long long)mcap * ncap;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_sum_partials<<<blocks, 256, 0, s>>>(part, zstride, nz, out, ldo, ldp, m, n, dims);
}

void gemm(const GemmDesc& g, int mcap, int ncap, int batch, const int* dims, hipStream_t s) {
  if (mcap <= 0 || ncap <= 0 || batch <= 0) return;
  dim3 grid((ncap + 63) / 64, (mcap + 63) / 64, batch);
  if (!g.transA && !g.transB) k_gemm<0, 0><<<grid, 256, 0, s>>>(g, dims);
  else if (g.transA && !g.transB) k_gemm<1, 0><<<grid, 256, 0, s>>>(g, dims);
  else if (!g.transA && g.transB) k_gemm<0, 1><<<grid, 256, 0, s>>>(g, dims);
  else k_gemm<1, 1><<<grid, 256, 0, s>>>(g, dims);
}

// ---------------------------------------------------------------------------
// MFMA f64 16x16x4 operand/result layout (CDNA3/CDNA4):
//   A operand: lane l supplies A[row = l % 16][k = l / 16]
//   B operand: lane l supplies B[k = l / 16][col = l % 16]
//   D result : lane l, item r holds D[row = l / 16 + 4 * r][col = l % 16]
__device__ inline f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Tall Gram: partial[slice][pair] = A[rows of slice, tile ti]^T A[rows, tile tj]
// for the upper-triangular 64x64 tile pairs (ti <= tj).  Four waves per
// block, each owning a 32x32 quarter of the tile (2x2 MFMA blocks).
__global__ __launch_bounds__(256) void k_gram_tall(const double* __restrict__ A, int lda, int K,
                                                   int kslice, DimExpr ndim,
                                                   const int* __restrict__ dims, int tiles,
                                                   double* __restrict__ partial) {
  const int n = eval_dim(dims, ndim);
  const int pair = blockIdx.x, slice = blockIdx.y;
  int ti = 0, rem = pair;
  while (rem >= tiles - ti) { rem -= tiles - ti; ++ti; }
  const int tj = ti + rem;
  if (ti * 64 >= n || tj * 64 >= n) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int a0 = ti * 64 + wr * 32, b0 = tj * 64 + wc * 32;
  const int col = lane & 15, krow = lane >> 4;
  const int k_begin = slice * kslice;
  const int k_end = min(K, k_begin + kslice);
  f64x4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  const bool va0 = a0 + col < n, va1 = a0 + 16 + col < n;
  const bool vb0 = b0 + col < n, vb1 = b0 + 16 + col < n;
  for (int k = k_begin; k < k_end; k += 4) {
    const int row = k + krow;
    const bool vr = row < k_end;
    const double* rp = A + (long long)row * lda;
    const double x0 = (vr && va0) ? rp[a0 + col] : 0.0;
    const double x1 = (vr && va1) ? rp[a0 + 16 + col] : 0.0;
    const double y0 = (vr && vb0) ? rp[b0 + col] : 0.0;
    const double y1 = (vr && vb1) ? rp[b0 + 16 + col] : 0.0;
    acc[0][0] = mfma16(x0, y0, acc[0][0]);
    acc[0][1] = mfma16(x0, y1, acc[0][1]);
    acc[1][0] = mfma16(x1, y0, acc[1][0]);
    acc[1][1] = mfma16(x1, y1, acc[1][1]);
  }
  const int npairs = gridDim.x;
  double* out = partial + ((long long)slice * npairs + pair) * 4096;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = wr * 32 + 16 * p + (lane >> 4) + 4 * r;
        const int jj = wc * 32 + 16 * q + (lane & 15);
        out[ii * 64 + jj] = acc[p][q][r];
      }
}

// Fixed-order reduction of the slices (deterministic), mirrored into G.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ partial,
                                                     int slices, int npairs, int tiles,
                                                     DimExpr ndim, const int* __restrict__ dims,
                                                     double* __restrict__ G, int ldg) {
  const int n = eval_dim(dims, ndim);
  const int pair = blockIdx.y;
  int ti = 0, rem = pair;
  while (rem >= tiles - ti) { rem -= tiles - ti; ++ti; }
  const int tj = ti + rem;
  if (ti * 64 >= n || tj * 64 >= n) return;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < 4096; e += gridDim.x * 256) {
    const int ii = e >> 6, jj = e & 63;
    const int i = ti * 64 + ii, j = tj * 64 + jj;
    if (i >= n || j >= n) continue;
    double s = 0.0;
    for (int sl = 0; sl < slices; ++sl) s += partial[((long long)sl * npairs + pair) * 4096 + e];
    G[(long long)i * ldg + j] = s;
    G[(long long)j * ldg + i] = s;
  }
}

GramPlan gram_plan(int K, int ncap, int lda) {
  GramPlan p;
  p.K = K;
  p.ncap = ncap;
  p.lda = lda;
  p.tiles = (ncap + 63) / 64;
  p.pairs = p.tiles * (p.tiles + 1) / 2;
  int want = (2048 + p.pairs - 1) / p.pairs;          // aim at ~2048 blocks
  int maxs = (K + 63) / 64;                            // at least 64 rows a slice
  p.slices = want < maxs ? want : maxs;
  if (p.slices < 1) p.slices = 1;
  int ks = (K + p.slices - 1) / p.slices;
  p.kslice = (ks + 3) / 4 * 4;
  p.slices = (K + p.kslice - 1) / p.kslice;
  if (p.slices < 1) p.slices = 1;
  return p;
}

size_t gram_partial_doubles(const GramPlan& p) { return (size_t)p.slices * p.pairs * 4096; }

void gram_tall_partial(const GramPlan& p, const double* A, DimExpr n, double* partial,
                       const int* dims, hipStream_t s) {
  k_gram_tall<<<dim3(p.pairs, p.slices), 256, 0, s>>>(A, p.lda, p.K, p.kslice, n, dims, p.tiles,
                                                      partial);
}
void gram_tall_reduce(const GramPlan& p, DimExpr n, const double* partial, double* G, int ldg,
                      const int* dims, hipStream_t s) {
  k_gram_reduce<<<dim3(4, p.pairs), 256, 0, s>>>(partial, p.slices, p.pairs, p.tiles, n, dims, G,
                                                 ldg);
}
void gram_tall(const GramPlan& p, const double* A, DimExpr n, double* partial, double* G, int ldg,
               const int* dims, hipStream_t s) {
  gram_tall_partial(p, A, n, partial, dims, s);
  gram_tall_reduce(p, n, partial, G, ldg, dims, s);
}

// ---------------------------------------------------------------------------
// Tall GEMM C[K x n] = A[K x k] B[k x n] on MFMA; 64x64 output tile per
// block, 32x32 per wave.
__global__ __launch_bounds__(256) void k_gemm_tall(int K, const double* __restrict__ A, int lda,
                                                   const double* __restrict__ B, int ldb,
                                                   double* __restrict__ C, int ldc,
                                                   DimExpr kdim, DimExpr ndim,
                                                   const int* __restrict__ dims) {
  const int kk = eval_dim(dims, kdim), n = eval_dim(dims, ndim);
  const int j0b = blockIdx.x * 64, i0b = blockIdx.y * 64;
  if (j0b >= n) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = i0b + (wave >> 1) * 32, j0 = j0b + (wave & 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int ra0 = i0 + l16, ra1 = i0 + 16 + l16;
  const bool vra0 = ra0 < K, vra1 = ra1 < K;
  const bool vc0 = j0 + l16 < n, vc1 = j0 + 16 + l16 < n;
  for (int k0 = 0; k0 < kk; k0 += 4) {
    const int kq = k0 + l4;
    const bool vk = kq < kk;
    const double x0 = (vk && vra0) ? A[(long long)ra0 * lda + kq] : 0.0;
    const double x1 = (vk && vra1) ? A[(long long)ra1 * lda + kq] : 0.0;
    const double y0 = (vk && vc0) ? B[(long long)kq * ldb + j0 + l16] : 0.0;
    const double y1 = (vk && vc1) ? B[(long long)kq * ldb + j0 + 16 + l16] : 0.0;
    acc[0][0] = mfma16(x0, y0, acc[0][0]);
    acc[0][1] = mfma16(x0, y1, acc[0][1]);
    acc[1][0] = mfma16(x1, y0, acc[1][0]);
    acc[1][1] = mfma16(x1, y1, acc[1][1]);
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * p + l4 + 4 * r;
        const int j = j0 + 16 * q + l16;
        if (i < K && j < n) C[(long long)i * ldc + j] = acc[p][q][r];
      }
}

void gemm_tall(int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
               DimExpr kdim, DimExpr ndim, int kcap, int ncap, const int* dims, hipStream_t s) {
  (void)kcap;
  dim3 grid((ncap + 63) / 64, (K + 63) / 64);
  k_gemm_tall<<<grid, 256, 0, s>>>(K, A, lda, B, ldb, C, ldc, kdim, ndim, dims);
}

}  // namespace tt
