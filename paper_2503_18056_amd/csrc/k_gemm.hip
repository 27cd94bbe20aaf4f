// Dense FP64 contractions: a generic LDS-tiled GEMM for the rank-sized
// products, and MFMA kernels for the two N_s-long contractions of the step:
// the left Gram of the spatial core (G = X_cat^T X_cat, App. A.2 G_A = A^T A)
// and the spatial core update (X' = X_cat P, App. A.2 A' = A V_A S_A^-1 U).
#include "tt_internal.h"
#include "gemm_tile.h"

namespace tt {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// row-slice Gram (k_gram_rows) shape
constexpr int GR_CH = 16;     // rows per LDS chunk
constexpr int GR_MAXN = 384;  // columns held per LDS row
constexpr int GR_LD = 400;    // LDS row stride: row groups r and r+1 fall in opposite bank halves
// waves per block and 32x32 tasks per wave and pass: FP64 sixteen waves of
// one task (four waves a SIMD, held in registers without spilling); FP32 (the
// sliced products need more registers per task) eight waves of two
template <typename T> struct GrShape;
template <> struct GrShape<double> { static constexpr int WAVES = 16, TPW = 1; };
template <> struct GrShape<float> { static constexpr int WAVES = 8, TPW = 2; };


// Generic GEMM (vector FP64, 64x64 tiles, 32-deep K slabs staged in LDS,
// the next slab prefetched into registers).
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gemm(GemmDesc g, const int* __restrict__ dims) {
  if (g.cond_idx >= 0 && dims[g.cond_idx] != g.cond_val) return;
  const int z = blockIdx.z;
  const int bidx = g.bclip_idx;
  int m = eval_dim(dims, g.m), n = eval_dim(dims, g.n), k = eval_dim(dims, g.k);
  const long long coff = (long long)z * g.sC;
  if (bidx >= 0) {
    const int lim = dims[bidx] - z * g.bclip_mul;
    if (lim <= g.bclip_min) return;
    m = min(m, lim);
    n = min(n, lim);
    k = min(k, lim);
  }
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  if (i0 >= m || j0 >= n) return;
  const double* A = g.A + (long long)z * g.sA;
  const double* B = g.B + (long long)z * g.sB;
  double* C = g.C + coff;
  const double* kscale = g.kscale;
  if (g.ksplit > 0) {
    const long long k0 = (long long)z * g.ksplit;
    k = (int)max(0LL, min((long long)g.ksplit, (long long)k - k0));
    A = g.A + (TA == 0 ? k0 : k0 * g.lda);
    B = g.B + (TB == 0 ? k0 * g.ldb : k0);
    if (kscale) kscale += k0;
  }
  __shared__ double As[GEMM_GK][65];
  __shared__ double Bs[GEMM_GK][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
  gemm_tile_acc<TA, TB>(acc, A, B, g.lda, g.ldb, kscale, i0, j0, m, n, k, As, Bs);
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
                               DimExpr ndim, const int* __restrict__ dims, double beta) {
  const int m = eval_dim(dims, mdim), n = eval_dim(dims, ndim);
  const long long tot = (long long)m * n;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e % n);
    double acc = 0.0;
    for (int z = 0; z < nz; ++z) acc += part[z * zstride + (long long)i * ldp + j];
    double* o = out + (long long)i * ldo + j;
    *o = beta == 0.0 ? acc : acc + beta * *o;
  }
}

void sum_partials(const double* part, long long zstride, int nz, double* out, int ldo, int ldp,
                  DimExpr m, DimExpr n, int mcap, int ncap, const int* dims, hipStream_t s,
                  double beta) {
  long long tot = (long long)mcap * ncap;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_sum_partials<<<blocks, 256, 0, s>>>(part, zstride, nz, out, ldo, ldp, m, n, dims, beta);
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

// Wide Gram (more than 384 columns, FP64): partial[slice][pair] =
// A[rows of slice, tile ti]^T A[rows, tile tj] for the upper 128 x 128 tile
// pairs (ti <= tj).  Rows stream through LDS in stages of GW_KB rows (double
// buffered: the next stage is loaded into registers while the current one
// feeds the MFMAs); each of the four waves owns a 64 x 64 quarter, sixteen
// independent 16 x 16 accumulators.  16 x 16 blocks wholly past n are
// skipped.  A diagonal pair forms only its 36 upper 16 x 16 blocks (block row
// p, block column q >= p), dealt to the waves by block rows {w, 7 - w}, nine
// each.  When the last live tile holds at most 16 columns, the diagonal pair
// (t, t) also forms tile t against those columns as a ninth block column
// (eleven blocks per wave), and the pair (t, last) is skipped: it would
// stream all of tile t's rows again for one narrow block.  XCD-aware order:
// consecutive blocks go to consecutive XCDs, and all tile pairs of one row
// slice go to the same XCD, so the rows they share are fetched into one L2.
constexpr int GW_T = 128;
constexpr int GW_KB = 16;
constexpr int GW_LD = 144;  // LDS row stride: rows r and r+1 fall in opposite bank halves
constexpr int GW_XCD = 8;

__device__ inline void gw_pair(int pair, int tiles, int& ti, int& tj) {
  int t = 0, rem = pair;
  while (rem >= tiles - t) { rem -= tiles - t; ++t; }
  ti = t;
  tj = t + rem;
}

__device__ inline int gw_pair_index(int ti, int tj, int tiles) {
  return ti * tiles - ti * (ti - 1) / 2 + (tj - ti);
}

// Diagonal tile pair (ti, ti) of k_gram_wide, wave W: block rows W and 7 - W,
// block columns q >= the row (q == 8: the folded thin columns).  Operands are
// read from LDS for every kk step whether or not a block is live, so the reads
// are issued ahead of the MFMAs; a block is formed when both its row and its
// column hold live columns.
template <int W, typename Load, typename Store>
__device__ __forceinline__ void gram_wide_diag_wave(int nt, bool fold, int nstage, int k_begin,
                                                    const double (*sA)[GW_KB][GW_LD],
                                                    const double (*sX)[GW_KB][16],
                                                    double* __restrict__ out,
                                                    double* __restrict__ outx,
                                                    const Load& load, const Store& store) {
  constexpr int P1 = W, P2 = 7 - W;
  const int lane = threadIdx.x & 63, col = lane & 15, kr = lane >> 4;
  auto live = [&](int p, int q) { return q == 8 ? fold : (16 * p < nt && 16 * q < nt); };
  f64x4 acc1[9 - P1], acc2[9 - P2];
#pragma unroll
  for (int m = 0; m < 9 - P1; ++m) acc1[m] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < 9 - P2; ++m) acc2[m] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) load(k_begin + (st + 1) * GW_KB);
    const double(*SA)[GW_LD] = sA[buf];
    const double(*SX)[16] = sX[buf];
#pragma unroll
    for (int kk = 0; kk < GW_KB; kk += 4) {
      const double fa1 = SA[kk + kr][16 * P1 + col];
      const double fa2 = SA[kk + kr][16 * P2 + col];
      double fb[9 - P1];
#pragma unroll
      for (int m = 0; m < 9 - P1; ++m)
        fb[m] = P1 + m == 8 ? SX[kk + kr][col] : SA[kk + kr][16 * (P1 + m) + col];
#pragma unroll
      for (int m = 0; m < 9 - P1; ++m)
        if (live(P1, P1 + m)) acc1[m] = mfma16(fa1, fb[m], acc1[m]);
#pragma unroll
      for (int m = 0; m < 9 - P2; ++m)
        if (live(P2, P2 + m)) acc2[m] = mfma16(fa2, fb[m + P2 - P1], acc2[m]);
    }
    if (st + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
  auto put = [&](int p, int q, const f64x4& a) {
    double* o = q == 8 ? outx : out;
    const int jj = (q == 8 ? 0 : 16 * q) + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) o[(16 * p + (lane >> 4) + 4 * r) * GW_T + jj] = a[r];
  };
#pragma unroll
  for (int m = 0; m < 9 - P1; ++m)
    if (live(P1, P1 + m)) put(P1, P1 + m, acc1[m]);
#pragma unroll
  for (int m = 0; m < 9 - P2; ++m)
    if (live(P2, P2 + m)) put(P2, P2 + m, acc2[m]);
}

// Diagonal tile pair (ti, ti) of k_gram_wide; with fold, also tile ti against
// the (at most 16) columns of the last live tile tl, written to pair (ti, tl)
// (outx).  Rows stream through LDS as in the off-diagonal pairs.
__device__ __forceinline__ void gram_wide_diag(const double* __restrict__ A, int lda, int n,
                                               int ti, int tl, bool fold, int k_begin, int k_end,
                                               double* __restrict__ out, double* __restrict__ outx,
                                               double (*sA)[GW_KB][GW_LD],
                                               double (*sX)[GW_KB][16]) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int ca = ti * GW_T, cx = tl * GW_T;
  const int nt = n - ca;  // live columns of the tile (all 128 unless it is the last)
  const int lc = tid & 127, lr = tid >> 7;
  const bool va = lc < nt;
  const int xr = tid >> 4, xc = tid & 15;  // thin columns: one element per thread
  const bool vx = fold && cx + xc < n;
  double ra[8], rx;
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = k0 + lr + 2 * u;
      ra[u] = (row < k_end && va) ? A[(long long)row * lda + ca + lc] : 0.0;
    }
    const int row = k0 + xr;
    rx = (row < k_end && vx) ? A[(long long)row * lda + cx + xc] : 0.0;
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) sA[buf][lr + 2 * u][lc] = ra[u];
    sX[buf][xr][xc] = rx;
  };
  const int nstage = (k_end - k_begin + GW_KB - 1) / GW_KB;
  if (nstage > 0) {
    load(k_begin);
    store(0);
  }
  __syncthreads();
  switch (wave) {
    case 0: gram_wide_diag_wave<0>(nt, fold, nstage, k_begin, sA, sX, out, outx, load, store); break;
    case 1: gram_wide_diag_wave<1>(nt, fold, nstage, k_begin, sA, sX, out, outx, load, store); break;
    case 2: gram_wide_diag_wave<2>(nt, fold, nstage, k_begin, sA, sX, out, outx, load, store); break;
    default: gram_wide_diag_wave<3>(nt, fold, nstage, k_begin, sA, sX, out, outx, load, store);
  }
}

__global__ __launch_bounds__(256) void k_gram_wide(const double* __restrict__ A, int lda, int K,
                                                   int kslice, int slices, DimExpr ndim,
                                                   const int* __restrict__ dims, int tiles,
                                                   int pairs, double* __restrict__ partial) {
  const int n = eval_dim(dims, ndim);
  const int x = blockIdx.x % GW_XCD, jx = blockIdx.x / GW_XCD;
  const int pair = jx % pairs, slice = x + GW_XCD * (jx / pairs);
  if (slice >= slices) return;
  int ti, tj;
  gw_pair(pair, tiles, ti, tj);
  if (ti * GW_T >= n || tj * GW_T >= n) return;
  // last live tile; when it holds at most 16 columns the diagonal pairs form
  // the products with it
  const int tl = (n - 1) / GW_T;
  const bool thin = tl > 0 && n - tl * GW_T <= 16;
  if (thin && tj == tl && ti < tl) return;
  const bool diag = ti == tj;
  __shared__ double sA[2][GW_KB][GW_LD], sB[2][GW_KB][GW_LD];
  const int k_begin = slice * kslice;
  const int k_end = min(K, k_begin + kslice);
  if (diag) {
    const bool fold = thin && ti < tl;
    double* out = partial + ((long long)slice * pairs + pair) * (GW_T * GW_T);
    double* outx =
        partial + ((long long)slice * pairs + gw_pair_index(ti, tl, tiles)) * (GW_T * GW_T);
    gram_wide_diag(A, lda, n, ti, tl, fold, k_begin, k_end, out, outx, sA,
                   reinterpret_cast<double(*)[GW_KB][16]>(&sB[0][0][0]));
    return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int ca = ti * GW_T, cb = tj * GW_T;
  // loads: thread t moves column t % 128 of rows t / 128 + 2u, u = 0..7
  const int lc = tid & 127, lr = tid >> 7;
  const bool va = ca + lc < n, vb = cb + lc < n;
  // valid 16 x 16 blocks of this wave
  const int a0 = wr * 64, b0 = wc * 64;
  int np = 0, nq = 0;
  for (int t = 0; t < 4; ++t) {
    if (ca + a0 + 16 * t < n) np = t + 1;
    if (cb + b0 + 16 * t < n) nq = t + 1;
  }
  f64x4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = k0 + lr + 2 * u;
      const bool vr = row < k_end;
      const double* rp = A + (long long)row * lda;
      ra[u] = (vr && va) ? rp[ca + lc] : 0.0;
      rb[u] = (vr && vb) ? rp[cb + lc] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sA[buf][lr + 2 * u][lc] = ra[u];
      sB[buf][lr + 2 * u][lc] = rb[u];
    }
  };
  const int nstage = (k_end - k_begin + GW_KB - 1) / GW_KB;
  if (nstage > 0) {
    load(k_begin);
    store(0);
  }
  __syncthreads();
  const int col = lane & 15, kr = lane >> 4;
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) load(k_begin + (st + 1) * GW_KB);
    const double(*SA)[GW_LD] = sA[buf];
    const double(*SB)[GW_LD] = sB[buf];
#pragma unroll
    for (int kk = 0; kk < GW_KB; kk += 4) {
      double fa[4], fb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fa[t] = SA[kk + kr][a0 + 16 * t + col];
        fb[t] = SB[kk + kr][b0 + 16 * t + col];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (p < np && q < nq) acc[p][q] = mfma16(fa[p], fb[q], acc[p][q]);
    }
    if (st + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
  double* out = partial + ((long long)slice * pairs + pair) * (GW_T * GW_T);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (p >= np || q >= nq) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = a0 + 16 * p + (lane >> 4) + 4 * r;
        const int jj = b0 + 16 * q + (lane & 15);
        out[ii * GW_T + jj] = acc[p][q][r];
      }
    }
}

// Fixed-order sum of the wide Gram's slices, mirrored into G.  Diagonal tiles
// take the upper triangle (ii <= jj) only: their blocks below the diagonal
// are not formed.
__global__ __launch_bounds__(256) void k_gram_wide_reduce(const double* __restrict__ partial,
                                                          int slices, int pairs, int tiles,
                                                          DimExpr ndim, const int* __restrict__ dims,
                                                          double* __restrict__ G, int ldg) {
  const int n = eval_dim(dims, ndim);
  const int pair = blockIdx.y;
  int ti, tj;
  gw_pair(pair, tiles, ti, tj);
  if (ti * GW_T >= n || tj * GW_T >= n) return;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < GW_T * GW_T; e += gridDim.x * 256) {
    const int ii = e / GW_T, jj = e % GW_T;
    const int i = ti * GW_T + ii, j = tj * GW_T + jj;
    if (i >= n || j >= n || (ti == tj && ii > jj)) continue;
    double sum = 0.0;
#pragma unroll 8
    for (int sl = 0; sl < slices; ++sl)
      sum += partial[((long long)sl * pairs + pair) * (GW_T * GW_T) + e];
    G[(long long)i * ldg + j] = sum;
    G[(long long)j * ldg + i] = sum;
  }
}

template <typename T>
__global__ void k_gram_rows(const T* __restrict__ A, int lda, int K, int rows_per_blk, DimExpr ndim,
                            const int* __restrict__ dims, const unsigned* __restrict__ colmax,
                            double* __restrict__ partial);
__global__ void k_gram_rows_reduce(const double* __restrict__ partial, int nblk, DimExpr ndim,
                                   const int* __restrict__ dims, double* __restrict__ G, int ldg);

GramPlan gram_plan(int K, int ncap, int lda) {
  GramPlan p;
  p.K = K;
  p.ncap = ncap;
  p.lda = lda;
  // row-slice form (LDS-staged) when the columns fit one LDS row
  p.rows_mode = ncap <= 384;
  const int t32 = (ncap + 31) / 32;
  p.ntask_cap = t32 * (t32 + 1) / 2;
  int nb = (K + 63) / 64;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  p.rows_per_blk = ((K + nb - 1) / nb + 15) / 16 * 16;
  p.nblk = (K + p.rows_per_blk - 1) / p.rows_per_blk;
  if (p.nblk < 1) p.nblk = 1;
  // wide form: 128-column tile pairs, a multiple of GW_XCD row slices of at
  // least 1024 rows (at most 64)
  p.wtiles = (ncap + GW_T - 1) / GW_T;
  p.wpairs = p.wtiles * (p.wtiles + 1) / 2;
  int ws = K / 1024;
  ws = ws < GW_XCD ? GW_XCD : (ws > 64 ? 64 : ws);
  ws = ws / GW_XCD * GW_XCD;
  p.wkslice = ((K + ws - 1) / ws + GW_KB - 1) / GW_KB * GW_KB;
  p.wslices = ws;
  return p;
}

size_t gram_partial_doubles(const GramPlan& p) {
  if (p.rows_mode) return (size_t)p.nblk * p.ntask_cap * 1024;
  return (size_t)p.wslices * p.wpairs * GW_T * GW_T;
}

void gram_tall_partial(const GramPlan& p, const double* A, DimExpr n, double* partial,
                       const int* dims, hipStream_t s) {
  if (p.rows_mode) {
    k_gram_rows<double><<<p.nblk, GrShape<double>::WAVES * 64, 0, s>>>(A, p.lda, p.K, p.rows_per_blk, n, dims, nullptr,
                                                partial);
    return;
  }
  k_gram_wide<<<p.wslices * p.wpairs, 256, 0, s>>>(A, p.lda, p.K, p.wkslice, p.wslices, n, dims,
                                                   p.wtiles, p.wpairs, partial);
}
void gram_tall_reduce(const GramPlan& p, DimExpr n, const double* partial, double* G, int ldg,
                      const int* dims, hipStream_t s) {
  if (p.rows_mode) {
    k_gram_rows_reduce<<<dim3(16, p.ntask_cap), 256, 0, s>>>(partial, p.nblk, n, dims, G, ldg);
    return;
  }
  k_gram_wide_reduce<<<dim3(8, p.wpairs), 256, 0, s>>>(partial, p.wslices, p.wpairs, p.wtiles, n,
                                                       dims, G, ldg);
}
void gram_split_reduce(const GramPlan& p, DimExpr n, const double* partial, double* G, int ldg,
                       const int* dims, hipStream_t s) {
  if (p.rows_mode) {
    k_gram_rows_reduce<<<dim3(16, p.ntask_cap), 256, 0, s>>>(partial, p.nblk, n, dims, G, ldg);
    return;
  }
  k_gram_wide_reduce<<<dim3(8, p.wpairs), 256, 0, s>>>(partial, p.wslices, p.wpairs, p.wtiles, n,
                                                       dims, G, ldg);
}
void gram_tall(const GramPlan& p, const double* A, DimExpr n, double* partial, double* G, int ldg,
               const int* dims, hipStream_t s) {
  gram_tall_partial(p, A, n, partial, dims, s);
  gram_tall_reduce(p, n, partial, G, ldg, dims, s);
}

// ---------------------------------------------------------------------------
// Tall GEMM C[K x n] = A[K x k] B[k x n] on MFMA: 128 x 128 output tile per block
// (a 128-row panel of A times all of B's columns when n <= 128, so A streams
// from HBM once), each wave a 64 x 64 quarter of sixteen 16 x 16
// accumulators.  A panels (128 rows x 16 k) and B chunks (16 k x 128 cols)
// are staged through LDS, double buffered.  The A panel's row stride of 17
// doubles puts the 16 rows an MFMA operand reads down one column in
// distinct banks; 16 x 16 output blocks wholly past K or n are skipped.
constexpr int GP_KB = 16;
constexpr int GP_LDA = 17;
constexpr int GP_LDB = 144;

__global__ __launch_bounds__(256) void k_gemm_panel(int K, const double* __restrict__ A, int lda,
                                                    const double* __restrict__ B, int ldb,
                                                    double* __restrict__ C, int ldc,
                                                    DimExpr kdim, DimExpr ndim,
                                                    const int* __restrict__ dims) {
  const int kk_tot = eval_dim(dims, kdim), n = eval_dim(dims, ndim);
  const int r0 = blockIdx.x * 128, c0 = blockIdx.y * 128;
  if (c0 >= n) return;
  __shared__ double sA[2][128][GP_LDA], sB[2][GP_KB][GP_LDB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int a0 = wr * 64, b0 = wc * 64;
  int np = 0, nq = 0;
  for (int t = 0; t < 4; ++t) {
    if (r0 + a0 + 16 * t < K) np = t + 1;
    if (c0 + b0 + 16 * t < n) nq = t + 1;
  }
  // loads: A panel, thread t -> row t / 2, k (t % 2) * 8 .. +8;
  //        B chunk, thread t -> k t / 16, columns (t % 16) * 8 .. +8
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bc = (tid & 15) * 8;
  const bool var = r0 + ar < K;
  const double* arow = A + (long long)(r0 + ar) * lda;
  double ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + ak + u;
      ra[u] = (var && k < kk_tot) ? arow[k] : 0.0;
      const int kb = k0 + bk, cb = c0 + bc + u;
      rb[u] = (kb < kk_tot && cb < n) ? B[(long long)kb * ldb + cb] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sA[buf][ar][ak + u] = ra[u];
      sB[buf][bk][bc + u] = rb[u];
    }
  };
  f64x4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nstage = (kk_tot + GP_KB - 1) / GP_KB;
  if (nstage > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int col = lane & 15, kr = lane >> 4;
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) load((st + 1) * GP_KB);
#pragma unroll
    for (int kk = 0; kk < GP_KB; kk += 4) {
      double fa[4], fb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fa[t] = sA[buf][a0 + 16 * t + col][kk + kr];
        fb[t] = sB[buf][kk + kr][b0 + 16 * t + col];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (p < np && q < nq) acc[p][q] = mfma16(fa[p], fb[q], acc[p][q]);
    }
    if (st + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (p >= np || q >= nq) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + a0 + 16 * p + (lane >> 4) + 4 * r;
        const int j = c0 + b0 + 16 * q + (lane & 15);
        if (i < K && j < n) C[(long long)i * ldc + j] = acc[p][q][r];
      }
    }
}

// ===========================================================================
// FP32-mixed precision form: the N_s-long contractions on FP32 MFMA.
typedef float f32x4 __attribute__((ext_vector_type(4)));
// D = A B + C for A 16x4, B 4x16 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; item r of lane l is D[4 (l/16) + r][l%16]).
__device__ inline f32x4 mfma16f(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Exponent E with |x| < 2^E for every entry of a column, from the bit
// pattern of its largest magnitude (0 for a zero column).
__device__ inline int col_exponent(unsigned bits) {
  const float m = __uint_as_float(bits);
  return m > 0.0f ? ilogbf(m) + 1 : 0;
}

// Error-free split of x (|x| < 2^E) into S integer slices of 11 bits:
// x = 2^E (s0 2^-11 + s1 2^-22 + ... + s_{S-1} 2^-11S) + remainder below
// 2^(E-11S-1); |s0| <= 2^11, |s1..| <= 2^10.  Every step is exact in FP32.
template <int S>
__device__ inline void split_slices(float x, int E, float s[S]) {
  float t = ldexpf(x, 11 - E);
#pragma unroll
  for (int q = 0; q < S; ++q) {
    s[q] = rintf(t);
    t = (t - s[q]) * 2048.0f;
  }
}

// acc += sum over slice pairs (a, b) with a + b = L < S of x_a y_b
// 2^-11 (L + 2), on FP32 MFMA 16x16x4.  Per level L the pairs (0, L) and
// (L, 0) share one accumulator and the pairs with both indices >= 1 (at
// most four for S <= 6) a second: four rows of products of at most 2^21
// (resp. 2^20) keep every partial an integer below 2^24, exact in FP32.
// Each level's two partials are added in FP64 and flushed at its scale.
template <int S>
__device__ inline void sliced_products(const float* xv, const float* yv, f64x4& acc) {
  static_assert(S >= 1 && S <= 6, "slice count");
  const f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int L = 0; L < S; ++L) {
    const f32x4 ga = L == 0 ? mfma16f(xv[0], yv[0], z) : mfma16f(xv[L], yv[0], mfma16f(xv[0], yv[L], z));
    f32x4 gb = z;
#pragma unroll
    for (int a = 1; a < L; ++a) gb = mfma16f(xv[a], yv[L - a], gb);
    const double sc = L == 0 ? 0x1p-22 : L == 1 ? 0x1p-33 : L == 2 ? 0x1p-44
                    : L == 3 ? 0x1p-55 : L == 4 ? 0x1p-66 : 0x1p-77;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc[r] = fma(L >= 2 ? (double)ga[r] + (double)gb[r] : (double)ga[r], sc, acc[r]);
  }
}

// Gram G = A^T A of an FP32 matrix on FP32 MFMA, exact to 2^-11S of each
// column's largest entry (Ozaki-style error-free splitting; S = 4 slices by
// default, 1 .. 6 selectable), for more than 384 columns.  Each entry is
// split on a per-column exponent grid into S 11-bit integer slices; the
// slice pairs (s, t), counted from 0, with s + t < S are multiplied on MFMA
// four rows at a time (sliced_products), where every partial sum is an
// integer of at most 2^24 and so exact in FP32; each exact partial is
// flushed into FP64.  Blocking, staging and block order as
// k_gram_wide (128 x 128 tile pairs, 16-row stages through LDS, each wave a
// 64 x 64 quarter); output in k_gram_wide's partial layout, scaled back by
// the column exponents, for k_gram_wide_reduce.
template <int S>
__global__ __launch_bounds__(256) void k_gram_split_wide(const float* __restrict__ A, int lda,
                                                         int K, int kslice, int slices,
                                                         DimExpr ndim, const int* __restrict__ dims,
                                                         int tiles, int pairs,
                                                         const unsigned* __restrict__ colmax,
                                                         double* __restrict__ partial) {
  const int n = eval_dim(dims, ndim);
  const int x = blockIdx.x % GW_XCD, jx = blockIdx.x / GW_XCD;
  const int pair = jx % pairs, slice = x + GW_XCD * (jx / pairs);
  if (slice >= slices) return;
  int ti, tj;
  gw_pair(pair, tiles, ti, tj);
  if (ti * GW_T >= n || tj * GW_T >= n) return;
  const bool diag = ti == tj;
  __shared__ float sA[2][GW_KB][GW_LD], sB[2][GW_KB][GW_LD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const bool idle = diag && wr > wc;
  const int ca = ti * GW_T, cb = tj * GW_T;
  const int lc = tid & 127, lr = tid >> 7;
  const bool va = ca + lc < n, vb = cb + lc < n;
  const int k_begin = slice * kslice;
  const int k_end = min(K, k_begin + kslice);
  const int a0 = wr * 64, b0 = wc * 64;
  const int col = lane & 15, kr = lane >> 4;
  int np = 0, nq = 0;
  int ea[4], eb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (ca + a0 + 16 * t < n) np = t + 1;
    if (cb + b0 + 16 * t < n) nq = t + 1;
    const int xa = ca + a0 + 16 * t + col, xb = cb + b0 + 16 * t + col;
    ea[t] = xa < n ? col_exponent(colmax[xa]) : 0;
    eb[t] = xb < n ? col_exponent(colmax[xb]) : 0;
  }
  if (idle) np = nq = 0;
  f64x4 acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  float ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = k0 + lr + 2 * u;
      const bool vr = row < k_end;
      const float* rp = A + (long long)row * lda;
      ra[u] = (vr && va) ? rp[ca + lc] : 0.0f;
      rb[u] = (vr && vb && !diag) ? rp[cb + lc] : 0.0f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sA[buf][lr + 2 * u][lc] = ra[u];
      if (!diag) sB[buf][lr + 2 * u][lc] = rb[u];
    }
  };
  const int nstage = (k_end - k_begin + GW_KB - 1) / GW_KB;
  if (nstage > 0) {
    load(k_begin);
    store(0);
  }
  __syncthreads();
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) load(k_begin + (st + 1) * GW_KB);
    const float(*SA)[GW_LD] = sA[buf];
    const float(*SB)[GW_LD] = diag ? sA[buf] : sB[buf];
    for (int kk = 0; kk < GW_KB; kk += 4) {
      float xs[4][S], ys[4][S];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        split_slices<S>(SA[kk + kr][a0 + 16 * t + col], ea[t], xs[t]);
        split_slices<S>(SB[kk + kr][b0 + 16 * t + col], eb[t], ys[t]);
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (p >= np || q >= nq) continue;
          sliced_products<S>(xs[p], ys[q], acc[p][q]);
        }
    }
    if (st + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
  double* out = partial + ((long long)slice * pairs + pair) * (GW_T * GW_T);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (p >= np || q >= nq) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // FP32 MFMA item r of lane l: row 4 (l / 16) + r, column l % 16
        const int ii = a0 + 16 * p + 4 * (lane >> 4) + r;
        const int jj = b0 + 16 * q + (lane & 15);
        const int gi = ca + ii, gj = cb + jj;
        const int e = (gi < n ? col_exponent(colmax[gi]) : 0) + (gj < n ? col_exponent(colmax[gj]) : 0);
        out[ii * GW_T + jj] = ldexp(acc[p][q][r], e);
      }
    }
}

// colmax[c] = bits of max_i |A[i][c]| over i < K, c < n (FP32 A, row-major);
// colmax must be zero on entry.  Non-negative floats order like their bits.
__global__ __launch_bounds__(256) void k_colmax(const float* __restrict__ A, int lda, int K,
                                                DimExpr ndim, const int* __restrict__ dims,
                                                unsigned* __restrict__ colmax) {
  const int n = eval_dim(dims, ndim);
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  if (c >= n) return;
  const int r0 = blockIdx.y * 256 + (threadIdx.x >> 6);
  unsigned m = 0;
  for (int i = r0; i < K && i < blockIdx.y * 256 + 256; i += 4)
    m = max(m, __float_as_uint(fabsf(A[(long long)i * lda + c])));
  atomicMax(colmax + c, m);
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// C[K x n] (FP32) = A[K x k] (FP32) B[k x n] (FP64) on FP32 MFMA with B
// split into FP32 hi + lo parts (separate accumulators); every four-term
// partial is flushed into FP64, and C is rounded to FP32 once at the end.
__global__ __launch_bounds__(256) void k_gemm_tall_f32(int K, const float* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb,
                                                       float* __restrict__ C, int ldc,
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
  const f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < kk; k0 += 4) {
    const int kq = k0 + l4;
    const bool vk = kq < kk;
    const float x[2] = {(vk && vra0) ? A[(long long)ra0 * lda + kq] : 0.0f,
                        (vk && vra1) ? A[(long long)ra1 * lda + kq] : 0.0f};
    const double b0d = (vk && vc0) ? B[(long long)kq * ldb + j0 + l16] : 0.0;
    const double b1d = (vk && vc1) ? B[(long long)kq * ldb + j0 + 16 + l16] : 0.0;
    const float bh[2] = {(float)b0d, (float)b1d};
    const float bl[2] = {(float)(b0d - (double)bh[0]), (float)(b1d - (double)bh[1])};
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const f32x4 hi = mfma16f(x[p], bh[q], z);
        const f32x4 lo = mfma16f(x[p], bl[q], z);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[p][q][r] += (double)hi[r] + (double)lo[r];
      }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * p + 4 * l4 + r;
        const int j = j0 + 16 * q + l16;
        if (i < K && j < n) C[(long long)i * ldc + j] = (float)acc[p][q][r];
      }
}

// ---------------------------------------------------------------------------
// Row-slice Gram: each block owns a contiguous slice of rows, stages it
// through LDS in chunks of GR_CH rows (the next chunk is loaded into
// registers while the current one is multiplied), and computes every
// upper-triangular 32x32 output task of the slice from LDS, two tasks per
// wavefront per pass, eight wavefronts per block (more passes re-stage the
// slice).  A is read from HBM
// once; each block writes its slice's partial Gram (tasks x 1024 doubles),
// reduced in a fixed order by k_gram_rows_reduce.  T = double: FP64 MFMA;
// T = float: the sliced error-free products of k_gram_split_wide.

__device__ inline void gr_task(int t, int& ti, int& tj, int T32) {
  int a = 0, rem = t;
  while (rem >= T32 - a) { rem -= T32 - a; ++a; }
  ti = a;
  tj = a + rem;
}

template <typename T, int S>
__device__ __forceinline__ void gram_rows_body(const T* __restrict__ A, int lda, int K,
                                                    int rows_per_blk, DimExpr ndim,
                                                    const int* __restrict__ dims,
                                                    const unsigned* __restrict__ colmax,
                                                    double* __restrict__ partial) {
  constexpr int GR_WAVES = GrShape<T>::WAVES, GR_TPW = GrShape<T>::TPW, GR_THREADS = GR_WAVES * 64;
  const int n = eval_dim(dims, ndim);
  const int T32 = (n + 31) / 32, ntask = T32 * (T32 + 1) / 2;
  const int k_begin = blockIdx.x * rows_per_blk;
  const int k_end = min(K, k_begin + rows_per_blk);
  __shared__ T lds[GR_CH][GR_LD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = lane & 15, krow = lane >> 4;
  const int nld = GR_CH * n;  // elements staged per chunk
  constexpr int PER = (GR_CH * GR_MAXN + GR_THREADS - 1) / GR_THREADS;
  for (int pass = 0; pass * GR_WAVES * GR_TPW < ntask; ++pass) {
    int tI[GR_TPW], tJ[GR_TPW];
    bool act[GR_TPW];
    // 16 x 16 blocks (a, b) of a task that hold entries: the second block
    // row / column only when it starts below n, and not the lower-left block
    // of a diagonal task (the transpose of its upper-right one)
    bool ok01[GR_TPW], ok10[GR_TPW], ok11[GR_TPW];
    int ea[GR_TPW][2], eb[GR_TPW][2];
#pragma unroll
    for (int q = 0; q < GR_TPW; ++q) {
      const int t = (pass * GR_TPW + q) * GR_WAVES + wave;
      act[q] = t < ntask;
      tI[q] = tJ[q] = 0;
      if (act[q]) gr_task(t, tI[q], tJ[q], T32);
      ok01[q] = tJ[q] * 32 + 16 < n;
      ok10[q] = tI[q] * 32 + 16 < n && tI[q] != tJ[q];
      ok11[q] = tI[q] * 32 + 16 < n && tJ[q] * 32 + 16 < n;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ca = tI[q] * 32 + 16 * h + col, cb = tJ[q] * 32 + 16 * h + col;
        ea[q][h] = (sizeof(T) == 4 && act[q] && ca < n) ? col_exponent(colmax[ca]) : 0;
        eb[q][h] = (sizeof(T) == 4 && act[q] && cb < n) ? col_exponent(colmax[cb]) : 0;
      }
    }
    f64x4 acc[GR_TPW][2][2];
#pragma unroll
    for (int q = 0; q < GR_TPW; ++q)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[q][a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // prefetch the first chunk
    T nxt[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * GR_THREADS;
      const int r = e / max(n, 1), c = e - r * max(n, 1);
      const int row = k_begin + r;
      nxt[u] = (e < nld && row < k_end) ? A[(long long)row * lda + c] : T(0);
    }
    for (int k0 = k_begin; k0 < k_end; k0 += GR_CH) {
      __syncthreads();  // the previous chunk is no longer read
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = tid + u * GR_THREADS;
        if (e < nld) {
          const int r = e / n, c = e - r * n;
          lds[r][c] = nxt[u];
        }
      }
      __syncthreads();
      // load the next chunk while this one is multiplied
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = tid + u * GR_THREADS;
        const int r = e / max(n, 1), c = e - r * max(n, 1);
        const int row = k0 + GR_CH + r;
        nxt[u] = (e < nld && row < k_end) ? A[(long long)row * lda + c] : T(0);
      }
#pragma unroll
      for (int q = 0; q < GR_TPW; ++q) {
        if (!act[q]) continue;
        const int ca = tI[q] * 32 + col, cb = tJ[q] * 32 + col;
#pragma unroll(sizeof(T) == 8 ? 4 : 1)
        for (int kk = 0; kk < GR_CH; kk += 4) {
          const int r = kk + krow;
          const T x0 = ca < n ? lds[r][ca] : T(0), x1 = ca + 16 < n ? lds[r][ca + 16] : T(0);
          const T y0 = cb < n ? lds[r][cb] : T(0), y1 = cb + 16 < n ? lds[r][cb + 16] : T(0);
          if constexpr (sizeof(T) == 8) {
            acc[q][0][0] = mfma16(x0, y0, acc[q][0][0]);
            if (ok01[q]) acc[q][0][1] = mfma16(x0, y1, acc[q][0][1]);
            if (ok10[q]) acc[q][1][0] = mfma16(x1, y0, acc[q][1][0]);
            if (ok11[q]) acc[q][1][1] = mfma16(x1, y1, acc[q][1][1]);
          } else {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              float xv[S];
              split_slices<S>(a == 0 ? x0 : x1, ea[q][a], xv);
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                if ((a == 0 && b == 1 && !ok01[q]) || (a == 1 && b == 0 && !ok10[q]) ||
                    (a == 1 && b == 1 && !ok11[q]))
                  continue;
                float yv[S];
                split_slices<S>(b == 0 ? y0 : y1, eb[q][b], yv);
                sliced_products<S>(xv, yv, acc[q][a][b]);
              }
            }
          }
        }
      }
    }
    // write this block's partial tasks
#pragma unroll
    for (int q = 0; q < GR_TPW; ++q) {
      if (!act[q]) continue;
      const int t = (pass * GR_TPW + q) * GR_WAVES + wave;
      double* out = partial + ((long long)blockIdx.x * ntask + t) * 1024;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            // FP64 MFMA item rr of lane l: row l/16 + 4 rr; FP32: row 4 (l/16) + rr
            const int ii = 16 * a + (sizeof(T) == 8 ? (lane >> 4) + 4 * rr : 4 * (lane >> 4) + rr);
            const int jj = 16 * b + (lane & 15);
            double v = acc[q][a][b][rr];
            if (sizeof(T) == 4) {
              const int ga = tI[q] * 32 + ii, gb = tJ[q] * 32 + jj;
              const int e = (ga < n ? col_exponent(colmax[ga]) : 0) + (gb < n ? col_exponent(colmax[gb]) : 0);
              v = ldexp(v, e);
            }
            out[ii * 32 + jj] = v;
          }
    }
  }
}

// FP64 form (MFMA 16x16x4 f64).
template <typename T>
__global__ __launch_bounds__(GrShape<T>::WAVES * 64) __attribute__((amdgpu_waves_per_eu(GrShape<T>::WAVES / 4, GrShape<T>::WAVES / 4))) void k_gram_rows(const T* __restrict__ A, int lda, int K,
                                                    int rows_per_blk, DimExpr ndim,
                                                    const int* __restrict__ dims,
                                                    const unsigned* __restrict__ colmax,
                                                    double* __restrict__ partial) {
  gram_rows_body<T, 1>(A, lda, K, rows_per_blk, ndim, dims, colmax, partial);
}

// FP32-mixed form: S 11-bit slices per entry (sliced_products).
template <int S>
__global__ __launch_bounds__(GrShape<float>::WAVES * 64) __attribute__((amdgpu_waves_per_eu(GrShape<float>::WAVES / 4, GrShape<float>::WAVES / 4))) void k_gram_rows_f32(const float* __restrict__ A, int lda, int K,
                                                    int rows_per_blk, DimExpr ndim,
                                                    const int* __restrict__ dims,
                                                    const unsigned* __restrict__ colmax,
                                                    double* __restrict__ partial) {
  gram_rows_body<float, S>(A, lda, K, rows_per_blk, ndim, dims, colmax, partial);
}

// G[a][b] = G[b][a] = sum over blocks of the partial tasks, in a fixed
// order: four thread groups sum the blocks b = g (mod 4) for 64 elements,
// then the four group sums are added in order (diagonal tasks from their
// upper triangle).
__global__ __launch_bounds__(256) void k_gram_rows_reduce(const double* __restrict__ partial,
                                                          int nblk, DimExpr ndim,
                                                          const int* __restrict__ dims,
                                                          double* __restrict__ G, int ldg) {
  const int n = eval_dim(dims, ndim);
  const int T32 = (n + 31) / 32, ntask = T32 * (T32 + 1) / 2;
  const int t = blockIdx.y;
  if (t >= ntask) return;
  int ti, tj;
  gr_task(t, ti, tj, T32);
  __shared__ double part[4][64];
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  // unrolled so that eight partial loads are in flight; the sum keeps its order
  double s = 0.0;
#pragma unroll 8
  for (int b = g; b < nblk; b += 4) s += partial[((long long)b * ntask + t) * 1024 + e];
  part[g][el] = s;
  __syncthreads();
  if (g != 0) return;
  const double v = ((part[0][el] + part[1][el]) + part[2][el]) + part[3][el];
  const int ii = e >> 5, jj = e & 31;
  const int i = ti * 32 + ii, j = tj * 32 + jj;
  // a diagonal tile's lower-left 16 x 16 block is not formed: its upper
  // triangle gives both halves
  if (i >= n || j >= n || (ti == tj && ii > jj)) return;
  G[(long long)i * ldg + j] = v;
  G[(long long)j * ldg + i] = v;
}

template <int S>
static void gram_split_launch(const GramPlan& p, const float* A, DimExpr n, const unsigned* colmax,
                              double* partial, const int* dims, hipStream_t s) {
  if (p.rows_mode)
    k_gram_rows_f32<S><<<p.nblk, GrShape<float>::WAVES * 64, 0, s>>>(A, p.lda, p.K, p.rows_per_blk, n,
                                                                        dims, colmax, partial);
  else
    k_gram_split_wide<S><<<p.wslices * p.wpairs, 256, 0, s>>>(A, p.lda, p.K, p.wkslice, p.wslices, n,
                                                              dims, p.wtiles, p.wpairs, colmax, partial);
}

void gram_split_partial(const GramPlan& p, const float* A, DimExpr n, unsigned* colmax,
                        double* partial, const int* dims, hipStream_t s, int slices) {
  k_zero_u32<<<(p.ncap + 255) / 256, 256, 0, s>>>(colmax, p.ncap);
  k_colmax<<<dim3((p.ncap + 63) / 64, (p.K + 255) / 256), 256, 0, s>>>(A, p.lda, p.K, n, dims,
                                                                       colmax);
  switch (slices) {
    case 1: gram_split_launch<1>(p, A, n, colmax, partial, dims, s); break;
    case 2: gram_split_launch<2>(p, A, n, colmax, partial, dims, s); break;
    case 3: gram_split_launch<3>(p, A, n, colmax, partial, dims, s); break;
    case 5: gram_split_launch<5>(p, A, n, colmax, partial, dims, s); break;
    case 6: gram_split_launch<6>(p, A, n, colmax, partial, dims, s); break;
    default: gram_split_launch<4>(p, A, n, colmax, partial, dims, s); break;
  }
}

void gemm_tall_f32(int K, const float* A, int lda, const double* B, int ldb, float* C, int ldc,
                   DimExpr kdim, DimExpr ndim, int ncap, const int* dims, hipStream_t s) {
  dim3 grid((ncap + 63) / 64, (K + 63) / 64);
  k_gemm_tall_f32<<<grid, 256, 0, s>>>(K, A, lda, B, ldb, C, ldc, kdim, ndim, dims);
}

void gemm_tall(int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
               DimExpr kdim, DimExpr ndim, int kcap, int ncap, const int* dims, hipStream_t s) {
  (void)kcap;
  k_gemm_panel<<<dim3((K + 127) / 128, (ncap + 127) / 128), 256, 0, s>>>(K, A, lda, B, ldb, C, ldc,
                                                                         kdim, ndim, dims);
}

}  // namespace tt
