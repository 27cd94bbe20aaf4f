// One 64 x 64 tile of an FP64 product C = op(A) op(B) on a 256-thread block
// (FP64 MFMA), shared by the generic GEMM kernel and the divide-and-conquer
// merge products.  op(A) is m x k, op(B) is k x n; TA / TB
// select the transposed reads (A[l][i] / B[j][l]).  Thread (ty, tx) =
// (tid / 16, tid % 16) accumulates rows i0 + ty + 16 r, columns j0 + tx + 16 c.
#pragma once
#include <hip/hip_runtime.h>

namespace tt {

constexpr int GEMM_GK = 32;  // K slab depth staged in LDS

// One K slab of the operands into registers (NL values of A and of B per
// thread), zero outside the matrices.
template <int TA, int TB, int GK, int NL>
__device__ __forceinline__ void gemm_slab_load(double (&ra)[NL], double (&rb)[NL], const double* A,
                                               const double* B, int lda, int ldb,
                                               const double* kscale, int i0, int j0, int m, int n,
                                               int k, int l0, int tid) {
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + 256 * q;
    int i, l;
    if (TA == 0) { i = e / GK; l = e % GK; } else { l = e >> 6; i = e & 63; }
    const int gi = i0 + i, gl = l0 + l;
    double v = 0.0;
    if (gi < m && gl < k) {
      v = TA == 0 ? A[(long long)gi * lda + gl] : A[(long long)gl * lda + gi];
      if (kscale) v *= kscale[gl];
    }
    ra[q] = v;
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + 256 * q;
    int j, l;
    if (TB == 0) { l = e >> 6; j = e & 63; } else { j = e / GK; l = e % GK; }
    const int gj = j0 + j, gl = l0 + l;
    double v = 0.0;
    if (gj < n && gl < k) v = TB == 0 ? B[(long long)gl * ldb + gj] : B[(long long)gj * ldb + gl];
    rb[q] = v;
  }
}

typedef double gemm_f64x4 __attribute__((ext_vector_type(4)));

// acc = op(A) op(B) over the tile (i0, j0), with op(A)'s columns scaled by
// kscale when given.  32-deep K slabs go through LDS (As, Bs: GEMM_GK x 65,
// As[l][i] = op(A)[i0 + i][l0 + l], Bs[l][j] = op(B)[l0 + l][j0 + j]); the
// next slab's global loads are issued into registers before the current
// slab's products, so their latency is covered.  The products run on FP64
// MFMA 16x16x4: wavefront w owns rows 16 w .. 16 w + 15 of the tile, four
// 16x16 blocks side by side; lane l feeds A[16 w + l % 16][k + l / 16] and
// B[k + l / 16][16 c + l % 16], and item r of block c's accumulator holds
// C[16 w + l / 16 + 4 r][16 c + l % 16].  At the end the accumulators go
// through LDS (rows 0..31 in As, 32..63 in Bs) into the layout the callers
// read: thread (ty, tx) = (tid / 16, tid % 16) gets rows ty + 16 r, columns
// tx + 16 c.  Every thread of the block must call it (it holds block
// barriers).
template <int TA, int TB>
__device__ __forceinline__ void gemm_tile_acc(double (&acc)[4][4], const double* A, const double* B,
                                              int lda, int ldb, const double* kscale, int i0, int j0,
                                              int m, int n, int k, double (*As)[65],
                                              double (*Bs)[65]) {
  constexpr int GK = GEMM_GK, NL = GK * 64 / 256;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lk = lane >> 4;
  gemm_f64x4 c4[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) c4[c] = gemm_f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[NL], rb[NL];
  gemm_slab_load<TA, TB, GK, NL>(ra, rb, A, B, lda, ldb, kscale, i0, j0, m, n, k, 0, tid);
  for (int l0 = 0; l0 < k; l0 += GK) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + 256 * q;
      if (TA == 0) As[e % GK][e / GK] = ra[q];
      else As[e >> 6][e & 63] = ra[q];
      if (TB == 0) Bs[e >> 6][e & 63] = rb[q];
      else Bs[e % GK][e / GK] = rb[q];
    }
    __syncthreads();
    if (l0 + GK < k)
      gemm_slab_load<TA, TB, GK, NL>(ra, rb, A, B, lda, ldb, kscale, i0, j0, m, n, k, l0 + GK, tid);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const double a = As[kk + lk][16 * w + lr];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        c4[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[kk + lk][16 * c + lr], c4[c], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulators to the (ty, tx) layout through LDS
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * w + lk + 4 * r;
      (i < 32 ? As[i] : Bs[i - 32])[16 * c + lr] = c4[c][r];
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ty + 16 * r;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = (i < 32 ? As[i] : Bs[i - 32])[tx + 16 * c];
  }
  __syncthreads();  // the staging rows are free for the next tile
}

}  // namespace tt
