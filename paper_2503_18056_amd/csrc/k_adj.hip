// Adjoint (reverse-mode) kernels of one step with frozen ranks: the pieces of
// the reverse sweep that are not plain GEMMs.  The step being differentiated
// is the upwind transport in TT form (Sec. 3.1, Sec. 4.3), absorption /
// emission with a frozen temperature (Sec. 3.2, Sec. 4.4), the TT sum by
// concatenation (Sec. 4.1) and the Gram-SVD truncation of both bonds (App. A,
// Algorithm 1; App. A.2).  The truncation is differentiated as a truncated
// SVD, by the standard first-order perturbation result for singular pairs
// (thin SVD M = U S V^T, F_ij = 1 / (s_j^2 - s_i^2)):
//   Mbar = U [diag(sbar) + (F o (U^T Ubar - Ubar^T U)) S + S (F o (V^T Vbar -
//          Vbar^T V))] V^T + (I - U U^T) Ubar S^-1 V^T + U S^-1 Vbar^T (I - V V^T).
// Singular values within 1e-12 s_1^2 of each other get F = 0 (the loss does
// not depend on the basis inside such a space).
#include "tt_step.h"

namespace tt {

// Inner matrix of the truncated-SVD adjoint (kc x kc), with the two
// complement-projector terms folded in:
//   In = diag(sbar) + (F o (G1 - G1^T)) S + S (F o (G2 - G2^T)) - G1 S_r^-1 - S_r^-1 G2^T,
// G1 = U^T Ubar, G2 = V^T Vbar (Ubar, Vbar zero beyond column r), F_ij =
// 1/(s_j^2 - s_i^2) off ties (|s_j^2 - s_i^2| <= 1e-12 s_1^2 counts as a tie),
// so that  Mbar = U In V^T + Ubar S_r^-1 V^T + U S_r^-1 Vbar^T.  G2 or sbar may
// be null (taken as zero).
__global__ void k_svd_adj_inner(const double* __restrict__ G1, const double* __restrict__ G2,
                                int ldg, const double* __restrict__ s,
                                const double* __restrict__ sbar, double* __restrict__ out,
                                int ldo, const int* __restrict__ dims, int kc_idx, int r_idx) {
  const int kc = dims[kc_idx], r = dims[r_idx];
  const double tie = 1e-12 * (kc > 0 ? s[0] * s[0] : 0.0);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)kc * kc;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / kc), j = (int)(e % kc);
    const double g1ij = G1[(long long)i * ldg + j], g1ji = G1[(long long)j * ldg + i];
    const double g2ij = G2 ? G2[(long long)i * ldg + j] : 0.0;
    const double g2ji = G2 ? G2[(long long)j * ldg + i] : 0.0;
    double v = 0.0;
    if (i == j) {
      v = (i < r && sbar) ? sbar[i] : 0.0;
    } else {
      const double dl = s[j] * s[j] - s[i] * s[i];
      if (fabs(dl) > tie) v = ((g1ij - g1ji) * s[j] + s[i] * (g2ij - g2ji)) / dl;
    }
    if (j < r) v -= g1ij / s[j];
    if (i < r) v -= g2ji / s[i];
    out[(long long)i * ldo + j] = v;
  }
}

// Copy the short-side singular vectors (rows < dims[rows_idx], columns <
// dims[kc_idx]) when dims[side_idx] == side.
__global__ void k_copy_cond(const double* __restrict__ src, int lds, double* __restrict__ dst,
                            int ldd, const int* __restrict__ dims, int rows_idx, int kc_idx,
                            int side_idx, int side) {
  if (dims[side_idx] != side) return;
  const int rows = dims[rows_idx], kc = dims[kc_idx];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)rows * kc;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / kc), j = (int)(e % kc);
    dst[(long long)i * ldd + j] = src[(long long)i * lds + j];
  }
}

// When dims[side_idx] == 1: sign-fix U's columns (largest |entry|, first on
// ties, positive) and apply the same signs to V's columns; a wavefront per
// column.  Matches the forward's gauge of U = M V S^-1.
__global__ __launch_bounds__(256) void k_gauge_pair(double* __restrict__ U, int ldu,
                                                    double* __restrict__ V, int ldv,
                                                    const int* __restrict__ dims, int ka_idx,
                                                    int kb_idx, int kc_idx, int side_idx) {
  if (dims[side_idx] != 1) return;
  const int kA = dims[ka_idx], kB = dims[kb_idx], kc = dims[kc_idx];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave;
  if (c >= kc) return;
  double best = -1.0, val = 0.0;
  int bi = 0x7fffffff;
  for (int i = lane; i < kA; i += 64) {
    const double v = U[(long long)i * ldu + c];
    if (fabs(v) > best) { best = fabs(v); val = v; bi = i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double b2 = __shfl_xor(best, o), v2 = __shfl_xor(val, o);
    const int i2 = __shfl_xor(bi, o);
    if (b2 > best || (b2 == best && i2 < bi)) { best = b2; val = v2; bi = i2; }
  }
  if (val < 0.0) {
    for (int i = lane; i < kA; i += 64) U[(long long)i * ldu + c] = -U[(long long)i * ldu + c];
    for (int i = lane; i < kB; i += 64) V[(long long)i * ldv + c] = -V[(long long)i * ldv + c];
  }
}

// Y[i][j] += X[i][j] * s[j] for i < rows, j < dims[c_idx].
__global__ void k_add_colscaled(const double* __restrict__ X, int ldx, const double* __restrict__ sc,
                                double* __restrict__ Y, int ldy, const int* __restrict__ dims,
                                DimExpr rdim, int c_idx) {
  const int rows = eval_dim(dims, rdim), cols = dims[c_idx];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)rows * cols;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    Y[(long long)i * ldy + j] += X[(long long)i * ldx + j] * sc[j];
  }
}

// Zero the leading rows x cols block.
__global__ void k_zero_block(double* __restrict__ A, int lda, const int* __restrict__ dims,
                             DimExpr rdim, DimExpr cdim) {
  const int rows = eval_dim(dims, rdim), cols = eval_dim(dims, cdim);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)rows * cols;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    A[(long long)i * lda + j] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Transposed concatenation for the spatial core, a wavefront per cell row:
//   Xbar[i][a] = sum_b (S_b^T (d o Xcatbar[:, block b]))[i][a],
// where S_0 = I, D_a^- X = X - X(. - e_a) has transpose Z - Z(. + e_a) and
// D_a^+ X = X(. + e_a) - X has transpose Z(. - e_a) - Z (zero ghosts, or
// wrapped when periodic); and the opacity gradient
//   kbar_i += dbar_i dd_i + sbar_i ds_i,   dbar_i = sum_{transport, inflow
//   columns} Xcatbar[i][col] * (unscaled X_cat)[i][col],   sbar_i = the
// emission column of Xcatbar.
__global__ __launch_bounds__(256) void k_xcat_adjoint(StepGeom G, const double* __restrict__ X,
                                                      int ldX, const double* __restrict__ bc_e,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ dd,
                                                      const double* __restrict__ ds,
                                                      const double* __restrict__ Xcb, int ldC,
                                                      double* __restrict__ Xb,
                                                      double* __restrict__ kbar,
                                                      const int* __restrict__ dims) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= G.ns) return;
  const int lane = threadIdx.x & 63;
  const int r1 = dims[D_R1];
  const int R1 = dims[D_RC1];
  const int nst = G.B * r1;
  const int ix = i % G.nx, iy = (i / G.nx) % G.ny, iz = i / (G.nx * G.ny);
  const int coord[3] = {ix, iy, iz};
  const double* xi = X + (long long)i * ldX;
  const double* gi = Xcb + (long long)i * ldC;
  const double di = d[i];
  double dbar = 0.0;
  for (int a = lane; a < r1; a += 64) {
    double acc = di * gi[a];  // identity block
    dbar += gi[a] * xi[a];
    for (int ax = 0; ax < 3; ++ax) {
      if (2 * ax + 2 >= G.B + 1) break;
      const int st = G.stride[ax], na = G.n[ax], ca = coord[ax];
      const int cm = (1 + 2 * ax) * r1 + a, cp = (2 + 2 * ax) * r1 + a;
      // unscaled stencil values of this row (for dbar)
      double xm = 0.0, xp = 0.0;
      if (ca > 0) xm = X[(long long)(i - st) * ldX + a];
      else if (G.periodic[ax]) xm = X[(long long)(i + (na - 1) * st) * ldX + a];
      if (ca < na - 1) xp = X[(long long)(i + st) * ldX + a];
      else if (G.periodic[ax]) xp = X[(long long)(i - (na - 1) * st) * ldX + a];
      dbar += gi[cm] * (xi[a] - xm) + gi[cp] * (xp - xi[a]);
      // D^- transpose: Z_i - Z_{i+e};  D^+ transpose: Z_{i-e} - Z_i
      acc += di * gi[cm] - di * gi[cp];
      long long jn = -1, jp = -1;  // rows i+e and i-e
      if (ca < na - 1) jn = i + st;
      else if (G.periodic[ax]) jn = i - (long long)(na - 1) * st;
      if (ca > 0) jp = i - st;
      else if (G.periodic[ax]) jp = i + (long long)(na - 1) * st;
      if (jn >= 0) acc -= d[jn] * Xcb[jn * ldC + cm];
      if (jp >= 0) acc += d[jp] * Xcb[jp * ldC + cp];
    }
    Xb[(long long)i * ldX + a] = acc;
  }
  for (int j = lane; j < G.nbc; j += 64) dbar += gi[nst + j] * bc_e[(long long)j * G.ns + i];
  for (int o = 32; o > 0; o >>= 1) dbar += __shfl_xor(dbar, o);
  if (lane == 0) {
    const double sbar = G.nem ? gi[R1 - 1] : 0.0;
    kbar[i] += dbar * dd[i] + sbar * ds[i];
  }
}

// Transposed concatenation of the angular cores:
//   Thbar[a][l][c] = sum_b tfac_b[l] Thcatbar[b r1 + a][l][b r2 + c],
//   Phbar[c][p]    = sum_b pfac_b[p] Phcatbar[b r2 + c][p].
__global__ void k_thcat_adjoint(StepGeom G, const double* __restrict__ tfac,
                                const double* __restrict__ Thcb, double* __restrict__ Thb,
                                const int* __restrict__ dims) {
  const int r1 = dims[D_R1], r2 = dims[D_R2];
  const long long tot = (long long)r1 * G.nt * r2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % r2);
    const long long al = e / r2;
    const int l = (int)(al % G.nt), a = (int)(al / G.nt);
    double v = 0.0;
    for (int b = 0; b < G.B; ++b)
      v += tfac[b * G.nt + l] * Thcb[((long long)(b * r1 + a) * G.nt + l) * G.R2c + b * r2 + c];
    Thb[((long long)a * G.nt + l) * G.r2c + c] = v;
  }
}
__global__ void k_phcat_adjoint(StepGeom G, const double* __restrict__ pfac,
                                const double* __restrict__ Phcb, double* __restrict__ Phb,
                                const int* __restrict__ dims) {
  const int r2 = dims[D_R2];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r2 * G.np; e += gridDim.x * blockDim.x) {
    const int c = e / G.np, p = e % G.np;
    double v = 0.0;
    for (int b = 0; b < G.B; ++b) v += pfac[b * G.np + p] * Phcb[(long long)(b * r2 + c) * G.np + p];
    Phb[(long long)c * G.np + p] = v;
  }
}

// Opacity derivatives of the frozen-temperature source coefficients:
// d = 1/(1 + c dt rho kappa): dd = -c dt rho d^2;
// s = d c dt rho kappa (c/4pi) a_r T^4: ds = c dt rho (c/4pi) a_r T^4 d^2.
__global__ void k_source_derivs(int ns, double c, double dt, double a_r,
                                const double* __restrict__ rho, const double* __restrict__ T,
                                const double* __restrict__ d, double* __restrict__ dd,
                                double* __restrict__ ds) {
  const double q = c / (4.0 * 3.14159265358979323846) * a_r;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
    const double di = d[i], t2 = T[i] * T[i];
    dd[i] = -c * dt * rho[i] * di * di;
    ds[i] = c * dt * rho[i] * q * t2 * t2 * di * di;
  }
}

// Loss L = dV sum_i w_i E_i with E_i = X_i z (z = (1/c) sum_l w_l Theta_l pv,
// pv = Phi v): its seed  Xbar_i = lbar dV w_i z  (scale = lbar dV).
__global__ void k_seed_x(const double* __restrict__ w, const double* __restrict__ z, double scale,
                         double* __restrict__ Xb, int ldX, int ns, const int* __restrict__ dims) {
  const int r1 = dims[D_R1];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)ns * ldX;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / ldX), a = (int)(e % ldX);
    Xb[e] = a < r1 ? scale * w[i] * z[a] : 0.0;
  }
}
// Thbar[a][l][c] = scale xg_a w_l pv_c,  Phbar[c][p] = scale v_p sum_a xg_a sum_l w_l Th[a][l][c]
// (xg = X^T w; scale = lbar dV / c).
__global__ void k_seed_angular(const double* __restrict__ xg, const double* __restrict__ wq,
                               const double* __restrict__ v, const double* __restrict__ pv,
                               const double* __restrict__ Th, int nt, int r2c, int np,
                               double scale, double* __restrict__ Thb, double* __restrict__ Phb,
                               const int* __restrict__ dims) {
  const int r1 = dims[D_R1], r2 = dims[D_R2];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nthr = gridDim.x * blockDim.x;
  for (long long e = t; e < (long long)r1 * nt * r2c; e += nthr) {
    const int c = (int)(e % r2c);
    const long long al = e / r2c;
    const int l = (int)(al % nt), a = (int)(al / nt);
    Thb[e] = c < r2 ? scale * xg[a] * wq[l] * pv[c] : 0.0;
  }
  for (int e = t; e < r2 * np; e += nthr) {
    const int c = e / np, p = e % np;
    double s = 0.0;
    for (int a = 0; a < r1; ++a) {
      double sl = 0.0;
      for (int l = 0; l < nt; ++l) sl += wq[l] * Th[((long long)a * nt + l) * r2c + c];
      s += xg[a] * sl;
    }
    Phb[(long long)c * np + p] = scale * v[p] * s;
  }
}

// xg[a] = sum_i w_i X[i][a] (a block per column).
__global__ __launch_bounds__(256) void k_xtw(const double* __restrict__ X, int ldX, int ns,
                                             const double* __restrict__ w, double* __restrict__ xg,
                                             const int* __restrict__ dims) {
  const int a = blockIdx.x;
  if (a >= dims[D_R1]) return;
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < ns; i += 256) s += w[i] * X[(long long)i * ldX + a];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) xg[a] = ((red[0] + red[1]) + red[2]) + red[3];
}

// out = sum_i w_i E_i (one block, fixed order).
__global__ __launch_bounds__(256) void k_wdot(const double* __restrict__ w,
                                              const double* __restrict__ E, int ns,
                                              double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < ns; i += 256) s += w[i] * E[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = ((red[0] + red[1]) + red[2]) + red[3];
}

// dims[D_REPLAY1/2] from the recorded rank history (step m).
__global__ void k_replay_from_hist(int* __restrict__ dims, const int* __restrict__ hist, int m) {
  if (threadIdx.x == 0) {
    dims[D_REPLAY1] = hist[2 * m];
    dims[D_REPLAY2] = hist[2 * m + 1];
  }
}
// ---------------------------------------------------------------------------
static int blocks_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_svd_adj_inner(const double* G1, const double* G2, int ldg, const double* sv,
                          const double* sbar, double* out, int ldo, const int* dims, int kc_idx,
                          int r_idx, int cap, hipStream_t s) {
  k_svd_adj_inner<<<blocks_for((long long)cap * cap), 256, 0, s>>>(G1, G2, ldg, sv, sbar, out, ldo,
                                                                   dims, kc_idx, r_idx);
}
void launch_copy_cond(const double* src, int lds, double* dst, int ldd, const int* dims,
                      int rows_idx, int kc_idx, int side_idx, int side, int cap, hipStream_t s) {
  k_copy_cond<<<blocks_for((long long)cap * cap), 256, 0, s>>>(src, lds, dst, ldd, dims, rows_idx,
                                                               kc_idx, side_idx, side);
}
void launch_gauge_pair(double* U, int ldu, double* V, int ldv, const int* dims, int ka_idx,
                       int kb_idx, int kc_idx, int side_idx, int cap, hipStream_t s) {
  k_gauge_pair<<<(cap + 3) / 4, 256, 0, s>>>(U, ldu, V, ldv, dims, ka_idx, kb_idx, kc_idx, side_idx);
}
void launch_add_colscaled(const double* X, int ldx, const double* sc, double* Y, int ldy,
                          const int* dims, DimExpr r, int c_idx, int cap, hipStream_t s) {
  k_add_colscaled<<<blocks_for((long long)cap * cap), 256, 0, s>>>(X, ldx, sc, Y, ldy, dims, r, c_idx);
}
void launch_zero_block(double* A, int lda, const int* dims, DimExpr r, DimExpr cdim, long long cap,
                       hipStream_t s) {
  k_zero_block<<<blocks_for(cap), 256, 0, s>>>(A, lda, dims, r, cdim);
}
void launch_xcat_adjoint(const StepGeom& G, const double* X, int ldX, const double* bc_e,
                         const double* d, const double* dd, const double* ds, const double* Xcb,
                         int ldC, double* Xb, double* kbar, const int* dims, hipStream_t s) {
  k_xcat_adjoint<<<(G.ns + 3) / 4, 256, 0, s>>>(G, X, ldX, bc_e, d, dd, ds, Xcb, ldC, Xb, kbar, dims);
}
void launch_cat_angular_adjoint(const StepGeom& G, const double* tfac, const double* pfac,
                                const double* Thcb, const double* Phcb, double* Thb, double* Phb,
                                const int* dims, hipStream_t s) {
  k_thcat_adjoint<<<blocks_for((long long)G.r1c * G.nt * G.r2c), 256, 0, s>>>(G, tfac, Thcb, Thb, dims);
  k_phcat_adjoint<<<blocks_for((long long)G.r2c * G.np), 256, 0, s>>>(G, pfac, Phcb, Phb, dims);
}
void launch_source_derivs(int ns, double c, double dt, double a_r, const double* rho,
                          const double* T, const double* d, double* dd, double* ds, hipStream_t s) {
  k_source_derivs<<<blocks_for(ns), 256, 0, s>>>(ns, c, dt, a_r, rho, T, d, dd, ds);
}
void launch_seed(const double* w, const double* z, const double* X, int ldX, int ns,
                 const double* wq, const double* v, const double* pv, const double* Th, int nt,
                 int r2c, int np, int r1c, double scale_x, double scale_ang, double* xg,
                 double* Xb, double* Thb, double* Phb, const int* dims, hipStream_t s) {
  k_seed_x<<<blocks_for((long long)ns * ldX), 256, 0, s>>>(w, z, scale_x, Xb, ldX, ns, dims);
  k_xtw<<<r1c, 256, 0, s>>>(X, ldX, ns, w, xg, dims);
  k_seed_angular<<<blocks_for((long long)r1c * nt * r2c), 256, 0, s>>>(
      xg, wq, v, pv, Th, nt, r2c, np, scale_ang, Thb, Phb, dims);
}
void launch_wdot(const double* w, const double* E, int ns, double* out, hipStream_t s) {
  k_wdot<<<1, 256, 0, s>>>(w, E, ns, out);
}
void launch_replay_from_hist(int* dims, const int* hist, int m, hipStream_t s) {
  k_replay_from_hist<<<1, 64, 0, s>>>(dims, hist, m);
}

}  // namespace tt
