// Per-step kernels other than the dense contractions and eigensolves:
//  - TT sum by core concatenation of the transport blocks (paper Sec. 4.3,
//    Sec. 4.1 Addition): stencil blocks of the spatial core, block-diagonal
//    middle core, stacked angular core, rank-1 inflow (Sec. 4.5) and
//    emission (Sec. 4.4) terms;
//  - backward-Euler absorption/emission coefficients and the per-cell
//    Newton solve for T_dag (Sec. 3.2), always in FP64;
//  - energy density from TT cores (Sec. 4.1 eq. tt_energy_density);
//  - the tolerance rank rule of the Gram-SVD truncation (App. A, note on
//    rank truncation) and the assembly of the truncated singular vectors.
#include "tt_step.h"

namespace tt {

// ---------------------------------------------------------------------------
// Row i + dir e_ax of X with the ghost rule of the face crossed (Sec. 4.5):
// zero (vacuum; inflow, whose ghost value enters as rank-1 blocks), wrapped
// (periodic), or row i itself (outflow).
template <typename TX>
__device__ inline double neighbour(const StepGeom& G, const TX* __restrict__ X, int ldX, int i,
                                   const int* coord, int ax, int dir, int a, double self) {
  const int st = G.stride[ax], na = G.n[ax], ca = coord[ax];
  if (dir < 0) {
    if (ca > 0) return (double)X[(long long)(i - st) * ldX + a];
    if (G.bclo[ax] == TT_BC_PERIODIC) return (double)X[(long long)(i + (na - 1) * st) * ldX + a];
    return G.bclo[ax] == TT_BC_OUTFLOW ? self : 0.0;
  }
  if (ca < na - 1) return (double)X[(long long)(i + st) * ldX + a];
  if (G.bchi[ax] == TT_BC_PERIODIC) return (double)X[(long long)(i - (na - 1) * st) * ldX + a];
  return G.bchi[ax] == TT_BC_OUTFLOW ? self : 0.0;
}

// HLL block entry (Sec. 3.1 eq. hll; Sec. 4.3) of cell i from its value x0
// and its neighbours m, p along ax: with the sign's weights at the cell's
// faces, (alpha_hi - beta_lo) x0 + beta_hi p - alpha_lo m; for n < 0 the
// weights are the n >= 0 pair swapped.
__device__ __forceinline__ double hll_entry(const StepGeom& G, int kind, int ax, int i, double x0,
                                            double m, double p) {
  const double* w = G.hllw + ((long long)ax * G.ns + i) * 4;
  const double aph = w[HLLW_AP_HI], bph = w[HLLW_BP_HI], apl = w[HLLW_AP_LO], bpl = w[HLLW_BP_LO];
  if (kind == BK_HLL_POS) return (aph - bpl) * x0 + bph * p - apl * m;
  return (bph - apl) * x0 + aph * p - bpl * m;
}

// Row i of the unscaled concatenation X_cat by column a of the state, for
// every transport block at once: X(i, a) and its neighbours along the axes
// the blocks use are loaded once, then block b's entry (column b r1 + a) is
// formed from them: the state row itself (BK_BASE), the one-sided
// differences (BK_MINUS, BK_PLUS), the central difference (BK_CENTRAL), the
// second difference (BK_DIFF) or the weighted HLL stencil (BK_HLL_*) along
// the block's axis.  f(b, v) receives each entry.  HLL: the HLL kinds are
// compiled in (a separate instantiation, so that the other fluxes' kernels
// keep their register budget).
template <bool HLL, typename TX, typename F>
__device__ __forceinline__ void xcat_row_blocks(const StepGeom& G, const TX* __restrict__ X, int ldX,
                                                int i, const int* coord, int a, int axm, F&& f) {
  const double x0 = (double)X[(long long)i * ldX + a];
  double xm[3] = {0.0, 0.0, 0.0}, xp[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
    if ((axm >> ax) & 1) {
      xm[ax] = neighbour(G, X, ldX, i, coord, ax, -1, a, x0);
      xp[ax] = neighbour(G, X, ldX, i, coord, ax, 1, a, x0);
    }
  for (int b = 0; b < G.B; ++b) {
    const int kind = G.bkind[b], ax = G.baxis[b];
    const double m = ax == 0 ? xm[0] : ax == 1 ? xm[1] : xm[2];
    const double p = ax == 0 ? xp[0] : ax == 1 ? xp[1] : xp[2];
    double v;
    if (kind == BK_BASE) v = x0;
    else if (kind == BK_MINUS) v = x0 - m;
    else if (kind == BK_PLUS) v = p - x0;
    else if (kind == BK_CENTRAL) v = 0.5 * (p - m);
    else if (!HLL || kind == BK_DIFF) v = (p - 2.0 * x0) + m;
    else v = hll_entry(G, kind, ax, i, x0, m, p);
    f(b, v);
  }
}

// Axes whose neighbours some transport block reads (bit ax).
__device__ inline int xcat_axes(const StepGeom& G) {
  int m = 0;
  for (int b = 0; b < G.B; ++b)
    if (G.bkind[b] != BK_BASE) m |= 1 << G.baxis[b];
  return m;
}

// Spatial core of the concatenation, a wavefront per cell row.
// TX / TC: element type of X and X_cat (double, or float in the FP32-mixed
// form; the arithmetic is FP64 and each entry is rounded once on store).
// scaled: rows times d_i and the emission column s_i (else 1 and 0).
// X_cat is written with non-temporal stores: it is read back only by the next
// kernels' streams, and keeping it out of the caches leaves them to the X
// rows that neighbouring cells load again (thick 3-D: 6.2 -> 5.3 ms).
template <typename TX, typename TC, bool HLL>
__global__ __launch_bounds__(256) void k_build_xcat(StepGeom G, const TX* __restrict__ X, int ldX,
                                                    const double* __restrict__ bc_e,
                                                    const double* __restrict__ d,
                                                    const double* __restrict__ s,
                                                    TC* __restrict__ Xc, int ldC,
                                                    const int* __restrict__ dims, int scaled) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);  // a wavefront per cell row
  if (i >= G.ns) return;
  const int lane = threadIdx.x & 63;
  const int r1 = dims[D_R1];
  const int R1 = dims[D_RC1];
  const int nstencil = G.B * r1;
  const int coord[3] = {i % G.nx, (i / G.nx) % G.ny, i / (G.nx * G.ny)};
  const int axm = xcat_axes(G);
  const double di = scaled ? d[i] : 1.0;
  TC* out = Xc + (long long)i * ldC;
  for (int a = lane; a < r1; a += 64)
    xcat_row_blocks<HLL>(G, X, ldX, i, coord, a, axm, [&](int b, double v) {
      __builtin_nontemporal_store((TC)(v * di), &out[b * r1 + a]);
    });
  for (int col = nstencil + lane; col < R1; col += 64) {
    const double v = col < nstencil + G.nbc ? bc_e[(long long)(col - nstencil) * G.ns + i] * di
                                            : (scaled ? s[i] : 0.0);
    __builtin_nontemporal_store((TC)v, &out[col]);
  }
}

// E_i = sum over the transport and inflow columns of the unscaled
// concatenation of X_cat[i][col] z[col], with the entries formed from X as
// k_build_xcat forms them (X_cat is neither written nor read): the
// post-transport energy density before the source coefficients exist, so
// that X_cat can then be built once with them.
template <typename TX, bool HLL>
__global__ __launch_bounds__(256) void k_xcat_row_dot(StepGeom G, const TX* __restrict__ X, int ldX,
                                                      const double* __restrict__ bc_e,
                                                      const double* __restrict__ z,
                                                      double* __restrict__ E,
                                                      const int* __restrict__ dims) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= G.ns) return;
  const int lane = threadIdx.x & 63;
  const int r1 = dims[D_R1];
  const int nstencil = G.B * r1;
  const int coord[3] = {i % G.nx, (i / G.nx) % G.ny, i / (G.nx * G.ny)};
  const int axm = xcat_axes(G);
  double acc = 0.0;
  for (int a = lane; a < r1; a += 64)
    xcat_row_blocks<HLL>(G, X, ldX, i, coord, a, axm, [&](int b, double v) { acc += v * z[b * r1 + a]; });
  for (int col = nstencil + lane; col < nstencil + G.nbc; col += 64)
    acc += bc_e[(long long)(col - nstencil) * G.ns + i] * z[col];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) E[i] = acc;
}

// The same E* in FP64 without forming X_cat's entries: the stencils are
// linear, so sum_b (D_b X)(i, :) z_b = sum_b (D_b y_b)(i) with y_b = X z_b.
// k_gemm_panel forms Y = X Zt (Zt[a][b] = z[b r1 + a], an N_s x B product
// that reads X once), then this kernel applies each block's stencil to its
// column of Y, with the ghost values of neighbour(), and adds the inflow
// columns.
__global__ void k_z_blocks(const double* __restrict__ z, double* __restrict__ Zt, int ldz, int B,
                           const int* __restrict__ dims) {
  const int r1 = dims[D_R1];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r1 * B; e += gridDim.x * blockDim.x) {
    const int a = e / B, b = e % B;
    Zt[(long long)a * ldz + b] = z[(long long)b * r1 + a];
  }
}
template <bool HLL>
__global__ __launch_bounds__(256) void k_energy_stencil(StepGeom G, const double* __restrict__ Y,
                                                        int ldy, const double* __restrict__ bc_e,
                                                        const double* __restrict__ z,
                                                        double* __restrict__ E,
                                                        const int* __restrict__ dims) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.ns) return;
  const int r1 = dims[D_R1];
  const int nstencil = G.B * r1;
  const int coord[3] = {i % G.nx, (i / G.nx) % G.ny, i / (G.nx * G.ny)};
  double acc = 0.0;
  for (int b = 0; b < G.B; ++b) {
    const int kind = G.bkind[b], ax = G.baxis[b];
    const double y0 = Y[(long long)i * ldy + b];
    double v;
    if (kind == BK_BASE) {
      v = y0;
    } else {
      const double m = neighbour(G, Y, ldy, i, coord, ax, -1, b, y0);
      const double p = neighbour(G, Y, ldy, i, coord, ax, 1, b, y0);
      if (kind == BK_MINUS) v = y0 - m;
      else if (kind == BK_PLUS) v = p - y0;
      else if (kind == BK_CENTRAL) v = 0.5 * (p - m);
      else if (!HLL || kind == BK_DIFF) v = (p - 2.0 * y0) + m;
      else v = hll_entry(G, kind, ax, i, y0, m, p);
    }
    acc += v;
  }
  for (int c = 0; c < G.nbc; ++c) acc += bc_e[(long long)c * G.ns + i] * z[nstencil + c];
  E[i] = acc;
}

// HLL weights of a face of optical depth tau (Sec. 3.1): with
// A = sqrt((1 - exp(-tau^2)) / tau^2) and B = sqrt((1 - exp(-tau^4)) / tau^2),
// or their series sqrt(1 - tau^2 / 2) and tau below the threshold, the
// wavespeeds S_R = c n A, S_L = -c n B (n >= 0) put eq. hll with F = c n U
// in the form c n (alpha_p U_L + beta_p U_R), alpha_p = A (1 + B) / (A + B),
// beta_p = B (1 - A) / (A + B).  tau -> 0 gives (1, 0), the upwind flux.
__device__ inline void hll_pair(double tau, double thr, double& ap, double& bp) {
  double A, B;
  if (tau < thr) {
    A = sqrt(fmax(1.0 - 0.5 * tau * tau, 0.0));
    B = tau;
  } else {
    const double t2 = tau * tau;
    A = sqrt((1.0 - exp(-t2)) / t2);
    B = sqrt((1.0 - exp(-t2 * t2)) / t2);
  }
  ap = A * (1.0 + B) / (A + B);
  bp = B * (1.0 - A) / (A + B);
}

// tau_c of eq. tauc for a face between extinctions ea and eb (rho (kappa +
// kappa_s) of the two cells): 2 beta h / (1/ea + 1/eb); zero when either
// side has none.
__device__ inline double hll_face_tau(double ea, double eb, double bh) {
  const double inv = 1.0 / ea + 1.0 / eb;
  return inv < __builtin_inf() ? 2.0 * bh / inv : 0.0;
}

// One thread per cell; per axis, the weights of its hi face (the neighbour
// i + e, wrapped on a periodic axis) and of its lo face (i - e).  A face on a
// non-periodic boundary sees the cell's own extinction on both sides.
__global__ void k_hll_weights(StepGeom G, int dim, const double* __restrict__ rho,
                              const double* __restrict__ kappa, const double* __restrict__ kappa_s,
                              double beta, double h0, double h1, double h2, double thr,
                              double* __restrict__ W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.ns) return;
  const int coord[3] = {i % G.nx, (i / G.nx) % G.ny, i / (G.nx * G.ny)};
  const double ei = rho[i] * (kappa[i] + kappa_s[i]);
  for (int ax = 0; ax < dim; ++ax) {
    const int st = G.stride[ax], na = G.n[ax], ca = coord[ax];
    const int jp = ca < na - 1 ? i + st : (G.periodic[ax] ? i - (na - 1) * st : i);
    const int jm = ca > 0 ? i - st : (G.periodic[ax] ? i + (na - 1) * st : i);
    const double ep = rho[jp] * (kappa[jp] + kappa_s[jp]);
    const double em = rho[jm] * (kappa[jm] + kappa_s[jm]);
    const double bh = beta * (ax == 0 ? h0 : ax == 1 ? h1 : h2);
    double* w = W + ((long long)ax * G.ns + i) * 4;
    double ap, bp;
    hll_pair(hll_face_tau(ei, ep, bh), thr, ap, bp);
    w[HLLW_AP_HI] = ap;
    w[HLLW_BP_HI] = bp;
    hll_pair(hll_face_tau(em, ei, bh), thr, ap, bp);
    w[HLLW_AP_LO] = ap;
    w[HLLW_BP_LO] = bp;
  }
}

__global__ void k_hll_inflow(int ns, const double* __restrict__ bc_e0, const int* __restrict__ code,
                             int nbc, const double* __restrict__ W, double* __restrict__ bc_e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  for (int c = 0; c < nbc; ++c) {
    const int ax = code[c] >> 2, sel = code[c] & 3;
    bc_e[(long long)c * ns + i] = bc_e0[(long long)c * ns + i] * W[((long long)ax * ns + i) * 4 + sel];
  }
}

// Core conversion between FP64 and FP32 storage (rows x cols, leading dims).
template <typename TA, typename TB>
__global__ void k_convert(const TA* __restrict__ a, int lda, TB* __restrict__ b, int ldb, int rows,
                          int cols) {
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    b[(long long)i * ldb + j] = (TB)a[(long long)i * lda + j];
  }
}

// Angular core of the concatenation: Phcat[R2c][np].
__global__ void k_build_phcat(StepGeom G, const double* __restrict__ Ph,
                              const double* __restrict__ pfac, const double* __restrict__ bc_p,
                              double* __restrict__ Pc, const int* __restrict__ dims) {
  const int r2 = dims[D_R2];
  const int total = G.R2c * G.np;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int row = e / G.np, p = e - row * G.np;
    const int nst = G.B * r2;
    double v = 0.0;
    if (row < nst) {
      const int b = row / r2, c = row - b * r2;
      v = pfac[b * G.np + p] * Ph[(long long)c * G.np + p];
    } else if (row < nst + G.nbc) {
      v = bc_p[(long long)(row - nst) * G.np + p];
    } else if (row < nst + G.nbc + G.nem) {
      v = 1.0;
    }
    Pc[e] = v;
  }
}

// Middle core of the concatenation: Thcat[a][l][c] (R1 x nt x R2c), block
// diagonal.  Rows a >= R1 are not written.
__global__ void k_build_thcat(StepGeom G, const double* __restrict__ Th,
                              const double* __restrict__ tfac, const double* __restrict__ bc_t,
                              double* __restrict__ Tc, const int* __restrict__ dims) {
  const int r1 = dims[D_R1], r2 = dims[D_R2], R1 = dims[D_RC1];
  const long long total = (long long)R1 * G.nt * G.R2c;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % G.R2c);
    const long long al = e / G.R2c;
    const int l = (int)(al % G.nt), a = (int)(al / G.nt);
    double v = 0.0;
    const int nst1 = G.B * r1, nst2 = G.B * r2;
    if (a < nst1) {
      const int b = a / r1, ai = a - b * r1;
      const int c0 = b * r2;
      if (c >= c0 && c < c0 + r2)
        v = tfac[b * G.nt + l] * Th[((long long)ai * G.nt + l) * G.r2c + (c - c0)];
    } else if (a < nst1 + G.nbc) {
      const int j = a - nst1;
      if (c == nst2 + j) v = bc_t[(long long)j * G.nt + l];
    } else {
      if (c == nst2 + G.nbc) v = 1.0;
    }
    Tc[e] = v;
  }
}

// dims after the concatenation: R1 = B r1 + n_bc + n_em, R2 likewise.
__global__ void k_concat_dims(StepGeom G, int* __restrict__ dims) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dims[D_RC1] = G.B * dims[D_R1] + G.nbc + G.nem;
    dims[D_RC2] = G.B * dims[D_R2] + G.nbc + G.nem;
  }
}

// dims of the transport-only concatenation: R = B r + n_bc.
__global__ void k_transport_dims(StepGeom G, int* __restrict__ dims) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dims[D_RC1] = G.B * dims[D_R1] + G.nbc;
    dims[D_RC2] = G.B * dims[D_R2] + G.nbc;
  }
}

// Source update of the two-rounding schedule as a TT sum: X_cat = [d X, s]
// (a wavefront per cell row), Theta_cat = blockdiag(Theta, 1), Phi_cat =
// [Phi; 1] (the source block only when G.nem).  dims[RC] = r + nem is set by
// the caller's k_source_dims before this kernel.
template <typename TX>
__global__ __launch_bounds__(256) void k_source_xcat(StepGeom G, const TX* __restrict__ X, int ldX,
                                                     const double* __restrict__ d,
                                                     const double* __restrict__ s,
                                                     TX* __restrict__ Xc, int ldC,
                                                     const int* __restrict__ dims) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= G.ns) return;
  const int lane = threadIdx.x & 63;
  const int r1 = dims[D_R1];
  const double di = d[i];
  const TX* xi = X + (long long)i * ldX;
  TX* ci = Xc + (long long)i * ldC;
  for (int a = lane; a < r1; a += 64) ci[a] = (TX)((double)xi[a] * di);
  if (G.nem && lane == 0) ci[r1] = (TX)s[i];
}
__global__ void k_source_dims(StepGeom G, int* __restrict__ dims) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dims[D_RC1] = dims[D_R1] + G.nem;
    dims[D_RC2] = dims[D_R2] + G.nem;
  }
}
// Theta_cat rows [0, r1 + nem) x nt x R2c and Phi_cat rows [0, R2c).
__global__ void k_source_angular(StepGeom G, const double* __restrict__ Th,
                                 const double* __restrict__ Ph, double* __restrict__ Tc,
                                 double* __restrict__ Pc, const int* __restrict__ dims) {
  const int r1 = dims[D_R1], r2 = dims[D_R2];
  const long long tot = (long long)(r1 + G.nem) * G.nt * G.R2c;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int cc = (int)(e % G.R2c);
    const long long al = e / G.R2c;
    const int a = (int)(al / G.nt);
    double v = 0.0;
    if (a < r1) v = cc < r2 ? Th[al * G.r2c + cc] : 0.0;
    else v = cc == r2 ? 1.0 : 0.0;
    Tc[e] = v;
  }
  const int tp = G.R2c * G.np;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tp; e += gridDim.x * blockDim.x) {
    const int row = e / G.np;
    Pc[e] = row < r2 ? Ph[e] : (row == r2 && G.nem ? 1.0 : 0.0);
  }
}

// dims for rounding the stored state itself (no concatenation).
__global__ void k_round_dims(int* __restrict__ dims) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dims[D_RC1] = dims[D_R1];
    dims[D_RC2] = dims[D_R2];
  }
}

// Copy Th (ld r2c) into Thcat layout (ld R2c), zero elsewhere; Ph -> Phcat.
__global__ void k_state_as_cat(StepGeom G, const double* __restrict__ Th,
                               const double* __restrict__ Ph, double* __restrict__ Tc,
                               double* __restrict__ Pc, const int* __restrict__ dims) {
  const int r1 = dims[D_R1], r2 = dims[D_R2];
  const long long tot = (long long)r1 * G.nt * G.R2c;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % G.R2c);
    const long long al = e / G.R2c;
    Tc[e] = c < r2 ? Th[al * G.r2c + c] : 0.0;
  }
  const int tp = G.R2c * G.np;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tp; e += gridDim.x * blockDim.x)
    Pc[e] = (e / G.np) < r2 ? Ph[e] : 0.0;
}

// ---------------------------------------------------------------------------
// Energy density of a TT: z = (sum_l w_l Theta_l)(sum_p v_p Phi_p), E = X z / c.
// pv[c] = sum_p v_p Phi[c][p]
__global__ void k_phi_moment(const double* __restrict__ Ph, int np, const double* __restrict__ v,
                             double* __restrict__ pv, DimExpr rows, const int* __restrict__ dims) {
  const int r = eval_dim(dims, rows);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < r; c += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < np; ++p) s += v[p] * Ph[(long long)c * np + p];
    pv[c] = s;
  }
}
// z[a] = (1/c) sum_l w_l sum_b Th[a][l][b] pv[b], a < r1 (Th ld = ldb per l)
__global__ __launch_bounds__(256) void k_theta_moment(const double* __restrict__ Th, int nt,
                                                      int ldb, const double* __restrict__ w,
                                                      const double* __restrict__ pv,
                                                      double* __restrict__ z, DimExpr rows,
                                                      DimExpr cols, double inv_c,
                                                      const int* __restrict__ dims) {
  // a wavefront per row a of the core: its nt x r2 slab is read once,
  // coalesced, lane l taking the columns b = l + 64 m of every ordinate
  const int r1 = eval_dim(dims, rows), r2 = eval_dim(dims, cols);
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (a >= r1) return;
  double acc = 0.0;
  for (int l = 0; l < nt; ++l) {
    const double* t = Th + ((long long)a * nt + l) * ldb;
    double sl = 0.0;
    for (int b = lane; b < r2; b += 64) sl += t[b] * pv[b];
    acc += w[l] * sl;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) z[a] = acc * inv_c;
}
// E[i] = sum_{a < ncols} X[i][a] z[a]
template <typename TX>
__global__ __launch_bounds__(256) void k_row_dot(const TX* __restrict__ X, int ldX, int ns,
                                                 const double* __restrict__ z, DimExpr cols,
                                                 double* __restrict__ E,
                                                 const int* __restrict__ dims) {
  const int nc = eval_dim(dims, cols);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  if (i >= ns) return;
  const TX* x = X + (long long)i * ldX;
  double s = 0.0;
  for (int a = lane; a < nc; a += 64) s += (double)x[a] * z[a];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) E[i] = s;
}

// ---------------------------------------------------------------------------
// Source coefficients (Sec. 3.2).  d = 1 / (1 + c dt rho (kappa + kappa_s)).
// Frozen: T_dag = T.  Coupled: Newton on
// f(T) = T - T^m + g (a_r T^4 - E*), g = c dt kappa / c_v / (1 + c dt rho kappa)
// (kappa_s drops out once J^{m+1} is eliminated), started at
// max(T^m, (max(E*,0)/a_r)^(1/4)) where f >= 0 (f increasing, convex),
// stopping at |dT| <= 4u T (at most 50 iterations).
// s = d (c dt rho kappa_s J^{m+1} + e), e = c dt rho kappa (c/4pi) a_r T_dag^4,
// J^{m+1} = ((c/4pi) E* + e) / (1 + c dt rho kappa).
__global__ void k_material(int ns, double c, double dt, double a_r, int coupled,
                           const double* __restrict__ kappa, const double* __restrict__ kappa_s,
                           const double* __restrict__ rho, const double* __restrict__ cv,
                           const double* __restrict__ T, const double* __restrict__ Estar,
                           double* __restrict__ Tdag, double* __restrict__ d,
                           double* __restrict__ s, int* __restrict__ dims) {
  const double c4pi = c / (4.0 * 3.14159265358979323846);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
    const double rk = rho[i] * kappa[i];
    const double rs = kappa_s ? rho[i] * kappa_s[i] : 0.0;
    const double da = 1.0 / (1.0 + c * dt * rk);
    const double di = kappa_s ? 1.0 / (1.0 + c * dt * (rk + rs)) : da;
    double Td = T[i];
    if (coupled) {
      const double g = c * dt * kappa[i] / cv[i] * da;
      const double Es = Estar[i];
      const double Tm = T[i];
      double x = fmax(Tm, sqrt(sqrt(fmax(Es, 0.0) / a_r)));
      bool ok = false;
      for (int it = 0; it < 50; ++it) {
        const double x3 = x * x * x;
        const double f = x - Tm + g * (a_r * x3 * x - Es);
        const double fp = 1.0 + 4.0 * g * a_r * x3;
        const double dx = f / fp;
        x -= dx;
        if (fabs(dx) <= 4.0 * 1.1102230246251565e-16 * fabs(x + dx)) {
          ok = true;
          break;
        }
      }
      if (!ok || !(x == x)) atomicOr(&dims[D_FLAG], FLAG_NEWTON);
      Td = x;
    }
    const double T2 = Td * Td;
    const double e = c * dt * rk * c4pi * a_r * T2 * T2;
    double si = di * e;
    if (kappa_s) {
      const double Jn = (c4pi * Estar[i] + e) / (1.0 + c * dt * rk);
      si = di * (c * dt * rs * Jn + e);
    }
    d[i] = di;
    s[i] = si;
    if (Tdag) Tdag[i] = Td;
  }
}

// Energy-conserving temperature update T += (E* - E_new) / (rho c_v).
__global__ void k_temperature(int ns, const double* __restrict__ rho,
                              const double* __restrict__ cv, const double* __restrict__ Estar,
                              const double* __restrict__ Enew, double* __restrict__ T) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x)
    T[i] += (Estar[i] - Enew[i]) / (rho[i] * cv[i]);
}

// ---------------------------------------------------------------------------
// Number of singular values of M and which side's vectors are computed.
// The kept counts are first clipped to the rank each side can have (its
// number of rows): eigenpairs of a Gram beyond that rank are rounding noise.
__global__ void k_mside(int* __restrict__ dims, int ka, int kb, int km, int side, DimExpr abound,
                        DimExpr bbound) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int a = min(dims[ka], eval_dim(dims, abound));
    const int b = min(dims[kb], eval_dim(dims, bbound));
    dims[ka] = a;
    dims[kb] = b;
    dims[km] = a < b ? a : b;
    dims[side] = a <= b ? 0 : 1;
  }
}

// Rank rule on the singular values sigma_j of M (descending).  Bond 1
// defines ||T||^2 = sum sigma^2 and delta^2 = tol^2 ||T||^2 / 2; bond 2
// reuses delta^2.
//   r = min{k >= 1: sum_{j>k} sigma_j^2 <= delta^2}; cluster rule: extend
//   while sigma_r - sigma_{r+1} <= max(eta sigma_1, R u sigma_1^2 / sigma_r);
//   cap: r = rmax and, if that splits a cluster, cut before it (keep rmax if
//   it starts at 1).
__global__ void k_rank(const double* __restrict__ sig, int* __restrict__ dims,
                       double* __restrict__ diag, RankArgs ra) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = dims[ra.km];
  const int kc = dims[ra.kc];
  double norm2 = 0.0;
  for (int j = 0; j < n; ++j) norm2 += fmax(sig[j], 0.0) * fmax(sig[j], 0.0);
  double delta2;
  if (ra.bond == 1) {
    delta2 = ra.tol * ra.tol * norm2 / 2.0;
    diag[G_NORM2] = norm2;
    diag[G_DELTA2] = delta2;
    if (!(norm2 == norm2) || norm2 > 1.79e308) atomicOr(&dims[D_FLAG], FLAG_NONFINITE);
  } else {
    delta2 = diag[G_DELTA2];
  }
  const double s0 = n > 0 ? fmax(sig[0], 0.0) : 0.0;
  int r = 1, zero = 0;
  if (n == 0 || !(s0 > 0.0) || kc == 0) {
    zero = 1;
  } else {
    // tails from the smallest up: tail(k) = sum_{j >= k} sigma_j^2
    double tail = 0.0;
    r = n;
    for (int k = n - 1; k >= 1; --k) {
      tail += fmax(sig[k], 0.0) * fmax(sig[k], 0.0);
      if (tail <= delta2) r = k;
      else break;
    }
    // sigma_j and sigma_{j+1} (1-based j) are tied when they differ by no more
    // than the Gram route resolves: max(eta s1, R u s1^2 / sigma_j)
    const double noise = (double)dims[ra.rdim] * 1.1102230246251565e-16;
#define SIG(j) fmax(sig[(j)], 0.0)
#define TIED(j) (SIG((j) - 1) - SIG(j) <= fmax(ra.eta * s0, SIG((j) - 1) > 0.0 ? noise * s0 * s0 / SIG((j) - 1) : 1.79e308))
    // ... but never into a singular value below the resolution sqrt(R u) s1,
    // where every gap is within the noise
    const double floor_res = sqrt(noise) * s0;
    while (r < n && TIED(r) && SIG(r) > floor_res) ++r;
    if (ra.rmax > 0 && r > ra.rmax) {
      r = ra.rmax;
      if (r < n && TIED(r)) {
        int k = r;
        while (k > 1 && TIED(k - 1)) --k;
        r = k > 1 ? k - 1 : ra.rmax;
      }
    }
    const int rep = dims[ra.replay];
    if (rep > 0) r = rep;
    if (r > kc) r = kc;
    if (r < 1) r = 1;
    double t = 0.0;
    for (int j = r; j < n; ++j) t += SIG(j) * SIG(j);
    diag[ra.g_tail] = delta2 > 0.0 ? t / delta2 : 0.0;
    diag[ra.g_sr] = SIG(r - 1);
    diag[ra.g_srp] = r < n ? SIG(r) : 0.0;
    if (ra.bond == 1) diag[G_S1] = s0;
#undef TIED
#undef SIG
  }
  dims[ra.rn] = r;
  dims[ra.zero] = zero;
  dims[ra.kea] = zero ? 0 : dims[ra.ka];
  dims[ra.keb] = zero ? 0 : dims[ra.kb];
  if (ra.rnt >= 0) dims[ra.rnt] = r * ra.nt;
  diag[ra.g_rn] = r;
  diag[ra.g_ka] = dims[ra.ka];
  diag[ra.g_kb] = dims[ra.kb];
}

// Truncated singular vectors of M from the vectors Uc of its short side.
// side 0 (kA <= kB): U~ = Uc[:, :r]; W = M^T U~ was formed by a GEMM.
// side 1: V~ = Uc[:, :r]; W = V~ S~; U~ = M V~ S~^-1 was formed by a GEMM
// and is sign-fixed here (largest |entry| positive), with the same signs
// applied to W.
__global__ __launch_bounds__(256) void k_svd_vectors(const double* __restrict__ Uc, int ldu,
                                                     const double* __restrict__ sqc,
                                                     double* __restrict__ Ur, int ldr,
                                                     double* __restrict__ Wm, int ldw,
                                                     const int* __restrict__ dims, int ka_i,
                                                     int kb_i, int side_i, int rn_i,
                                                     int zero_i) {
  if (dims[zero_i]) return;
  const int side = dims[side_i], r = dims[rn_i];
  const int ka = dims[ka_i], kb = dims[kb_i];
  const int c = blockIdx.x;
  if (c >= r) return;
  if (side == 0) {
    for (int i = threadIdx.x; i < ka; i += 256) Ur[(long long)i * ldr + c] = Uc[(long long)i * ldu + c];
    return;
  }
  const double sc = sqc[c];
  for (int i = threadIdx.x; i < kb; i += 256) Wm[(long long)i * ldw + c] = Uc[(long long)i * ldu + c] * sc;
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int idx = 0x7fffffff;
  for (int i = threadIdx.x; i < ka; i += 256) {
    const double a = fabs(Ur[(long long)i * ldr + c]);
    if (a > best) { best = a; idx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double b2 = bv[threadIdx.x + o];
      const int i2 = bi[threadIdx.x + o];
      if (b2 > bv[threadIdx.x] || (b2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
        bv[threadIdx.x] = b2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const int imax = bi[0];
  __syncthreads();
  if (imax < ka && Ur[(long long)imax * ldr + c] < 0.0) {
    for (int i = threadIdx.x; i < ka; i += 256) Ur[(long long)i * ldr + c] = -Ur[(long long)i * ldr + c];
    for (int i = threadIdx.x; i < kb; i += 256) Wm[(long long)i * ldw + c] = -Wm[(long long)i * ldw + c];
  }
}

// Close a step: new ranks become the state ranks; with hist, the ranks go
// to history slot dims[D_HSLOT] while it is below hmax, and the slot advances.
__global__ void k_finish(int* __restrict__ dims, int* __restrict__ hist, int hmax) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  dims[D_R1] = dims[D_R1N];
  dims[D_R2] = dims[D_R2N];
  const int slot = dims[D_HSLOT];
  if (hist && slot < hmax) {
    hist[2 * slot] = dims[D_R1N];
    hist[2 * slot + 1] = dims[D_R2N];
    dims[D_HSLOT] = slot + 1;
  }
}

// Finite check of a vector (flag only).
__global__ void k_check_finite(const double* __restrict__ x, int n, int* __restrict__ dims) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (!(x[i] == x[i]) || fabs(x[i]) > 1.79e308) {
      atomicOr(&dims[D_FLAG], FLAG_NONFINITE);
      return;
    }
}

// Finiteness of the live state: X (FP64 or FP32), Theta, Phi and T.
template <typename TX>
__global__ void k_check_state(const TX* __restrict__ X, int ldX, int ns,
                              const double* __restrict__ Th, int nt, int r2c,
                              const double* __restrict__ Ph, int np,
                              const double* __restrict__ T, int* __restrict__ dims) {
  const int r1 = dims[D_R1], r2 = dims[D_R2];
  bool bad = false;
  const long long nx = (long long)ns * r1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (long long e = t0; e < nx && !bad; e += stride) {
    const double v = (double)X[(e / r1) * ldX + e % r1];
    bad = !(fabs(v) <= 1.79e308);
  }
  const long long nth = (long long)r1 * nt * r2;
  for (long long e = t0; e < nth && !bad; e += stride) {
    const double v = Th[(e / r2) * r2c + e % r2];
    bad = !(fabs(v) <= 1.79e308);
  }
  for (long long e = t0; e < (long long)r2 * np && !bad; e += stride) bad = !(fabs(Ph[e]) <= 1.79e308);
  for (long long e = t0; e < ns && !bad; e += stride) bad = !(fabs(T[e]) <= 1.79e308);
  if (bad) atomicOr(&dims[D_FLAG], FLAG_NONFINITE);
}

// ---------------------------------------------------------------------------
// host launchers
void launch_build_xcat(const StepGeom& G, const double* X, int ldX, const double* bc_e,
                       const double* d, const double* s, double* Xc, int ldC, const int* dims,
                       int scaled, hipStream_t st) {
  if (G.hllw)
    k_build_xcat<double, double, true><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, bc_e, d, s, Xc, ldC, dims,
                                                                       scaled);
  else
    k_build_xcat<double, double, false><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, bc_e, d, s, Xc, ldC, dims,
                                                                        scaled);
}
void launch_build_xcat(const StepGeom& G, const float* X, int ldX, const double* bc_e,
                       const double* d, const double* s, float* Xc, int ldC, const int* dims,
                       int scaled, hipStream_t st) {
  if (G.hllw)
    k_build_xcat<float, float, true><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, bc_e, d, s, Xc, ldC, dims,
                                                                     scaled);
  else
    k_build_xcat<float, float, false><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, bc_e, d, s, Xc, ldC, dims,
                                                                      scaled);
}
void launch_build_phcat(const StepGeom& G, const double* Ph, const double* pfac,
                        const double* bc_p, double* Pc, const int* dims, hipStream_t st) {
  const int tot = G.R2c * G.np;
  k_build_phcat<<<(tot + 255) / 256, 256, 0, st>>>(G, Ph, pfac, bc_p, Pc, dims);
}
void launch_build_thcat(const StepGeom& G, const double* Th, const double* tfac,
                        const double* bc_t, double* Tc, const int* dims, hipStream_t st) {
  const long long tot = (long long)G.R1c * G.nt * G.R2c;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 65535) blocks = 65535;
  k_build_thcat<<<blocks, 256, 0, st>>>(G, Th, tfac, bc_t, Tc, dims);
}
void launch_concat_dims(const StepGeom& G, int* dims, hipStream_t st) {
  k_concat_dims<<<1, 64, 0, st>>>(G, dims);
}
void launch_round_dims(int* dims, hipStream_t st) { k_round_dims<<<1, 64, 0, st>>>(dims); }
void launch_state_as_cat(const StepGeom& G, const double* Th, const double* Ph, double* Tc,
                         double* Pc, const int* dims, hipStream_t st) {
  const long long tot = (long long)G.r1c * G.nt * G.R2c;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  k_state_as_cat<<<blocks, 256, 0, st>>>(G, Th, Ph, Tc, Pc, dims);
}
template <typename TX>
static void energy_impl(const TX* X, int ldX, int ns, const double* Th, int nt, int ldb,
                        const double* Ph, int np, const double* w, const double* v, double* pv,
                        double* z, DimExpr r1, DimExpr r2, double inv_c, double* E,
                        const int* dims, int rcap1, int rcap2, hipStream_t st) {
  k_phi_moment<<<(rcap2 + 63) / 64, 64, 0, st>>>(Ph, np, v, pv, r2, dims);
  k_theta_moment<<<(rcap1 + 3) / 4, 256, 0, st>>>(Th, nt, ldb, w, pv, z, r1, r2, inv_c, dims);
  k_row_dot<TX><<<(ns + 3) / 4, 256, 0, st>>>(X, ldX, ns, z, r1, E, dims);
}
void launch_energy(const double* X, int ldX, int ns, const double* Th, int nt, int ldb,
                   const double* Ph, int np, const double* w, const double* v, double* pv,
                   double* z, DimExpr r1, DimExpr r2, double inv_c, double* E, const int* dims,
                   int rcap1, int rcap2, hipStream_t st) {
  energy_impl(X, ldX, ns, Th, nt, ldb, Ph, np, w, v, pv, z, r1, r2, inv_c, E, dims, rcap1, rcap2, st);
}
void launch_energy(const float* X, int ldX, int ns, const double* Th, int nt, int ldb,
                   const double* Ph, int np, const double* w, const double* v, double* pv,
                   double* z, DimExpr r1, DimExpr r2, double inv_c, double* E, const int* dims,
                   int rcap1, int rcap2, hipStream_t st) {
  energy_impl(X, ldX, ns, Th, nt, ldb, Ph, np, w, v, pv, z, r1, r2, inv_c, E, dims, rcap1, rcap2, st);
}
template <typename TX>
static void energy_xcat_impl(const StepGeom& G, const TX* X, int ldX, const double* bc_e,
                             const double* Tc, const double* Pc, const double* w, const double* v,
                             double* pv, double* z, DimExpr r2, double inv_c, double* E,
                             const int* dims, hipStream_t st) {
  const DimExpr ncol = dimv(D_RC1, 1, -G.nem);
  k_phi_moment<<<(G.R2c + 63) / 64, 64, 0, st>>>(Pc, G.np, v, pv, r2, dims);
  k_theta_moment<<<(G.R1c + 3) / 4, 256, 0, st>>>(Tc, G.nt, G.R2c, w, pv, z, ncol, r2, inv_c, dims);
  if (G.hllw) k_xcat_row_dot<TX, true><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, bc_e, z, E, dims);
  else k_xcat_row_dot<TX, false><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, bc_e, z, E, dims);
}
void launch_energy_xcat(const StepGeom& G, const double* X, int ldX, const double* bc_e,
                        const double* Tc, const double* Pc, const double* w, const double* v,
                        double* pv, double* z, DimExpr r2, double inv_c, double* E, double* Y,
                        double* Zt, const int* dims, hipStream_t st) {
  const DimExpr ncol = dimv(D_RC1, 1, -G.nem);
  k_phi_moment<<<(G.R2c + 63) / 64, 64, 0, st>>>(Pc, G.np, v, pv, r2, dims);
  k_theta_moment<<<(G.R1c + 3) / 4, 256, 0, st>>>(Tc, G.nt, G.R2c, w, pv, z, ncol, r2, inv_c, dims);
  constexpr int LDY = MAX_BLOCKS;
  k_z_blocks<<<(G.r1c * G.B + 255) / 256, 256, 0, st>>>(z, Zt, LDY, G.B, dims);
  gemm_tall(G.ns, X, ldX, Zt, LDY, Y, LDY, dimv(D_R1), dimc(G.B), G.r1c, LDY, dims, st);
  if (G.hllw) k_energy_stencil<true><<<(G.ns + 255) / 256, 256, 0, st>>>(G, Y, LDY, bc_e, z, E, dims);
  else k_energy_stencil<false><<<(G.ns + 255) / 256, 256, 0, st>>>(G, Y, LDY, bc_e, z, E, dims);
}
void launch_energy_xcat(const StepGeom& G, const float* X, int ldX, const double* bc_e,
                        const double* Tc, const double* Pc, const double* w, const double* v,
                        double* pv, double* z, DimExpr r2, double inv_c, double* E,
                        const int* dims, hipStream_t st) {
  energy_xcat_impl(G, X, ldX, bc_e, Tc, Pc, w, v, pv, z, r2, inv_c, E, dims, st);
}
void launch_hll_weights(const StepGeom& G, int dim, const double* rho, const double* kappa,
                        const double* kappa_s, double beta, const double* h, double thr, double* W,
                        hipStream_t st) {
  k_hll_weights<<<(G.ns + 255) / 256, 256, 0, st>>>(G, dim, rho, kappa, kappa_s, beta, h[0], h[1], h[2],
                                                    thr, W);
}
void launch_hll_inflow(const StepGeom& G, const double* bc_e0, const int* code, int nbc,
                       const double* W, double* bc_e, hipStream_t st) {
  if (nbc > 0) k_hll_inflow<<<(G.ns + 255) / 256, 256, 0, st>>>(G.ns, bc_e0, code, nbc, W, bc_e);
}
void launch_convert(const double* a, int lda, float* b, int ldb, int rows, int cols, hipStream_t st) {
  k_convert<double, float><<<1024, 256, 0, st>>>(a, lda, b, ldb, rows, cols);
}
void launch_convert(const float* a, int lda, double* b, int ldb, int rows, int cols, hipStream_t st) {
  k_convert<float, double><<<1024, 256, 0, st>>>(a, lda, b, ldb, rows, cols);
}
void launch_material(int ns, double c, double dt, double a_r, int coupled, const double* kappa,
                     const double* kappa_s, const double* rho, const double* cv, const double* T,
                     const double* Estar, double* Tdag, double* d, double* s, int* dims,
                     hipStream_t st) {
  k_material<<<(ns + 255) / 256, 256, 0, st>>>(ns, c, dt, a_r, coupled, kappa, kappa_s, rho, cv, T,
                                               Estar, Tdag, d, s, dims);
}
void launch_check_state(const double* X, const float* Xf, int ldX, int ns, const double* Th,
                        int nt, int r2c, const double* Ph, int np, const double* T, int* dims,
                        hipStream_t st) {
  if (Xf) k_check_state<float><<<1024, 256, 0, st>>>(Xf, ldX, ns, Th, nt, r2c, Ph, np, T, dims);
  else k_check_state<double><<<1024, 256, 0, st>>>(X, ldX, ns, Th, nt, r2c, Ph, np, T, dims);
}
template <typename TX>
static void source_cat_impl(const StepGeom& G, const TX* X, int ldX, const double* d,
                            const double* s, TX* Xc, int ldC, const double* Th, const double* Ph,
                            double* Tc, double* Pc, int* dims, hipStream_t st) {
  k_source_dims<<<1, 64, 0, st>>>(G, dims);
  k_source_xcat<TX><<<(G.ns + 3) / 4, 256, 0, st>>>(G, X, ldX, d, s, Xc, ldC, dims);
  const long long tot = (long long)(G.r1c + 1) * G.nt * G.R2c;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  k_source_angular<<<blocks, 256, 0, st>>>(G, Th, Ph, Tc, Pc, dims);
}
void launch_source_cat(const StepGeom& G, const double* X, int ldX, const double* d,
                       const double* s, double* Xc, int ldC, const double* Th, const double* Ph,
                       double* Tc, double* Pc, int* dims, hipStream_t st) {
  source_cat_impl(G, X, ldX, d, s, Xc, ldC, Th, Ph, Tc, Pc, dims, st);
}
void launch_source_cat(const StepGeom& G, const float* X, int ldX, const double* d,
                       const double* s, float* Xc, int ldC, const double* Th, const double* Ph,
                       double* Tc, double* Pc, int* dims, hipStream_t st) {
  source_cat_impl(G, X, ldX, d, s, Xc, ldC, Th, Ph, Tc, Pc, dims, st);
}
void launch_transport_dims(const StepGeom& G, int* dims, hipStream_t st) {
  k_transport_dims<<<1, 64, 0, st>>>(G, dims);
}
void launch_temperature(int ns, const double* rho, const double* cv, const double* Estar,
                        const double* Enew, double* T, hipStream_t st) {
  k_temperature<<<(ns + 255) / 256, 256, 0, st>>>(ns, rho, cv, Estar, Enew, T);
}
void launch_mside(int* dims, int ka, int kb, int km, int side, DimExpr abound, DimExpr bbound,
                  hipStream_t st) {
  k_mside<<<1, 64, 0, st>>>(dims, ka, kb, km, side, abound, bbound);
}
void launch_rank(const double* sig, int* dims, double* diag, const RankArgs& ra, hipStream_t st) {
  k_rank<<<1, 64, 0, st>>>(sig, dims, diag, ra);
}
void launch_svd_vectors(const double* Uc, int ldu, const double* sqc, double* Ur, int ldr,
                        double* Wm, int ldw, const int* dims, int ka, int kb, int side, int rn,
                        int zero, int rcap, hipStream_t st) {
  k_svd_vectors<<<rcap, 256, 0, st>>>(Uc, ldu, sqc, Ur, ldr, Wm, ldw, dims, ka, kb, side, rn, zero);
}
void launch_finish(int* dims, int* hist, int hmax, hipStream_t st) {
  k_finish<<<1, 64, 0, st>>>(dims, hist, hmax);
}
void launch_check_finite(const double* x, int n, int* dims, hipStream_t st) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_check_finite<<<blocks, 256, 0, st>>>(x, n, dims);
}

}  // namespace tt
