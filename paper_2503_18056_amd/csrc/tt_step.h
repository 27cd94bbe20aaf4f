// Geometry of one context and the launchers of the per-step kernels.
#pragma once

#include "../../include/tt.h"
#include "tt_internal.h"

namespace tt {

// Stencil of a transport block of the spatial core (Sec. 4.3): the base
// block X, the upwind differences X_i - X_{i-e} and X_{i+e} - X_i, the
// Rusanov central difference (X_{i+e} - X_{i-e}) / 2 and diffusion
// X_{i+e} - 2 X_i + X_{i-e}, and the HLL blocks of n >= 0 and n < 0:
// (alpha_hi - beta_lo) X_i + beta_hi X_{i+e} - alpha_lo X_{i-e} with the
// sign's weights at the cell's hi and lo faces (HllW).
enum : int { BK_BASE = 0, BK_MINUS = 1, BK_PLUS = 2, BK_CENTRAL = 3, BK_DIFF = 4, BK_HLL_POS = 5,
             BK_HLL_NEG = 6 };
constexpr int MAX_BLOCKS = 8;
// HLL face weights per axis and cell, four doubles at
// hllw[(axis * N_s + i) * 4]: alpha_p and beta_p (n >= 0) of the cell's hi
// face, then of its lo face.  The n < 0 pair is the swap: alpha_m = beta_p,
// beta_m = alpha_p.
enum : int { HLLW_AP_HI = 0, HLLW_BP_HI = 1, HLLW_AP_LO = 2, HLLW_BP_LO = 3 };

struct StepGeom {
  int ns, nx, ny, nz;
  int n[3], stride[3], periodic[3];
  int bclo[3], bchi[3];   // TT_BC_* of each face (axes >= dim: vacuum)
  int bkind[MAX_BLOCKS];  // BK_* of transport block b (b < B)
  int baxis[MAX_BLOCKS];  // its axis
  int nt, np;
  int B;        // transport blocks: 1 + 2 dim
  int nbc;      // rank-1 inflow terms
  int nem;      // emission block present (0/1)
  int r1c, r2c; // state rank capacities
  int R1c, R2c; // concatenated rank capacities
  const double* hllw;  // HLL face weights (device; null for the other fluxes)
};

struct RankArgs {
  int bond;           // 1 or 2
  int km, kc, ka, kb; // dims indices: Gram-of-M size, computed vectors, kept A, kept B
  int rn, zero, kea, keb, replay, rnt;
  int nt;
  double tol, eta;
  int rmax;
  int rdim;           // dims index of the Gram dimension R (resolution R u sigma_1^2 / sigma)
  int g_tail, g_sr, g_srp, g_rn, g_ka, g_kb;
};

void launch_build_xcat(const StepGeom& G, const double* X, int ldX, const double* bc_e,
                       const double* d, const double* s, double* Xc, int ldC, const int* dims,
                       int scaled, hipStream_t st);
// FP32-mixed form: X and X_cat stored in FP32 (FP64 arithmetic inside).
void launch_build_xcat(const StepGeom& G, const float* X, int ldX, const double* bc_e,
                       const double* d, const double* s, float* Xc, int ldC, const int* dims,
                       int scaled, hipStream_t st);
void launch_energy(const float* X, int ldX, int ns, const double* Th, int nt, int ldb,
                   const double* Ph, int np, const double* w, const double* v, double* pv,
                   double* z, DimExpr r1, DimExpr r2, double inv_c, double* E, const int* dims,
                   int rcap1, int rcap2, hipStream_t st);
// The post-transport energy density E = (1/c) X_cat z of the unscaled
// concatenation (transport and inflow columns; Tc, Pc its angular cores),
// with X_cat's entries formed from X on the fly.
// FP64: E* through Y = X Zt (Y: N_s x MAX_BLOCKS doubles, Zt: r1c x
// MAX_BLOCKS, the blocks of z as columns) and the stencils applied to Y.
void launch_energy_xcat(const StepGeom& G, const double* X, int ldX, const double* bc_e,
                        const double* Tc, const double* Pc, const double* w, const double* v,
                        double* pv, double* z, DimExpr r2, double inv_c, double* E, double* Y,
                        double* Zt, const int* dims, hipStream_t st);
void launch_energy_xcat(const StepGeom& G, const float* X, int ldX, const double* bc_e,
                        const double* Tc, const double* Pc, const double* w, const double* v,
                        double* pv, double* z, DimExpr r2, double inv_c, double* E,
                        const int* dims, hipStream_t st);
// HLL face weights (layout above) from rho, kappa and kappa_s: tau_c of
// eq. tauc with beta and the cell sizes h[3], then the weights of eq. hll
// with the wavespeeds of Sec. 3.1 (series forms below thr).
void launch_hll_weights(const StepGeom& G, int dim, const double* rho, const double* kappa,
                        const double* kappa_s, double beta, const double* h, double thr, double* W,
                        hipStream_t st);
// Inflow columns of the HLL flux: bc_e[c][i] = bc_e0[c][i] * W[ax_c][i][sel_c]
// with code[c] = 4 ax_c + sel_c (host-built; one code per rank-1 term).
void launch_hll_inflow(const StepGeom& G, const double* bc_e0, const int* code, int nbc,
                       const double* W, double* bc_e, hipStream_t st);
void launch_convert(const double* a, int lda, float* b, int ldb, int rows, int cols, hipStream_t st);
void launch_convert(const float* a, int lda, double* b, int ldb, int rows, int cols, hipStream_t st);
void launch_build_phcat(const StepGeom& G, const double* Ph, const double* pfac,
                        const double* bc_p, double* Pc, const int* dims, hipStream_t st);
void launch_build_thcat(const StepGeom& G, const double* Th, const double* tfac,
                        const double* bc_t, double* Tc, const int* dims, hipStream_t st);
void launch_concat_dims(const StepGeom& G, int* dims, hipStream_t st);
void launch_round_dims(int* dims, hipStream_t st);
void launch_state_as_cat(const StepGeom& G, const double* Th, const double* Ph, double* Tc,
                         double* Pc, const int* dims, hipStream_t st);
void launch_energy(const double* X, int ldX, int ns, const double* Th, int nt, int ldb,
                   const double* Ph, int np, const double* w, const double* v, double* pv,
                   double* z, DimExpr r1, DimExpr r2, double inv_c, double* E, const int* dims,
                   int rcap1, int rcap2, hipStream_t st);
// Source coefficients (Sec. 3.2): d = 1 / (1 + c dt rho (kappa + kappa_s)),
// s = d (c dt rho kappa_s J^{m+1} + c dt rho kappa (c/4pi) a_r T_dag^4); T_dag
// from Newton when coupled; kappa_s may be null (no scattering), else Estar
// is the post-transport energy density.
void launch_material(int ns, double c, double dt, double a_r, int coupled, const double* kappa,
                     const double* kappa_s, const double* rho, const double* cv, const double* T,
                     const double* Estar, double* Tdag, double* d, double* s, int* dims,
                     hipStream_t st);
void launch_temperature(int ns, const double* rho, const double* cv, const double* Estar,
                        const double* Enew, double* T, hipStream_t st);
void launch_mside(int* dims, int ka, int kb, int km, int side, DimExpr abound, DimExpr bbound,
                  hipStream_t st);
void launch_rank(const double* sig, int* dims, double* diag, const RankArgs& ra, hipStream_t st);
void launch_svd_vectors(const double* Uc, int ldu, const double* sqc, double* Ur, int ldr,
                        double* Wm, int ldw, const int* dims, int ka, int kb, int side, int rn,
                        int zero, int rcap, hipStream_t st);
// Close a step (state ranks <- new ranks); with hist, record them in the
// history slot dims[D_HSLOT] while it is below hmax.
void launch_finish(int* dims, int* hist, int hmax, hipStream_t st);
void launch_check_finite(const double* x, int n, int* dims, hipStream_t st);
// Finiteness of the state: X (N_s x r1 live, ld ldX), Theta (r1 x nt x r2
// live, ld r2c), Phi (r2 x np) and T (N_s); raises FLAG_NONFINITE.
void launch_check_state(const double* X, const float* Xf, int ldX, int ns, const double* Th,
                        int nt, int r2c, const double* Ph, int np, const double* T, int* dims,
                        hipStream_t st);
// Concatenation of the source update of the two-rounding schedule
// (Sec. 4.2): X_cat = [d X, s], Theta_cat = blockdiag(Theta, 1),
// Phi_cat = [Phi; 1] (the source column only when G.nem); sets dims[RC1],
// dims[RC2] to r + nem.
void launch_source_cat(const StepGeom& G, const double* X, int ldX, const double* d,
                       const double* s, double* Xc, int ldC, const double* Th, const double* Ph,
                       double* Tc, double* Pc, int* dims, hipStream_t st);
void launch_source_cat(const StepGeom& G, const float* X, int ldX, const double* d,
                       const double* s, float* Xc, int ldC, const double* Th, const double* Ph,
                       double* Tc, double* Pc, int* dims, hipStream_t st);
// dims[RC1], dims[RC2] for the transport-only concatenation (no source
// column) of the two-rounding schedule.
void launch_transport_dims(const StepGeom& G, int* dims, hipStream_t st);

// ---- adjoint (reverse sweep) kernels -----------------------------------------
void launch_svd_adj_inner(const double* G1, const double* G2, int ldg, const double* sv,
                          const double* sbar, double* out, int ldo, const int* dims, int kc_idx,
                          int r_idx, int cap, hipStream_t s);
void launch_copy_cond(const double* src, int lds, double* dst, int ldd, const int* dims,
                      int rows_idx, int kc_idx, int side_idx, int side, int cap, hipStream_t s);
void launch_gauge_pair(double* U, int ldu, double* V, int ldv, const int* dims, int ka_idx,
                       int kb_idx, int kc_idx, int side_idx, int cap, hipStream_t s);
void launch_add_colscaled(const double* X, int ldx, const double* sc, double* Y, int ldy,
                          const int* dims, DimExpr r, int c_idx, int cap, hipStream_t s);
void launch_zero_block(double* A, int lda, const int* dims, DimExpr r, DimExpr cdim, long long cap,
                       hipStream_t s);
void launch_xcat_adjoint(const StepGeom& G, const double* X, int ldX, const double* bc_e,
                         const double* d, const double* dd, const double* ds, const double* Xcb,
                         int ldC, double* Xb, double* kbar, const int* dims, hipStream_t s);
void launch_cat_angular_adjoint(const StepGeom& G, const double* tfac, const double* pfac,
                                const double* Thcb, const double* Phcb, double* Thb, double* Phb,
                                const int* dims, hipStream_t s);
void launch_source_derivs(int ns, double c, double dt, double a_r, const double* rho,
                          const double* T, const double* d, double* dd, double* ds, hipStream_t s);
void launch_seed(const double* w, const double* z, const double* X, int ldX, int ns,
                 const double* wq, const double* v, const double* pv, const double* Th, int nt,
                 int r2c, int np, int r1c, double scale_x, double scale_ang, double* xg,
                 double* Xb, double* Thb, double* Phb, const int* dims, hipStream_t s);
void launch_wdot(const double* w, const double* E, int ns, double* out, hipStream_t s);
void launch_replay_from_hist(int* dims, const int* hist, int m, hipStream_t s);

}  // namespace tt
