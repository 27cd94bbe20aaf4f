// Reverse-mode gradient of a detector loss L = dV sum_i w_i E_i(final) with
// respect to the per-cell absorption opacity kappa, over the steps taken
// since tt_set_cores with frozen material (Sec. 3.2: kappa enters each step
// through d = 1/(1 + c dt rho kappa) on the transport and inflow blocks and
// through the emission term s).
//
// Ranks are frozen at the forward's: each step's truncation ranks are
// replayed from the rank history, so the step is a smooth map of its input
// cores and of kappa, and the reverse sweep is the adjoint of that map.  The
// cotangents are dense cores (X bar, Theta bar, Phi bar); the sweep runs each
// piece of the step backwards:
//   spatial core update  X' = X_cat P1            (App. A.2, A' = A V_A S_A^-1 U)
//   angular cores        Theta' = M_upd Theta_cat, then the bond-2 update
//   Gram-SVD truncation  (App. A.2) as the truncated SVD of the bond's
//                        matrix, through the singular-vector perturbation
//                        formula (see bond_adjoint)
//   concatenation        transposed stencils (Sec. 4.3) and the kappa terms.
//
// The FP32-mixed form is recomputed in its own precision (so the tape is
// reproduced exactly) and reversed in FP64 on FP64 copies of its FP32-stored
// X and X_cat: the result is the derivative of the step map at the mixed
// trajectory.
//
// Memory: a checkpoint of the state every ckpt_every steps; a segment's
// states are recomputed from its checkpoint, then each step is recomputed
// once more right before its reverse.  Every
// reduction in the forward has a fixed order, so recomputation reproduces the
// taped forward bit for bit.
#include <math.h>

#include <algorithm>

#include "tt_ctx.h"

namespace tt {

namespace {

#define GCHK(ctx, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ctx_fail(ctx, TT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The current state (X or X_f, Theta, Phi, ranks) to or from a stored slot.
hipError_t copy_state(tt_ctx* c, char* X, double* Th, double* Ph, int* R, bool save) {
  const GradBufs& g = c->gb;
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  hipStream_t s = c->st;
  char* cx = c->mixed ? reinterpret_cast<char*>(c->Xf) : reinterpret_cast<char*>(c->X);
  hipError_t e;
  if (save) {
    if ((e = hipMemcpyAsync(X, cx, g.xbytes, k, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(Th, c->Th, g.ths * 8, k, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(Ph, c->Ph, g.phs * 8, k, s)) != hipSuccess) return e;
    return hipMemcpyAsync(R, c->dims + D_R1, 2 * sizeof(int), k, s);
  }
  if ((e = hipMemcpyAsync(cx, X, g.xbytes, k, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->Th, Th, g.ths * 8, k, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->Ph, Ph, g.phs * 8, k, s)) != hipSuccess) return e;
  return hipMemcpyAsync(c->dims + D_R1, R, 2 * sizeof(int), k, s);
}

// Mixed form: FP64 copies of the FP32-stored X (and, after a step, X_cat and
// X') for the reverse products (exact: every FP32 value is an FP64 value).
void widen_state(tt_ctx* c, bool step_done) {
  if (!c->mixed) return;
  launch_convert(c->Xf, c->ldX, c->X, c->ldX, c->ns, c->ldX, c->st);
  if (!step_done) return;
  launch_convert(c->Xcatf, c->ldC, c->Xcat, c->ldC, c->ns, c->ldC, c->st);
  launch_convert(c->Xnf, c->ldX, c->Xn, c->ldX, c->ns, c->ldX, c->st);
}

void swap_state(tt_ctx* c) {
  if (c->mixed) std::swap(c->Xf, c->Xnf);
  else std::swap(c->X, c->Xn);
}

// out (m x n, ldo) = A^T B + beta out, contracted over `rows` rows (A: rows x m,
// B: rows x n), split over row slices into fixed-order partial sums.
void contract_rows(tt_ctx* c, const double* A, int lda, const double* B, int ldb, double* out,
                   int ldo, DimExpr m, DimExpr n, DimExpr rows, int mcap, int ncap, int rowcap,
                   double beta = 0.0) {
  GradBufs& g = c->gb;
  const size_t tile = (size_t)mcap * ncap;
  const int zmax = (int)std::max<size_t>(1, g.part_n / tile);
  int ks = std::max(g.ksl, (rowcap + zmax - 1) / zmax);
  ks = (ks + 15) / 16 * 16;
  const int nz = std::max(1, (rowcap + ks - 1) / ks);
  GemmDesc p = gd(A, lda, 1, B, ldb, 0, g.part, ncap, m, n, rows);
  p.ksplit = ks;
  p.sC = (long long)tile;
  gemm(p, mcap, ncap, nz, c->dims, c->st);
  sum_partials(g.part, (long long)tile, nz, out, ldo, ncap, m, n, mcap, ncap, c->dims, c->st, beta);
}

// Factors of one bond's truncation that the reverse needs, from the forward's
// eigen slots: U_M (kA x kc) and V_M (kB x kc), the kc resolved singular
// vectors of M on both sides with the forward's signs (side 1: U_M = M V_M
// S^-1, sign-fixed on U_M), and Y = V_A S_A U_M S^-1 (R x kc), for which
// A^T U = Y S with U = A V_A S_A^-1 U_M the left singular vectors of K = A W.
struct BondF {
  double *U, *V, *Y;
};

void bond_factors(tt_ctx* c, int bond, const EigSlot& ea, const EigSlot& em, int Rcap, int Rdim,
                  const BondF& f) {
  hipStream_t s = c->st;
  const int N = c->N;
  int* d = c->dims;
  const int ka = bond == 1 ? D_KA1 : D_KA2, kb = bond == 1 ? D_KB1 : D_KB2;
  const int kc = bond == 1 ? D_KC1 : D_KC2;
  const int side = bond == 1 ? D_SIDE1 : D_SIDE2;
  const double* M = bond == 1 ? c->M1 : c->M2;
  launch_copy_cond(em.V, N, f.U, N, d, ka, kc, side, 0, N, s);
  launch_copy_cond(em.V, N, f.V, N, d, kb, kc, side, 1, N, s);
  GemmDesc v = gd(M, Rcap, 1, f.U, N, 0, f.V, N, dimv(kb), dimv(kc), dimv(ka));
  v.colscale = em.isq;
  v.cond_idx = side; v.cond_val = 0;
  gemm(v, N, N, 1, d, s);
  GemmDesc u = gd(M, Rcap, 0, f.V, N, 0, f.U, N, dimv(ka), dimv(kc), dimv(kb));
  u.colscale = em.isq;
  u.cond_idx = side; u.cond_val = 1;
  gemm(u, N, N, 1, d, s);
  launch_gauge_pair(f.U, N, f.V, N, d, ka, kb, kc, side, N, s);
  GemmDesc y = gd(ea.V, N, 0, f.U, N, 0, f.Y, N, dimv(Rdim), dimv(kc), dimv(ka));
  y.kscale = ea.sq;
  y.colscale = em.isq;
  gemm(y, Rcap, N, 1, d, s);
}

// Reverse of one Gram-SVD truncation, taken as the map it computes with the
// rank r frozen: for K = A W (A: rows x R; W, the other side, enters only
// through its Gram G_B = W W^T),
//   A' = U_r   (the r leading left singular vectors of K; A' = A P),
//   M_upd = A'^T A   (up to the clipped, numerically null part of W).
// Given A' bar (in Abt) and M_upd bar (g.Mub), with U S V^T the kc singular
// triplets that the forward resolved (V = W^T Y):
//   A' bar_tot = A' bar + A M_upd bar^T,   A bar = A' M_upd bar + Z Y^T G_B,
//   K bar = Z V^T,  W bar = H W,  H = (A_e^T Z) Y^T,   Z = U In + A' bar_tot S_r^-1,
//   In = (F o (G1 - G1^T)) S - G1 S_r^-1,  G1 = U^T A' bar_tot,  F_ij = 1/(s_j^2 - s_i^2)
// (the truncated-SVD perturbation result with the complement of the kc
// triplets treated as null space).  A_e is the A through which K depends on
// W: A itself at bond 1; at bond 2, where A = Theta' = M_upd1 Theta_cat and
// the forward's M_upd1 carries bond 1's projector onto the range of its W,
// A_e = (X_cat^T X')^T Theta_cat (the same K, without that projector).  The
// direct cotangent of W from M_upd is A_e^T A' (in g.Mt).  Nothing here
// divides by a Gram eigenvalue: kept eigenpairs of G_A and G_B near the
// rounding floor, whose individual derivatives are unbounded, never enter on
// their own.  Outputs: Abt (A' bar_tot), Ab (A bar, rows x R), g.Hm (H,
// R x R); g.Mt only when Ae is given.
void bond_adjoint(tt_ctx* c, int bond, const double* A, int lda, const double* Ae, int ldae,
                  DimExpr rows, int rowcap, const double* Ap, int ldap, double* Abt, int ldabt,
                  double* Ab, int ldab, double* Uh, int lduh, const EigSlot& ea,
                  const EigSlot& em, const BondF& f, const double* GB, int Rcap, int rcap,
                  int Rdim) {
  GradBufs& g = c->gb;
  hipStream_t s = c->st;
  const int N = c->N;
  int* d = c->dims;
  const int kc = bond == 1 ? D_KC1 : D_KC2, rn = bond == 1 ? D_R1N : D_R2N;
  const int ka = bond == 1 ? D_KA1 : D_KA2;
  const DimExpr R = dimv(Rdim);
  // M_upd = A'^T A
  {
    GemmDesc t = gd(A, lda, 0, g.Mub, Rcap, 1, Abt, ldabt, rows, dimv(rn), R);
    t.beta = 1.0;
    gemm(t, rowcap, rcap, 1, d, s);
    gemm(gd(Ap, ldap, 0, g.Mub, Rcap, 0, Ab, ldab, rows, R, dimv(rn)), rowcap, Rcap, 1, d, s);
  }
  // left singular vectors of K: U = A (V_A S_A^-1 U_M)
  {
    GemmDesc p = gd(ea.V, N, 0, f.U, N, 0, g.Pf, N, R, dimv(kc), dimv(ka));
    p.kscale = ea.isq;
    gemm(p, Rcap, N, 1, d, s);
    gemm(gd(A, lda, 0, g.Pf, N, 0, Uh, lduh, rows, dimv(kc), R), rowcap, Rcap, 1, d, s);
  }
  // G1 = U^T A' bar_tot (columns r..kc zero), In
  launch_zero_block(g.G1, N, d, dimv(kc), dimv(kc), (long long)N * N, s);
  contract_rows(c, Uh, lduh, Abt, ldabt, g.G1, N, dimv(kc), dimv(rn), rows, Rcap, rcap, rowcap);
  launch_svd_adj_inner(g.G1, nullptr, N, em.sq, nullptr, g.In, N, d, kc, rn, N, s);
  // A bar += U (In Y^T G_B) + A' bar_tot S_r^-1 (Y^T G_B)_r
  {
    gemm(gd(f.Y, N, 1, GB, N, 0, g.YG, N, dimv(kc), R, R), N, Rcap, 1, d, s);
    gemm(gd(g.In, N, 0, g.YG, N, 0, g.Qm, N, dimv(kc), R, dimv(kc)), N, Rcap, 1, d, s);
    GemmDesc a = gd(Uh, lduh, 0, g.Qm, N, 0, Ab, ldab, rows, R, dimv(kc));
    a.beta = 1.0;
    gemm(a, rowcap, Rcap, 1, d, s);
    GemmDesc b = gd(Abt, ldabt, 0, g.YG, N, 0, Ab, ldab, rows, R, dimv(rn));
    b.kscale = em.isq;
    b.beta = 1.0;
    gemm(b, rowcap, Rcap, 1, d, s);
  }
  // H = (A_e^T Z) Y^T
  if (!Ae) {  // A^T Z = Y S In + (A^T A' bar_tot) S_r^-1
    contract_rows(c, A, lda, Abt, ldabt, g.Ta, N, R, dimv(rn), rows, Rcap, rcap, rowcap);
    GemmDesc z = gd(f.Y, N, 0, g.In, N, 0, g.AZ, N, R, dimv(kc), dimv(kc));
    z.kscale = em.sq;
    gemm(z, Rcap, N, 1, d, s);
    launch_add_colscaled(g.Ta, N, em.isq, g.AZ, N, d, R, rn, N, s);
  } else {  // Z formed explicitly (rows are few at bond 2)
    gemm(gd(Uh, lduh, 0, g.In, N, 0, g.Z2, Rcap, rows, dimv(kc), dimv(kc)), rowcap, Rcap, 1, d, s);
    launch_add_colscaled(Abt, ldabt, em.isq, g.Z2, Rcap, d, rows, rn, rowcap > Rcap ? rowcap : Rcap, s);
    contract_rows(c, Ae, ldae, g.Z2, Rcap, g.AZ, N, R, dimv(kc), rows, Rcap, Rcap, rowcap);
    contract_rows(c, Ae, ldae, Ap, ldap, g.Mt, N, R, dimv(rn), rows, Rcap, rcap, rowcap);
  }
  gemm(gd(g.AZ, N, 0, f.Y, N, 1, g.Hm, N, R, R, dimv(kc)), Rcap, Rcap, 1, d, s);
}

// Reverse of one recomputed step: (Xb, Thb, Phb) = cotangents of the step's
// output cores; writes those of its input cores to (Xnb, Thnb, Phnb) and adds
// the step's kappa terms to kbar.
void reverse_step(tt_ctx* c) {
  GradBufs& g = c->gb;
  hipStream_t s = c->st;
  const int N = c->N, nt = c->nt, np = c->np, ns = c->ns;
  const int R1c = c->R1c, R2c = c->R2c, r1c = c->r1c, r2c = c->r2c;
  const int ldX = c->ldX, ldC = c->ldC, ldT = nt * R2c;
  int* d = c->dims;
  const BondF f1{g.U1, g.V1, g.Y1}, f2{g.U2, g.V2, g.Y2};
  bond_factors(c, 1, c->E[0], c->E[3], R1c, D_RC1, f1);
  bond_factors(c, 2, c->E[4], c->E[5], R2c, D_RC2, f2);
  // Mt1 = X_cat^T X' = Y1_r S_r;  A_e of bond 2 = Mt1^T Theta_cat (laid out as Theta_p)
  launch_zero_block(g.Mt1, N, d, dimv(D_RC1), dimv(D_R1N), (long long)N * N, s);
  launch_add_colscaled(g.Y1, N, c->E[3].sq, g.Mt1, N, d, dimv(D_RC1), D_R1N, N, s);
  {
    GemmDesc e = gd(g.Mt1, N, 1, c->Thcat, ldT, 0, g.A2e, ldT, dimv(D_R1N), dimv(D_RC2), dimv(D_RC1));
    e.sB = e.sC = R2c;
    gemm(e, r1c, R2c, nt, d, s);
  }
  // ---- bond 2: A2 = Theta_p (r1' N_theta x R2), W = Phi_cat; Theta'' = A2 P2
  // (in Th), Phi' = M_upd2 Phi_cat
  gemm(gd(g.Phb, np, 0, c->Phcat, np, 1, g.Mub, R2c, dimv(D_R2N), dimv(D_RC2), dimc(np)), r2c, R2c,
       1, d, s);
  hipMemcpyAsync(g.Tbt, g.Thb, g.ths * 8, hipMemcpyDeviceToDevice, s);
  gemm(gd(c->Phcat, np, 0, c->Phcat, np, 1, g.GBs, N, dimv(D_RC2), dimv(D_RC2), dimc(np)), R2c, R2c,
       1, d, s);
  bond_adjoint(c, 2, c->Thp, R2c, g.A2e, R2c, dimv(D_R1NT), r1c * nt, c->Th, r2c, g.Tbt, r2c, g.A2b,
               R2c, g.Uh2, R2c, c->E[4], c->E[5], f2, g.GBs, R2c, r2c, D_RC2);
  // Phi_cat bar = Mt2 Phi' bar + H2 Phi_cat
  gemm(gd(g.Mt, N, 0, g.Phb, np, 0, g.Phcb, np, dimv(D_RC2), dimc(np), dimv(D_R2N)), R2c, np, 1, d, s);
  {
    GemmDesc p = gd(g.Hm, N, 0, c->Phcat, np, 0, g.Phcb, np, dimv(D_RC2), dimc(np), dimv(D_RC2));
    p.beta = 1.0;
    gemm(p, R2c, np, 1, d, s);
  }
  // ---- bond 1: A = X_cat, W = Theta_cat Phi_cat; X' = X_cat P1 (in Xn),
  // Theta_p = M_upd1 Theta_cat
  {  // M_upd1 bar = sum_l Theta_p bar_l Theta_cat_l^T (one partial per ordinate)
    GemmDesc m = gd(g.A2b, ldT, 0, c->Thcat, ldT, 1, g.part, R1c, dimv(D_R1N), dimv(D_RC1), dimv(D_RC2));
    m.sA = m.sB = R2c;
    m.sC = (long long)r1c * R1c;
    gemm(m, r1c, R1c, nt, d, s);
    sum_partials(g.part, (long long)r1c * R1c, nt, g.Mub, R1c, R1c, dimv(D_R1N), dimv(D_RC1), r1c,
                 R1c, d, s);
  }
  {  // Theta_cat bar_l = Mt1 Theta_p bar_l  (M_upd1 taken as X'^T X_cat)
    GemmDesc t = gd(g.Mt1, N, 0, g.A2b, ldT, 0, g.Thcb, ldT, dimv(D_RC1), dimv(D_RC2), dimv(D_R1N));
    t.sB = t.sC = R2c;
    gemm(t, R1c, R2c, nt, d, s);
  }
  {  // G_B1 = sum_l T1_l Theta_cat_l^T (T1 = Theta_cat G_R3), as in the forward
    GemmDesc b = gd(c->T1, ldT, 0, c->Thcat, ldT, 1, g.part, R1c, dimv(D_RC1), dimv(D_RC1), dimv(D_RC2));
    b.sA = b.sB = R2c;
    b.sC = (long long)R1c * R1c;
    gemm(b, R1c, R1c, nt, d, s);
    sum_partials(g.part, (long long)R1c * R1c, nt, g.GBs, N, R1c, dimv(D_RC1), dimv(D_RC1), R1c,
                 R1c, d, s);
  }
  hipMemcpyAsync(g.Xbt, g.Xb, g.xs * 8, hipMemcpyDeviceToDevice, s);
  bond_adjoint(c, 1, c->Xcat, ldC, nullptr, 0, dimc(ns), ns, c->Xn, ldX, g.Xbt, ldX, g.Xcb, ldC,
               g.Uh, ldC, c->E[0], c->E[3], f1, g.GBs, R1c, r1c, D_RC1);
  {  // W bar = H1 W:  Theta_cat bar_l += H1 T1_l,  Phi_cat bar += (sum_l Theta_cat_l^T H1 Theta_cat_l) Phi_cat
    GemmDesc t = gd(g.Hm, N, 0, c->T1, ldT, 0, g.Thcb, ldT, dimv(D_RC1), dimv(D_RC2), dimv(D_RC1));
    t.sB = t.sC = R2c;
    t.beta = 1.0;
    gemm(t, R1c, R2c, nt, d, s);
    GemmDesc y = gd(g.Hm, N, 0, c->Thcat, ldT, 0, g.Y, ldT, dimv(D_RC1), dimv(D_RC2), dimv(D_RC1));
    y.sB = y.sC = R2c;
    gemm(y, R1c, R2c, nt, d, s);
    contract_rows(c, c->Thcat, R2c, g.Y, R2c, g.S3, N, dimv(D_RC2), dimv(D_RC2), dimv(D_RC1, nt),
                  R2c, R2c, R1c * nt);
    GemmDesc p = gd(g.S3, N, 0, c->Phcat, np, 0, g.Phcb, np, dimv(D_RC2), dimc(np), dimv(D_RC2));
    p.beta = 1.0;
    gemm(p, R2c, np, 1, d, s);
  }
  // ---- concatenation of the step operator's blocks
  launch_xcat_adjoint(c->G, c->X, ldX, c->bc_e, c->d, g.dd, g.ds, g.Xcb, ldC, g.Xnb, g.kbar, d, s);
  launch_cat_angular_adjoint(c->G, c->tfac, c->pfac, g.Thcb, g.Phcb, g.Thnb, g.Phnb, d, s);
}

}  // namespace

void grad_carve(tt_ctx* c, Carve& cv) {
  GradBufs& g = c->gb;
  g.on = true;
  g.K = c->cfg.ckpt_every;
  const int ms = std::max(1, c->cfg.max_steps);
  g.nck = (ms + g.K - 1) / g.K;
  const int kseg = std::min(g.K, ms);
  const int ns = c->ns, nt = c->nt, np = c->np, N = c->N;
  g.xs = (size_t)ns * c->ldX;
  g.xbytes = g.xs * (c->mixed ? sizeof(float) : sizeof(double));
  g.ths = (size_t)c->r1c * nt * c->r2c;
  g.phs = (size_t)c->r2c * np;
  g.ckX = cv.take<char>(g.nck * g.xbytes);
  g.ckTh = cv.take<double>(g.nck * g.ths);
  g.ckPh = cv.take<double>(g.nck * g.phs);
  g.ckR = cv.take<int>(2 * (size_t)g.nck);
  g.sgX = cv.take<char>(kseg * g.xbytes);
  g.sgTh = cv.take<double>(kseg * g.ths);
  g.sgPh = cv.take<double>(kseg * g.phs);
  g.sgR = cv.take<int>(2 * (size_t)kseg);
  g.fX = cv.take<char>(g.xbytes);
  g.fTh = cv.take<double>(g.ths);
  g.fPh = cv.take<double>(g.phs);
  g.fR = cv.take<int>(2);
  g.Xb = cv.take<double>(g.xs);
  g.Xnb = cv.take<double>(g.xs);
  g.Thb = cv.take<double>(g.ths);
  g.Thnb = cv.take<double>(g.ths);
  g.Phb = cv.take<double>(g.phs);
  g.Phnb = cv.take<double>(g.phs);
  g.Xcb = cv.take<double>((size_t)ns * c->ldC);
  g.Thcb = cv.take<double>((size_t)c->R1c * nt * c->R2c);
  g.Phcb = cv.take<double>((size_t)c->R2c * np);
  g.A2b = cv.take<double>((size_t)c->r1c * nt * c->R2c);
  double** vecs_ns[] = {&g.kbar, &g.dd, &g.ds, &g.wdet};
  for (double** p : vecs_ns) *p = cv.take<double>(ns);
  g.xg = cv.take<double>(c->r1c + 8);
  g.loss = cv.take<double>(8);
  g.Mub = cv.take<double>(std::max((size_t)c->R1c * c->r1c, (size_t)c->R2c * c->r2c));
  g.Xbt = cv.take<double>(g.xs);
  g.Tbt = cv.take<double>(g.ths);
  g.Uh = cv.take<double>((size_t)ns * c->ldC);
  g.Uh2 = cv.take<double>((size_t)c->r1c * nt * c->R2c);
  g.Z2 = cv.take<double>((size_t)c->r1c * nt * c->R2c);
  g.A2e = cv.take<double>((size_t)c->r1c * nt * c->R2c);
  double** mats[] = {&g.U1, &g.V1, &g.Y1, &g.U2, &g.V2, &g.Y2, &g.G1, &g.In, &g.Pf, &g.YG,
                     &g.Qm, &g.AZ, &g.Ta, &g.Hm, &g.GBs, &g.S3, &g.Mt, &g.Mt1};
  for (double** p : mats) *p = cv.take<double>((size_t)N * N);
  g.Y = cv.take<double>((size_t)c->R1c * nt * c->R2c);
  // row-sliced contractions: at most 64 slices of a multiple of 16 rows
  g.ksl = ((ns + 63) / 64 + 15) / 16 * 16;
  g.part_n = std::max({(size_t)64 * N * std::max(c->r1c, c->r2c), (size_t)nt * c->R1c * c->R1c,
                       (size_t)64 * c->R2c * c->R2c});
  g.part = cv.take<double>(g.part_n);
}

hipError_t grad_record(tt_ctx* c) {
  GradBufs& g = c->gb;
  if (c->nhist % g.K) return hipSuccess;
  const int slot = c->nhist / g.K;
  if (slot >= g.nck) return hipSuccess;
  return copy_state(c, g.ckX + slot * g.xbytes, g.ckTh + slot * g.ths, g.ckPh + slot * g.phs,
                    g.ckR + 2 * slot, true);
}

}  // namespace tt

using namespace tt;

extern "C" tt_status tt_grad(tt_ctx* c, const double* detector_w, double loss_bar, double* loss_out,
                             double* dkappa_dev) {
  if (!c) return ctx_fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (!detector_w || !dkappa_dev) return ctx_fail(c, TT_ERR_INVALID_ARG, "null argument");
  GradBufs& g = c->gb;
  if (!g.on) return ctx_fail(c, TT_ERR_STATE, "no tape: the context was created with ckpt_every <= 0");
  if (c->poisoned) return ctx_fail(c, TT_ERR_STATE, "context poisoned by an earlier numerical failure");
  if (c->nhist == 0) return ctx_fail(c, TT_ERR_STATE, "no steps taped since tt_set_cores");
  if (g.stale)
    return ctx_fail(c, TT_ERR_STATE,
                    "the tape is stale: tt_set_kappa or tt_round after the recorded steps");
  hipStream_t s = c->st;
  const int nsteps = c->nhist, ns = c->ns;
  const tt_config& cf = c->cfg;
  const double dV = (cf.lx / cf.nx) * (cf.ly / cf.ny) * (cf.dim == 3 ? cf.lz / cf.nz : 1.0);
  int* d = c->dims;
  // final state: kept aside, restored at the end
  GCHK(c, copy_state(c, g.fX, g.fTh, g.fPh, g.fR, true));
  GCHK(c, hipMemcpyAsync(g.wdet, detector_w, (size_t)ns * 8, hipMemcpyHostToDevice, s));
  // loss and its seed
  widen_state(c, false);
  launch_energy(c->X, c->ldX, ns, c->Th, c->nt, c->r2c, c->Ph, c->np, c->w, c->v, c->pv, c->z,
                dimv(D_R1), dimv(D_R2), 1.0 / cf.c, c->Enew, d, c->r1c, c->r2c, s);
  launch_wdot(g.wdet, c->Enew, ns, g.loss, s);
  launch_seed(g.wdet, c->z, c->X, c->ldX, ns, c->w, c->v, c->pv, c->Th, c->nt, c->r2c, c->np,
              c->r1c, loss_bar * dV, loss_bar * dV / cf.c, g.xg, g.Xb, g.Thb, g.Phb, d, s);
  GCHK(c, hipMemsetAsync(g.kbar, 0, (size_t)ns * 8, s));
  launch_source_derivs(ns, cf.c, c->dt, cf.a_r, c->rho, c->T, c->d, g.dd, g.ds, s);
  const int nseg = (nsteps + g.K - 1) / g.K;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int m0 = seg * g.K, m1 = std::min(m0 + g.K, nsteps);
    GCHK(c, copy_state(c, g.ckX + seg * g.xbytes, g.ckTh + seg * g.ths, g.ckPh + seg * g.phs,
                       g.ckR + 2 * seg, false));
    // the segment's states m0 .. m1-1
    for (int m = m0; m < m1; ++m) {
      const int k = m - m0;
      GCHK(c, copy_state(c, g.sgX + k * g.xbytes, g.sgTh + k * g.ths, g.sgPh + k * g.phs,
                         g.sgR + 2 * k, true));
      if (m == m1 - 1) break;
      launch_replay_from_hist(d, c->hist, m, s);
      step_body_frozen(c);
      launch_finish(d, nullptr, 0, s);
      swap_state(c);
    }
    for (int m = m1 - 1; m >= m0; --m) {
      const int k = m - m0;
      GCHK(c, copy_state(c, g.sgX + k * g.xbytes, g.sgTh + k * g.ths, g.sgPh + k * g.phs,
                         g.sgR + 2 * k, false));
      launch_replay_from_hist(d, c->hist, m, s);
      step_body_frozen(c);
      widen_state(c, true);
      reverse_step(c);
      std::swap(g.Xb, g.Xnb);
      std::swap(g.Thb, g.Thnb);
      std::swap(g.Phb, g.Phnb);
    }
  }
  // back to the final state, rank rule no longer replayed
  GCHK(c, copy_state(c, g.fX, g.fTh, g.fPh, g.fR, false));
  GCHK(c, hipMemsetAsync(d + D_REPLAY1, 0, 2 * sizeof(int), s));
  GCHK(c, hipMemcpyAsync(dkappa_dev, g.kbar, (size_t)ns * 8, hipMemcpyDeviceToDevice, s));
  double L = 0.0;
  GCHK(c, hipMemcpyAsync(&L, g.loss, 8, hipMemcpyDeviceToHost, s));
  GCHK(c, hipGetLastError());
  GCHK(c, hipStreamSynchronize(s));
  if (loss_out) *loss_out = L * dV;
  int flag = 0;
  GCHK(c, hipMemcpy(&flag, d + D_FLAG, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return ctx_fail(c, TT_ERR_NUMERIC, "numerical failure during the recomputation");
  return TT_OK;
}
