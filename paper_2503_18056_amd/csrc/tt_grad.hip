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
//   Gram-SVD truncation  (App. A.2) through the eigen and SVD perturbation
//                        formulas, with every eigenvector of each Gram
//   Gram products        A bar += A (G bar + G bar^T)
//   concatenation        transposed stencils (Sec. 4.3) and the kappa terms.
//
// Memory: a checkpoint of the state every ckpt_every steps; a segment's
// states are recomputed from its checkpoint, then each step is recomputed
// once more, with all eigenvectors, right before its reverse.  Every
// reduction in the forward has a fixed order, so recomputation reproduces the
// taped forward bit for bit.
#include <math.h>

#include <algorithm>

#include "tt_ctx.h"

namespace tt {

namespace {

constexpr int KSPLIT_GR3 = 512;  // split of the R1 N_theta-long contraction (G_R3 bar)

#define GCHK(ctx, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ctx_fail(ctx, TT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int nsplit_gr3(const tt_ctx* c) { return (c->R1c * c->nt + KSPLIT_GR3 - 1) / KSPLIT_GR3; }

hipError_t copy_state(tt_ctx* c, double* X, double* Th, double* Ph, int* R, bool save) {
  const GradBufs& g = c->gb;
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  hipStream_t s = c->st;
  hipError_t e;
  if (save) {
    if ((e = hipMemcpyAsync(X, c->X, g.xs * 8, k, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(Th, c->Th, g.ths * 8, k, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(Ph, c->Ph, g.phs * 8, k, s)) != hipSuccess) return e;
    return hipMemcpyAsync(R, c->dims + D_R1, 2 * sizeof(int), k, s);
  }
  if ((e = hipMemcpyAsync(c->X, X, g.xs * 8, k, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->Th, Th, g.ths * 8, k, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->Ph, Ph, g.phs * 8, k, s)) != hipSuccess) return e;
  return hipMemcpyAsync(c->dims + D_R1, R, 2 * sizeof(int), k, s);
}

// G bar of a symmetric eigendecomposition G = V diag(lambda) V^T from the
// cotangents of its kept pairs (Vb: R x k, lb: k), with every eigenpair:
//   G bar = sym( V_all (diag(lb) + F o (V_all^T Vb)) V_k^T ),
// F_ij = 1/(lambda_j - lambda_i) (0 for equal eigenvalues).
void eig_adjoint(tt_ctx* c, const EigSlot& e, const double* Vb, const double* lb, int Rdim,
                 int k, double* out) {
  GradBufs& g = c->gb;
  hipStream_t s = c->st;
  const int N = c->N;
  int* d = c->dims;
  gemm(gd(e.V, N, 1, Vb, N, 0, g.Ce, N, dimv(Rdim), dimv(k), dimv(Rdim)), N, N, 1, d, s);
  launch_eig_adj_inner(g.Ce, N, e.lam, lb, d, Rdim, k, N, s);
  gemm(gd(e.V, N, 0, g.Ce, N, 0, g.Te, N, dimv(Rdim), dimv(k), dimv(Rdim)), N, N, 1, d, s);
  gemm(gd(g.Te, N, 0, e.V, N, 1, out, N, dimv(Rdim), dimv(Rdim), dimv(k)), N, N, 1, d, s);
  launch_symmetrize(out, N, d, Rdim, N, s);
}

// Adjoint of one Gram-SVD truncation (App. A.2):
//   M = S_A V_A^T V_B S_B = U S V^T,  P = V_A D_A U_r,  M_upd = S_r V_r^T D_B V_B^T,
// D = S^-1, S = sqrt(lambda).  Inputs: P bar (g.Pb, R x r, ld rcap) and
// M_upd bar (g.Mub, r x R, ld Rcap); outputs the Gram cotangents G_A bar and
// G_B bar (R x R, ld N, symmetric).
void trunc_adjoint(tt_ctx* c, int bond, const EigSlot& ea, const EigSlot& eb, const EigSlot& em,
                   const double* M, int Rcap, int rcap, int Rdim, double* GbA, double* GbB) {
  GradBufs& g = c->gb;
  hipStream_t s = c->st;
  const int N = c->N;
  int* d = c->dims;
  const int ka = bond == 1 ? D_KA1 : D_KA2, kb = bond == 1 ? D_KB1 : D_KB2;
  const int kc = bond == 1 ? D_KC1 : D_KC2, rn = bond == 1 ? D_R1N : D_R2N;
  const int side = bond == 1 ? D_SIDE1 : D_SIDE2;
  // singular vectors of M on both sides for the kc computed pairs, with the
  // forward's signs (side 1: U = M V S^-1, sign-fixed on U)
  launch_copy_cond(em.V, N, g.U, N, d, ka, kc, side, 0, N, s);
  launch_copy_cond(em.V, N, g.V, N, d, kb, kc, side, 1, N, s);
  {
    GemmDesc v = gd(M, Rcap, 1, g.U, N, 0, g.V, N, dimv(kb), dimv(kc), dimv(ka));
    v.colscale = em.isq;
    v.cond_idx = side; v.cond_val = 0;
    gemm(v, N, N, 1, d, s);
    GemmDesc u = gd(M, Rcap, 0, g.V, N, 0, g.U, N, dimv(ka), dimv(kc), dimv(kb));
    u.colscale = em.isq;
    u.cond_idx = side; u.cond_val = 1;
    gemm(u, N, N, 1, d, s);
    launch_gauge_pair(g.U, N, g.V, N, d, ka, kb, kc, side, N, s);
  }
  // P = V_A D_A U_r:  V_A bar = P bar (D_A U_r)^T,  U bar = D_A V_A^T P bar
  {
    GemmDesc a = gd(g.Pb, rcap, 0, g.U, N, 1, g.VAb, N, dimv(Rdim), dimv(ka), dimv(rn));
    a.colscale = ea.isq;
    gemm(a, Rcap, N, 1, d, s);
    launch_coldot(ea.V, N, g.VAb, N, nullptr, g.cA, d, dimv(Rdim), dimv(ka), N, s);
    launch_zero_block(g.Ub, N, d, dimv(ka), dimv(kc), (long long)N * N, s);
    GemmDesc u = gd(ea.V, N, 1, g.Pb, rcap, 0, g.Ub, N, dimv(ka), dimv(rn), dimv(Rdim));
    u.rowscale = ea.isq;
    gemm(u, N, rcap, 1, d, s);
  }
  // M_upd = S_r V_r^T D_B V_B^T:  W = M_upd bar V_B, then s bar, D_B term, V bar;
  // V_B bar = M_upd bar^T S_r V_r^T D_B
  {
    gemm(gd(g.Mub, Rcap, 0, eb.V, N, 0, g.W, N, dimv(rn), dimv(kb), dimv(Rdim)), rcap, N, 1, d, s);
    launch_trunc_w(g.W, N, eb.isq, g.V, N, em.sq, g.sb, g.cB, g.Vb, N, d, rn, kb, kc, s);
    GemmDesc b = gd(g.Mub, Rcap, 1, g.V, N, 1, g.VBb, N, dimv(Rdim), dimv(kb), dimv(rn));
    b.kscale = em.sq;
    b.colscale = eb.isq;
    gemm(b, Rcap, N, 1, d, s);
  }
  // truncated SVD:  M bar = U In V^T + U bar S_r^-1 V^T + U S_r^-1 V bar^T
  {
    gemm(gd(g.U, N, 1, g.Ub, N, 0, g.G1, N, dimv(kc), dimv(kc), dimv(ka)), N, N, 1, d, s);
    gemm(gd(g.V, N, 1, g.Vb, N, 0, g.G2, N, dimv(kc), dimv(kc), dimv(kb)), N, N, 1, d, s);
    launch_svd_adj_inner(g.G1, g.G2, N, em.sq, g.sb, g.In, N, d, kc, rn, N, s);
    gemm(gd(g.U, N, 0, g.In, N, 0, g.Tm, N, dimv(ka), dimv(kc), dimv(kc)), N, N, 1, d, s);
    gemm(gd(g.Tm, N, 0, g.V, N, 1, g.Mb, N, dimv(ka), dimv(kb), dimv(kc)), N, N, 1, d, s);
    GemmDesc p = gd(g.Ub, N, 0, g.V, N, 1, g.Mb, N, dimv(ka), dimv(kb), dimv(rn));
    p.kscale = em.isq;
    p.beta = 1.0;
    gemm(p, N, N, 1, d, s);
    GemmDesc q = gd(g.U, N, 0, g.Vb, N, 1, g.Mb, N, dimv(ka), dimv(kb), dimv(rn));
    q.kscale = em.isq;
    q.beta = 1.0;
    gemm(q, N, N, 1, d, s);
  }
  // M = S_A C S_B with C = V_A^T V_B
  {
    gemm(gd(ea.V, N, 1, eb.V, N, 0, g.Cm, N, dimv(ka), dimv(kb), dimv(Rdim)), N, N, 1, d, s);
    launch_mb_vecs(g.Mb, N, g.Cm, N, ea.sq, eb.sq, g.SAb, g.SBb, d, ka, kb, s);
    GemmDesc a = gd(eb.V, N, 0, g.Mb, N, 1, g.VAb, N, dimv(Rdim), dimv(ka), dimv(kb));
    a.kscale = eb.sq;
    a.colscale = ea.sq;
    a.beta = 1.0;
    gemm(a, Rcap, N, 1, d, s);
    GemmDesc b = gd(ea.V, N, 0, g.Mb, N, 0, g.VBb, N, dimv(Rdim), dimv(kb), dimv(ka));
    b.kscale = ea.sq;
    b.colscale = eb.sq;
    b.beta = 1.0;
    gemm(b, Rcap, N, 1, d, s);
  }
  launch_lambar(g.SAb, g.cA, ea.sq, g.lbA, d, ka, N, s);
  launch_lambar(g.SBb, g.cB, eb.sq, g.lbB, d, kb, N, s);
  eig_adjoint(c, ea, g.VAb, g.lbA, Rdim, ka, GbA);
  eig_adjoint(c, eb, g.VBb, g.lbB, Rdim, kb, GbB);
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
  // ---- bond 2: Theta' = A2 P2 (A2 = Theta_p as r1' N_theta x R2), Phi' = M_upd2 Phi_cat
  gemm(gd(g.Thb, r2c, 0, c->P2, r2c, 1, g.A2b, R2c, dimv(D_R1NT), dimv(D_RC2), dimv(D_R2N)),
       r1c * nt, R2c, 1, d, s);
  gemm(gd(c->Thp, R2c, 1, g.Thb, r2c, 0, g.Pb, r2c, dimv(D_RC2), dimv(D_R2N), dimv(D_R1NT)), R2c,
       r2c, 1, d, s);
  gemm(gd(g.Phb, np, 0, c->Phcat, np, 1, g.Mub, R2c, dimv(D_R2N), dimv(D_RC2), dimc(np)), r2c, R2c,
       1, d, s);
  gemm(gd(c->Mupd2, R2c, 1, g.Phb, np, 0, g.Phcb, np, dimv(D_RC2), dimc(np), dimv(D_R2N)), R2c, np,
       1, d, s);
  trunc_adjoint(c, 2, c->E[4], c->E[2], c->E[5], c->M2, R2c, r2c, D_RC2, g.GbA, g.GbR3);
  {  // G_L2 = A2^T A2
    GemmDesc a = gd(c->Thp, R2c, 0, g.GbA, N, 0, g.A2b, R2c, dimv(D_R1NT), dimv(D_RC2), dimv(D_RC2));
    a.alpha = 2.0;
    a.beta = 1.0;
    gemm(a, r1c * nt, R2c, 1, d, s);
  }
  // ---- bond 1: X' = X_cat P1, Theta_p = M_upd1 Theta_cat
  gemm(gd(g.Xb, ldX, 0, c->P1, r1c, 1, g.Xcb, ldC, dimc(ns), dimv(D_RC1), dimv(D_R1N)), ns, R1c, 1,
       d, s);
  {  // P1 bar = X_cat^T X' bar, split over N_s
    GemmDesc p = gd(c->Xcat, ldC, 1, g.Xb, ldX, 0, g.part, r1c, dimv(D_RC1), dimv(D_R1N), dimc(ns));
    p.ksplit = g.ksl;
    p.sC = (long long)R1c * r1c;
    gemm(p, R1c, r1c, g.nsplit, d, s);
    sum_partials(g.part, (long long)R1c * r1c, g.nsplit, g.Pb, r1c, r1c, dimv(D_RC1), dimv(D_R1N),
                 R1c, r1c, d, s);
  }
  {  // M_upd1 bar = sum_l Theta_p bar_l Theta_cat_l^T (one partial per ordinate)
    GemmDesc m = gd(g.A2b, ldT, 0, c->Thcat, ldT, 1, g.part, R1c, dimv(D_R1N), dimv(D_RC1), dimv(D_RC2));
    m.sA = m.sB = R2c;
    m.sC = (long long)r1c * R1c;
    gemm(m, r1c, R1c, nt, d, s);
    sum_partials(g.part, (long long)r1c * R1c, nt, g.Mub, R1c, R1c, dimv(D_R1N), dimv(D_RC1), r1c,
                 R1c, d, s);
  }
  {  // Theta_cat bar_l = M_upd1^T Theta_p bar_l
    GemmDesc t = gd(c->Mupd1, R1c, 1, g.A2b, ldT, 0, g.Thcb, ldT, dimv(D_RC1), dimv(D_RC2), dimv(D_R1N));
    t.sB = t.sC = R2c;
    gemm(t, R1c, R2c, nt, d, s);
  }
  trunc_adjoint(c, 1, c->E[0], c->E[1], c->E[3], c->M1, R1c, r1c, D_RC1, g.GbA, g.GbB);
  {  // G_A = X_cat^T X_cat
    GemmDesc a = gd(c->Xcat, ldC, 0, g.GbA, N, 0, g.Xcb, ldC, dimc(ns), dimv(D_RC1), dimv(D_RC1));
    a.alpha = 2.0;
    a.beta = 1.0;
    gemm(a, ns, R1c, 1, d, s);
  }
  {  // G_B1 = sum_l Theta_cat_l G_R3 Theta_cat_l^T (T1 = Theta_cat G_R3)
    GemmDesc t = gd(g.GbB, N, 0, c->T1, ldT, 0, g.Thcb, ldT, dimv(D_RC1), dimv(D_RC2), dimv(D_RC1));
    t.sB = t.sC = R2c;
    t.alpha = 2.0;
    t.beta = 1.0;
    gemm(t, R1c, R2c, nt, d, s);
    GemmDesc y = gd(g.GbB, N, 0, c->Thcat, ldT, 0, g.Y, ldT, dimv(D_RC1), dimv(D_RC2), dimv(D_RC1));
    y.sB = y.sC = R2c;
    gemm(y, R1c, R2c, nt, d, s);
    const int nz = nsplit_gr3(c);
    GemmDesc r = gd(c->Thcat, R2c, 1, g.Y, R2c, 0, g.part, R2c, dimv(D_RC2), dimv(D_RC2),
                    dimv(D_RC1, nt));
    r.ksplit = KSPLIT_GR3;
    r.sC = (long long)R2c * R2c;
    gemm(r, R2c, R2c, nz, d, s);
    sum_partials(g.part, (long long)R2c * R2c, nz, g.GbR3, N, R2c, dimv(D_RC2), dimv(D_RC2), R2c,
                 R2c, d, s, 1.0);
  }
  {  // G_R3 = Phi_cat Phi_cat^T
    GemmDesc p = gd(g.GbR3, N, 0, c->Phcat, np, 0, g.Phcb, np, dimv(D_RC2), dimc(np), dimv(D_RC2));
    p.alpha = 2.0;
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
  g.ths = (size_t)c->r1c * nt * c->r2c;
  g.phs = (size_t)c->r2c * np;
  g.ckX = cv.take<double>(g.nck * g.xs);
  g.ckTh = cv.take<double>(g.nck * g.ths);
  g.ckPh = cv.take<double>(g.nck * g.phs);
  g.ckR = cv.take<int>(2 * (size_t)g.nck);
  g.sgX = cv.take<double>(kseg * g.xs);
  g.sgTh = cv.take<double>(kseg * g.ths);
  g.sgPh = cv.take<double>(kseg * g.phs);
  g.sgR = cv.take<int>(2 * (size_t)kseg);
  g.fX = cv.take<double>(g.xs);
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
  const size_t pr = std::max((size_t)c->R1c * c->r1c, (size_t)c->R2c * c->r2c);
  g.Pb = cv.take<double>(pr);
  g.Mub = cv.take<double>(pr);
  double** mats[] = {&g.U, &g.V, &g.Ub, &g.Vb, &g.G1, &g.G2, &g.In, &g.Tm, &g.Mb, &g.Cm,
                     &g.VAb, &g.VBb, &g.W, &g.Ce, &g.Te, &g.GbA, &g.GbB, &g.GbR3};
  for (double** p : mats) *p = cv.take<double>((size_t)N * N);
  g.Y = cv.take<double>((size_t)c->R1c * nt * c->R2c);
  double** vecs[] = {&g.sb, &g.SAb, &g.SBb, &g.cA, &g.cB, &g.lbA, &g.lbB};
  for (double** p : vecs) *p = cv.take<double>(N);
  // N_s-long contractions: at most 64 slices of a multiple of 16 rows
  g.ksl = ((ns + 63) / 64 + 15) / 16 * 16;
  g.nsplit = (ns + g.ksl - 1) / g.ksl;
  g.part_n = std::max({(size_t)g.nsplit * c->R1c * c->r1c, (size_t)nt * c->r1c * c->R1c,
                       (size_t)nsplit_gr3(c) * c->R2c * c->R2c});
  g.part = cv.take<double>(g.part_n);
}

hipError_t grad_record(tt_ctx* c) {
  GradBufs& g = c->gb;
  if (c->nhist % g.K) return hipSuccess;
  const int slot = c->nhist / g.K;
  if (slot >= g.nck) return hipSuccess;
  return copy_state(c, g.ckX + slot * g.xs, g.ckTh + slot * g.ths, g.ckPh + slot * g.phs,
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
  if (g.stale) return ctx_fail(c, TT_ERR_STATE, "kappa changed after the steps were taped");
  hipStream_t s = c->st;
  const int nsteps = c->nhist, ns = c->ns;
  const tt_config& cf = c->cfg;
  const double dV = (cf.lx / cf.nx) * (cf.ly / cf.ny) * (cf.dim == 3 ? cf.lz / cf.nz : 1.0);
  int* d = c->dims;
  // final state: kept aside, restored at the end
  GCHK(c, copy_state(c, g.fX, g.fTh, g.fPh, g.fR, true));
  GCHK(c, hipMemcpyAsync(g.wdet, detector_w, (size_t)ns * 8, hipMemcpyHostToDevice, s));
  // loss and its seed
  launch_energy(c->X, c->ldX, ns, c->Th, c->nt, c->r2c, c->Ph, c->np, c->w, c->v, c->pv, c->z,
                dimv(D_R1), dimv(D_R2), 1.0 / cf.c, c->Enew, d, c->r1c, c->r2c, s);
  launch_wdot(g.wdet, c->Enew, ns, g.loss, s);
  launch_seed(g.wdet, c->z, c->X, c->ldX, ns, c->w, c->v, c->pv, c->Th, c->nt, c->r2c, c->np,
              c->r1c, loss_bar * dV, loss_bar * dV / cf.c, g.xg, g.Xb, g.Thb, g.Phb, d, s);
  GCHK(c, hipMemsetAsync(g.kbar, 0, (size_t)ns * 8, s));
  launch_source_derivs(ns, cf.c, c->dt, cf.a_r, c->rho, c->T, c->d, g.dd, g.ds, s);
  c->eig_all = 1;
  const int nseg = (nsteps + g.K - 1) / g.K;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int m0 = seg * g.K, m1 = std::min(m0 + g.K, nsteps);
    GCHK(c, copy_state(c, g.ckX + seg * g.xs, g.ckTh + seg * g.ths, g.ckPh + seg * g.phs,
                       g.ckR + 2 * seg, false));
    // the segment's states m0 .. m1-1
    for (int m = m0; m < m1; ++m) {
      const int k = m - m0;
      GCHK(c, copy_state(c, g.sgX + k * g.xs, g.sgTh + k * g.ths, g.sgPh + k * g.phs, g.sgR + 2 * k, true));
      if (m == m1 - 1) break;
      launch_replay_from_hist(d, c->hist, m, s);
      step_body_fp64_frozen(c);
      launch_finish(d, nullptr, -1, s);
      std::swap(c->X, c->Xn);
    }
    for (int m = m1 - 1; m >= m0; --m) {
      const int k = m - m0;
      GCHK(c, copy_state(c, g.sgX + k * g.xs, g.sgTh + k * g.ths, g.sgPh + k * g.phs, g.sgR + 2 * k, false));
      launch_replay_from_hist(d, c->hist, m, s);
      step_body_fp64_frozen(c);
      reverse_step(c);
      std::swap(g.Xb, g.Xnb);
      std::swap(g.Thb, g.Thnb);
      std::swap(g.Phb, g.Phnb);
    }
  }
  c->eig_all = 0;
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
