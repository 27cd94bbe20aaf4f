// The library context (one TT state on one stream) and what the forward step
// and the adjoint sweep share: the workspace carver, eigen slots, the GEMM
// descriptor helper and the step body.
#pragma once

#include <string.h>

#include <string>
#include <vector>

#include "../../include/tt.h"
#include "tt_step.h"

namespace tt {

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct EigSlot {
  double *lam, *V, *sq, *isq, *work;
};

// Device buffers of the reverse sweep (present when ckpt_every > 0).
struct GradBufs {
  bool on = false;
  int K = 0;                   // steps per checkpoint
  int nck = 0;                 // checkpoint slots
  size_t xs = 0, ths = 0, phs = 0;  // doubles per stored X (cotangent), Theta, Phi
  size_t xbytes = 0;           // bytes of a stored X (FP64, or FP32 in the mixed form)
  char *ckX, *sgX, *fX;         // stored X (xbytes each; FP32 in the mixed form)
  double *ckTh, *ckPh;         // checkpoints (state before steps 0, K, 2K, ...)
  int* ckR;                    // their ranks (r1, r2)
  double *sgTh, *sgPh;         // the K states of the segment being reversed
  int* sgR;
  double *fTh, *fPh;           // the final state, restored after the sweep
  int* fR;
  // cotangents: of the step output (…b) and of its input (…nb)
  double *Xb, *Xnb, *Thb, *Thnb, *Phb, *Phnb;
  double *Xcb, *Thcb, *Phcb, *A2b;
  double *kbar, *dd, *ds, *wdet, *xg, *loss;
  // truncation adjoint scratch (N x N, ld N, unless noted)
  double* Mub;                 // M_upd bar (r x R, ld R cap)
  double *Xbt, *Tbt;           // A' bar_tot of bond 1 (N_s x ldX) and bond 2 (as Theta)
  double *Uh, *Uh2;            // left singular vectors of the bond matrix (N_s x ldC; r1 N_theta x R2 cap)
  double *Z2, *A2e;            // bond 2: Z and the effective A (r1 N_theta x R2 cap)
  double *U1, *V1, *Y1, *U2, *V2, *Y2;  // per-bond factors of the truncation
  double *G1, *In, *Pf, *YG, *Qm, *AZ, *Ta, *Hm, *GBs, *S3, *Mt, *Mt1;
  double *Y;                   // R1 x N_theta R2 cap
  double* part;                // split-K partial products
  size_t part_n = 0;
  int ksl = 0;                 // row slice of the N_s-long contractions
  bool stale = false;          // kappa changed after the steps were taped
};

inline GemmDesc gd(const double* A, int lda, int ta, const double* B, int ldb, int tb, double* C,
                   int ldc, DimExpr m, DimExpr n, DimExpr k) {
  GemmDesc g;
  memset(&g, 0, sizeof(g));
  g.A = A; g.B = B; g.C = C;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.transA = ta; g.transB = tb;
  g.m = m; g.n = n; g.k = k;
  g.alpha = 1.0; g.beta = 0.0;
  g.cond_idx = -1;
  g.bclip_idx = -1;
  return g;
}

}  // namespace tt

struct tt_ctx {
  tt_config cfg;
  hipStream_t st;
  tt::StepGeom G;
  int ns, nt, np, dim, B, nbc, nem;
  int r1c, r2c, R1c, R2c, ldX, ldC, N;
  int q1c, q2c;  // capacities of the number of singular values of M per bond
  double dt, lam[3];
  std::vector<double> h_rho, h_cv;
  // device
  int *dims, *hist, *sched;
  double* diag;
  double *w, *v, *tfac, *pfac, *bc_e, *bc_t, *bc_p;
  double* hllw;              // HLL face weights (dim x N_s x 4), HLL flux only
  double* bc_e0;             // HLL: unweighted inflow columns (nbc x N_s)
  int* bc_code;              // HLL: weight selector of each inflow column (4 axis + slot)
  double *kappa, *rho, *cv, *T, *d, *s, *Estar, *Enew, *Tdag;
  double* kappa_s;           // scattering opacity (zero unless tt_set_scattering)
  double *wbuf, *lossbuf;    // detector weights and the loss of tt_detector_loss
  bool scatter = false;      // some kappa_s > 0: the source depends on E* every step
  int nem_base = 0;          // source block present without scattering
  double *X, *Xn, *Th, *Ph;
  bool mixed = false;        // TT_FP32_MIXED: X and X_cat stored in FP32
  float *Xf, *Xnf, *Xcatf;   // FP32 state / update / concatenation (mixed form only)
  unsigned* colmax;          // per-column max |X_cat| bits for the sliced Gram
  double *Thcat, *Phcat, *Xcat, *gpart;
  double *GA, *GB1, *GR3, *GL2, *T1;
  tt::EigSlot E[6];  // bond 1: 0 G_A, 1 G_B1, 2 G_R3, 3 SVD of M1; bond 2: 4 G_L2, 5 SVD of M2
  double *M1, *C1, *Wm1, *Ur1, *P1, *Mupd1, *Thp;
  double *M2, *C2, *Wm2, *Ur2, *P2, *Mupd2;
  double *pv, *z;
  double* zt;  // z by stencil block, r1c x MAX_BLOCKS (energy through Y = X Zt)
  tt::GradBufs gb;
  size_t ws_need;
  int nhist = 0, nsched = 0, sched_pos = 0;
  bool poisoned = false;
  std::string err;
  // step graphs: one per state buffer (the step swaps buffers), captured on
  // cap_st; gafter / gafterf / gsched are the host bookkeeping one replay
  // performs (buffers after the step, schedule entries consumed)
  bool graphs = true;
  int gram_slices = tt::GRAM_SLICES_DEFAULT;
  int jac_maxsw = 0;  // tt_set_solver_limits (0: the solver's own limit)  // 11-bit slices of the FP32-mixed Gram
  hipStream_t cap_st = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  const void* gkey[2] = {nullptr, nullptr};
  double* gafter[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  float* gafterf[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int gsched[2] = {0, 0};
  // profiling
  bool prof = false;
  unsigned prof_mask = 0;    // classes recorded (bit k: class k)
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  size_t ev_used = 0;
};

namespace tt {

tt_status ctx_fail(tt_ctx* c, tt_status code, const std::string& msg);
// Concatenation and rounding of one step with frozen material (FP64 or the
// FP32-mixed form), leaving dims[R1], dims[R2] at the input ranks (no close
// of the step): X_cat, Theta_cat, Phi_cat and every rounding intermediate
// stay in the context; X' is in Xn (FP64) or Xnf (mixed).
void step_body_frozen(tt_ctx* c);
// Adjoint buffers (appended to the workspace when ckpt_every > 0).
void grad_carve(tt_ctx* c, Carve& cv);
// Before step number c->nhist: store a checkpoint if one is due.
hipError_t grad_record(tt_ctx* c);

}  // namespace tt
