// C ABI of the tensor-train S_N library (see include/tt.h) and the host-side
// orchestration of one step on a single HIP stream.  All buffers are carved
// from the caller's device workspace; ranks live in the device dims table.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "tt_ctx.h"

using namespace tt;

namespace {

thread_local std::string g_err;

constexpr double PI = 3.14159265358979323846;

enum ProfClass { P_CONCAT, P_GRAM, P_GRAMRED, P_EIG1, P_EIGM1, P_EIG2, P_EIGM2, P_XUPD, P_SMALL,
                 P_MAT, P_STEP, P_NCLS };
const char* kProfNames[P_NCLS] = {"concat", "gram_tall", "gram_reduce", "eig_bond1", "eig_M1",
                                  "eig_bond2", "eig_M2", "x_update", "small_gemm",
                                  "material_energy", "step"};

}  // namespace

namespace {

tt_status fail(tt_ctx* c, tt_status code, const std::string& msg) {
  if (c) c->err = msg;
  else g_err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                        \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(ctx, TT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---- validation and sizes --------------------------------------------------
bool validate(const tt_config* c, int n_inflow, std::string& why) {
  if (!c) { why = "null config"; return false; }
  if (c->dim != 2 && c->dim != 3) { why = "dim must be 2 or 3"; return false; }
  if (c->nx < 1 || c->ny < 1 || (c->dim == 3 && c->nz < 1)) { why = "bad grid"; return false; }
  if (c->ntheta < 2 || c->ntheta % 2) { why = "ntheta must be even"; return false; }
  if (c->nphi < 4 || c->nphi % 4) { why = "nphi must be a multiple of 4"; return false; }
  if (!(c->c > 0) || !(c->a_r > 0)) { why = "c and a_r must be positive"; return false; }
  if (!(c->lx > 0) || !(c->ly > 0) || (c->dim == 3 && !(c->lz > 0))) { why = "bad extents"; return false; }
  if (!(c->dt > 0) && !(c->cfl > 0)) { why = "need dt > 0 or cfl > 0"; return false; }
  if (!(c->tol >= 0)) { why = "tol must be >= 0"; return false; }
  if (c->precision != TT_FP64 && c->precision != TT_FP32_MIXED) { why = "bad precision"; return false; }
  if (c->schedule != TT_ROUND_ONCE && c->schedule != TT_ROUND_TWICE) { why = "bad schedule"; return false; }
  if (c->flux != TT_FLUX_UPWIND && c->flux != TT_FLUX_RUSANOV && c->flux != TT_FLUX_HLL) {
    why = "bad flux";
    return false;
  }
  if (c->flux == TT_FLUX_HLL && !(c->hll_beta > 0 && c->hll_beta < 1e300 && c->hll_tau_threshold > 0 &&
                                  c->hll_tau_threshold < 1e300)) {
    why = "hll_beta and hll_tau_threshold must be finite and > 0";
    return false;
  }
  if (c->flux == TT_FLUX_RUSANOV && !(c->s_plus >= 0 && c->s_plus < 1e300)) {
    why = "s_plus must be finite and >= 0";
    return false;
  }
  if (c->material != TT_MAT_FROZEN && c->material != TT_MAT_COUPLED) { why = "bad material"; return false; }
  if (c->rank_mode != TT_RANK_AUTO && c->rank_mode != TT_RANK_REPLAY) { why = "bad rank_mode"; return false; }
  for (int a = 0; a < c->dim; ++a) {
    const int lo = c->bc_lo[a], hi = c->bc_hi[a];
    if (lo < 0 || lo > 3 || hi < 0 || hi > 3) { why = "bad bc code"; return false; }
    if ((lo == TT_BC_PERIODIC) != (hi == TT_BC_PERIODIC)) { why = "periodic bc must be paired"; return false; }
  }
  if (n_inflow < 0 || n_inflow > 64) { why = "n_inflow out of range"; return false; }
  if (c->max_steps < 0) { why = "max_steps < 0"; return false; }
  if (c->ckpt_every > 0 && c->material != TT_MAT_FROZEN) {
    why = "ckpt_every > 0 (the adjoint) needs TT_MAT_FROZEN";
    return false;
  }
  if (c->ckpt_every > 0 && (c->flux != TT_FLUX_UPWIND || c->schedule != TT_ROUND_ONCE)) {
    why = "ckpt_every > 0 (the adjoint) needs TT_FLUX_UPWIND and TT_ROUND_ONCE";
    return false;
  }
  for (int a = 0; a < c->dim && c->ckpt_every > 0; ++a)
    if (c->bc_lo[a] == TT_BC_OUTFLOW || c->bc_hi[a] == TT_BC_OUTFLOW) {
      why = "ckpt_every > 0 (the adjoint) does not cover TT_BC_OUTFLOW";
      return false;
    }
  return true;
}

// Rusanov with S+ > 0 has a diffusion block per axis and two rank-1 terms
// per Dirichlet face entry; HLL two rank-1 terms per entry (one per sign of n).
bool rusanov_diffusion(const tt_config& c) { return c.flux == TT_FLUX_RUSANOV && c.s_plus != 0.0; }
int inflow_blocks(const tt_config& c, int n_inflow) {
  return n_inflow * (rusanov_diffusion(c) || c.flux == TT_FLUX_HLL ? 2 : 1);
}
bool all_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!(fabs(a[i]) <= 1.79e308)) return false;
  return true;
}

void geometry(tt_ctx* x, const tt_config& c, int n_inflow, int nem) {
  x->cfg = c;
  x->dim = c.dim;
  const int nz = c.dim == 3 ? c.nz : 1;
  x->ns = c.nx * c.ny * nz;
  x->nt = c.ntheta;
  x->np = c.nphi;
  const bool rus = c.flux == TT_FLUX_RUSANOV, dif = rusanov_diffusion(c);
  x->B = rus ? 1 + (dif ? 2 : 1) * c.dim : 1 + 2 * c.dim;
  x->nbc = inflow_blocks(c, n_inflow);
  x->nem = nem;
  const long long big = 1LL << 30;
  long long cap1 = std::min<long long>(x->ns, (long long)x->nt * x->np);
  long long cap2 = std::min<long long>(x->np, (long long)x->ns * x->nt);
  if (c.rmax > 0) { cap1 = std::min<long long>(cap1, c.rmax); cap2 = std::min<long long>(cap2, c.rmax); }
  if (c.r1_cap > 0) cap1 = c.r1_cap;
  if (c.r2_cap > 0) cap2 = c.r2_cap;
  x->r1c = (int)std::min(cap1, big);
  x->r2c = (int)std::min(cap2, big);
  x->R1c = x->B * x->r1c + x->nbc + x->nem;
  x->R2c = x->B * x->r2c + x->nbc + x->nem;
  x->ldX = round_up(x->r1c, 8);
  x->ldC = round_up(x->R1c, 8);
  x->N = std::max(x->R1c, x->R2c);
  // M at bond 1 is at most min(R1, N_s, N_theta N_phi) in rank, at bond 2
  // min(R2, r1 N_theta, N_phi)
  x->q1c = (int)std::min<long long>(std::min<long long>(x->R1c, x->ns), (long long)x->nt * x->np);
  x->q2c = (int)std::min<long long>(std::min<long long>(x->R2c, (long long)x->r1c * x->nt), x->np);
  const double dx = c.lx / c.nx, dy = c.ly / c.ny, dz = c.dim == 3 ? c.lz / nz : 1e300;
  const double hmin = std::min(dx, std::min(dy, dz));
  x->dt = c.dt > 0 ? c.dt : c.cfl * hmin / c.c;
  x->lam[0] = c.c * x->dt / dx;
  x->lam[1] = c.c * x->dt / dy;
  x->lam[2] = c.dim == 3 ? c.c * x->dt / dz : 0.0;
  StepGeom& G = x->G;
  G.ns = x->ns; G.nx = c.nx; G.ny = c.ny; G.nz = nz;
  G.n[0] = c.nx; G.n[1] = c.ny; G.n[2] = nz;
  G.stride[0] = 1; G.stride[1] = c.nx; G.stride[2] = c.nx * c.ny;
  for (int a = 0; a < 3; ++a) {
    G.periodic[a] = a < c.dim && c.bc_lo[a] == TT_BC_PERIODIC;
    G.bclo[a] = a < c.dim ? c.bc_lo[a] : TT_BC_VACUUM;
    G.bchi[a] = a < c.dim ? c.bc_hi[a] : TT_BC_VACUUM;
  }
  // transport blocks: base, then per axis (minus, plus) or (central[, diffusion])
  for (int b = 0; b < MAX_BLOCKS; ++b) { G.bkind[b] = BK_BASE; G.baxis[b] = 0; }
  for (int a = 0, b = 1; a < c.dim; ++a) {
    if (rus) {
      G.bkind[b] = BK_CENTRAL; G.baxis[b++] = a;
      if (dif) { G.bkind[b] = BK_DIFF; G.baxis[b++] = a; }
    } else if (c.flux == TT_FLUX_HLL) {
      G.bkind[b] = BK_HLL_POS; G.baxis[b++] = a;
      G.bkind[b] = BK_HLL_NEG; G.baxis[b++] = a;
    } else {
      G.bkind[b] = BK_MINUS; G.baxis[b++] = a;
      G.bkind[b] = BK_PLUS; G.baxis[b++] = a;
    }
  }
  G.hllw = nullptr;
  G.nt = x->nt; G.np = x->np; G.B = x->B; G.nbc = x->nbc; G.nem = x->nem;
  G.r1c = x->r1c; G.r2c = x->r2c; G.R1c = x->R1c; G.R2c = x->R2c;
}

size_t carve(tt_ctx* x, char* base) {
  Carve cv{base};
  const int ns = x->ns, nt = x->nt, np = x->np, N = x->N;
  const int ms = std::max(1, x->cfg.max_steps);
  x->dims = cv.take<int>(D_NDIMS);
  x->hist = cv.take<int>(2 * (size_t)ms);
  // one replay entry per rounding: two per step with TT_ROUND_TWICE
  x->sched = cv.take<int>(2 * (size_t)ms * (x->cfg.schedule == TT_ROUND_TWICE ? 2 : 1));
  x->diag = cv.take<double>(G_NDIAG);
  x->w = cv.take<double>(nt);
  x->v = cv.take<double>(np);
  x->tfac = cv.take<double>((size_t)x->B * nt);
  x->pfac = cv.take<double>((size_t)x->B * np);
  x->bc_e = cv.take<double>((size_t)std::max(1, x->nbc) * ns);
  x->bc_t = cv.take<double>((size_t)std::max(1, x->nbc) * nt);
  x->bc_p = cv.take<double>((size_t)std::max(1, x->nbc) * np);
  const bool hll = x->cfg.flux == TT_FLUX_HLL;
  x->hllw = hll ? cv.take<double>((size_t)x->dim * ns * 4) : nullptr;
  x->bc_e0 = hll ? cv.take<double>((size_t)std::max(1, x->nbc) * ns) : nullptr;
  x->bc_code = hll ? cv.take<int>((size_t)std::max(1, x->nbc)) : nullptr;
  x->G.hllw = x->hllw;
  double** fields[] = {&x->kappa, &x->rho, &x->cv, &x->T, &x->d, &x->s, &x->Estar, &x->Enew, &x->Tdag,
                       &x->kappa_s, &x->wbuf};
  for (double** f : fields) *f = cv.take<double>(ns);
  x->lossbuf = cv.take<double>(8);
  x->X = cv.take<double>((size_t)ns * x->ldX);
  x->Xn = cv.take<double>((size_t)ns * x->ldX);
  x->Th = cv.take<double>((size_t)x->r1c * nt * x->r2c);
  x->Ph = cv.take<double>((size_t)x->r2c * np);
  x->Thcat = cv.take<double>((size_t)x->R1c * nt * x->R2c);
  x->Phcat = cv.take<double>((size_t)x->R2c * np);
  x->mixed = x->cfg.precision == TT_FP32_MIXED;
  // the mixed form keeps an FP64 X_cat only for the reverse sweep
  x->Xcat = (!x->mixed || x->cfg.ckpt_every > 0) ? cv.take<double>((size_t)ns * x->ldC) : nullptr;
  x->Xf = x->mixed ? cv.take<float>((size_t)ns * x->ldX) : nullptr;
  x->Xnf = x->mixed ? cv.take<float>((size_t)ns * x->ldX) : nullptr;
  x->Xcatf = x->mixed ? cv.take<float>((size_t)ns * x->ldC) : nullptr;
  x->colmax = x->mixed ? cv.take<unsigned>((size_t)std::max(x->R1c, x->r1c) + 64) : nullptr;
  GramPlan p1 = gram_plan(ns, x->R1c, x->ldC), p2 = gram_plan(ns, x->r1c, x->ldX);
  x->gpart = cv.take<double>(std::max(std::max(gram_partial_doubles(p1), gram_partial_doubles(p2)),
                                      std::max((size_t)nt * x->R1c * x->R1c,
                                               (size_t)nt * x->R2c * x->R2c)));
  x->GA = cv.take<double>((size_t)x->R1c * x->R1c);
  x->GB1 = cv.take<double>((size_t)x->R1c * x->R1c);
  x->GR3 = cv.take<double>((size_t)x->R2c * x->R2c);
  x->GL2 = cv.take<double>((size_t)x->R2c * x->R2c);
  x->T1 = cv.take<double>((size_t)x->R1c * nt * x->R2c);
  for (int k = 0; k < 6; ++k) {
    x->E[k].lam = cv.take<double>(N);
    x->E[k].V = cv.take<double>((size_t)N * N);
    x->E[k].sq = cv.take<double>(N);
    x->E[k].isq = cv.take<double>(N);
    // slots 3 and 5 hold the SVD of M at bonds 1 and 2 (Golub-Kahan order 2 q)
    const int ncap = k == 3 ? std::max(N, 2 * x->q1c) : k == 5 ? std::max(N, 2 * x->q2c) : N;
    x->E[k].work = cv.take<double>(eig_work_doubles(ncap));
  }
  x->M1 = cv.take<double>((size_t)x->R1c * x->R1c);
  x->C1 = cv.take<double>((size_t)x->R1c * x->R1c);
  x->Wm1 = cv.take<double>((size_t)x->R1c * x->r1c);
  x->Ur1 = cv.take<double>((size_t)x->R1c * x->r1c);
  x->P1 = cv.take<double>((size_t)x->R1c * x->r1c);
  x->Mupd1 = cv.take<double>((size_t)x->r1c * x->R1c);
  x->Thp = cv.take<double>((size_t)x->r1c * nt * x->R2c);
  x->M2 = cv.take<double>((size_t)x->R2c * x->R2c);
  x->C2 = cv.take<double>((size_t)x->R2c * x->R2c);
  x->Wm2 = cv.take<double>((size_t)x->R2c * x->r2c);
  x->Ur2 = cv.take<double>((size_t)x->R2c * x->r2c);
  x->P2 = cv.take<double>((size_t)x->R2c * x->r2c);
  x->Mupd2 = cv.take<double>((size_t)x->r2c * x->R2c);
  x->pv = cv.take<double>(std::max(x->R2c, x->r2c) + 8);
  x->z = cv.take<double>(std::max(x->R1c, x->r1c) + 8);
  x->zt = cv.take<double>((size_t)x->r1c * MAX_BLOCKS);
  if (x->cfg.ckpt_every > 0) grad_carve(x, cv);
  return cv.off + 256;
}

int emission_flag(const tt_config& c, const double* T0, int ns) {
  if (c.material == TT_MAT_COUPLED) return 1;
  if (!T0) return 1;
  for (int i = 0; i < ns; ++i)
    if (T0[i] != 0.0) return 1;
  return 0;
}

// Quadrature (midpoint cells in mu and phi) and the rank-1 angular factors of
// each transport block: (theta factor, phi factor) such that the block is
// (D X) (tfac Theta) (pfac Phi).
void host_factors(const tt_ctx* x, std::vector<double>& w, std::vector<double>& v,
                  std::vector<double>& tf, std::vector<double>& pf, std::vector<double>& mu,
                  std::vector<double>& sint, std::vector<double>& cosp, std::vector<double>& sinp) {
  const int nt = x->nt, np = x->np;
  w.assign(nt, 2.0 / nt);
  v.assign(np, 2.0 * PI / np);
  mu.resize(nt); sint.resize(nt); cosp.resize(np); sinp.resize(np);
  for (int l = 0; l < nt; ++l) {
    mu[l] = -1.0 + (l + 0.5) * (2.0 / nt);
    sint[l] = sqrt(1.0 - mu[l] * mu[l]);
  }
  for (int p = 0; p < np; ++p) {
    const double ph = (p + 0.5) * (2.0 * PI / np);
    cosp[p] = cos(ph);
    sinp[p] = sin(ph);
  }
  tf.assign((size_t)x->B * nt, 0.0);
  pf.assign((size_t)x->B * np, 0.0);
  const StepGeom& G = x->G;
  for (int b = 0; b < x->B; ++b) {
    const int a = G.baxis[b], kind = G.bkind[b];
    const double lam = x->lam[a];
    for (int l = 0; l < nt; ++l) {
      double t = 1.0;  // base and Rusanov diffusion blocks: isotropic in theta
      if (kind == BK_MINUS || kind == BK_HLL_POS) t = a < 2 ? sint[l] : std::max(mu[l], 0.0);
      else if (kind == BK_PLUS || kind == BK_HLL_NEG) t = a < 2 ? sint[l] : std::min(mu[l], 0.0);
      else if (kind == BK_CENTRAL) t = a < 2 ? sint[l] : mu[l];
      tf[(size_t)b * nt + l] = t;
    }
    for (int p = 0; p < np; ++p) {
      const double n = a == 0 ? cosp[p] : a == 1 ? sinp[p] : 1.0;
      double f = 1.0;
      if (kind == BK_MINUS || kind == BK_HLL_POS) f = a < 2 ? -lam * std::max(n, 0.0) : -lam;
      else if (kind == BK_PLUS || kind == BK_HLL_NEG) f = a < 2 ? -lam * std::min(n, 0.0) : -lam;
      else if (kind == BK_CENTRAL) f = -lam * n;
      else if (kind == BK_DIFF) f = 0.5 * lam * x->cfg.s_plus;
      pf[(size_t)b * np + p] = f;
    }
  }
}

// HLL flux: the face weights from the current rho, kappa and kappa_s, then
// the inflow columns weighted by them (queued on the context's stream).
void hll_refresh(tt_ctx* x) {
  if (x->cfg.flux != TT_FLUX_HLL) return;
  const tt_config& c = x->cfg;
  const double h[3] = {c.lx / c.nx, c.ly / c.ny, c.dim == 3 ? c.lz / x->G.nz : 1.0};
  launch_hll_weights(x->G, x->dim, x->rho, x->kappa, x->kappa_s, c.hll_beta, h, c.hll_tau_threshold,
                     x->hllw, x->st);
  launch_hll_inflow(x->G, x->bc_e0, x->bc_code, x->nbc, x->hllw, x->bc_e, x->st);
}

std::vector<int> face_cells(const tt_ctx* x, int face) {
  const int nx = x->G.nx, ny = x->G.ny, nz = x->G.nz;
  const int axis = face / 2, hi = face % 2;
  std::vector<int> out;
  if (axis == 0) {
    const int ix = hi ? nx - 1 : 0;
    for (int iz = 0; iz < nz; ++iz)
      for (int iy = 0; iy < ny; ++iy) out.push_back(ix + nx * (iy + ny * iz));
  } else if (axis == 1) {
    const int iy = hi ? ny - 1 : 0;
    for (int iz = 0; iz < nz; ++iz)
      for (int ix = 0; ix < nx; ++ix) out.push_back(ix + nx * (iy + ny * iz));
  } else {
    const int iz = hi ? nz - 1 : 0;
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) out.push_back(ix + nx * (iy + ny * iz));
  }
  return out;
}

// ---- profiling -------------------------------------------------------------
// Each timed region reserves one (start, end) event pair on the context's
// stream; tt_profile_read sums the elapsed times per class.
long prof_begin(tt_ctx* c, int cls) {
  if (!c->prof || !((c->prof_mask >> cls) & 1u)) return -1;
  if (c->ev_used >= c->ev.size()) {
    if (c->ev.size() >= 200000) return -1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      hipEventDestroy(a);
      return -1;
    }
    c->ev.push_back({cls, {a, b}});
  }
  const long k = (long)c->ev_used++;
  c->ev[k].first = cls;
  hipEventRecord(c->ev[k].second.first, c->st);
  return k;
}
void prof_end(tt_ctx* c, long k) {
  if (k < 0) return;
  hipEventRecord(c->ev[k].second.second, c->st);
}
struct Prof {
  tt_ctx* c;
  long k;
  Prof(tt_ctx* c_, int cls) : c(c_), k(prof_begin(c_, cls)) {}
  ~Prof() { prof_end(c, k); }
};

// One Gram-SVD truncation of the SVD of M given the eigen-decompositions of
// both Gram matrices in slots ea (A side) and eb (B side); writes P (R x r')
// and M_upd (r' x R).
void truncate_bond(tt_ctx* c, int bond, const EigSlot& ea, const EigSlot& eb, EigSlot& em,
                   double* M, double* Cm, double* Wm, double* Ur, double* P, double* Mupd,
                   int Rcap, int rcap, int Rdim, double tol, int rmax) {
  hipStream_t s = c->st;
  const int ka = bond == 1 ? D_KA1 : D_KA2, kb = bond == 1 ? D_KB1 : D_KB2;
  const int km = bond == 1 ? D_KM1 : D_KM2, side = bond == 1 ? D_SIDE1 : D_SIDE2;
  const int rn = bond == 1 ? D_R1N : D_R2N, zero = bond == 1 ? D_ZERO1 : D_ZERO2;
  const int kea = bond == 1 ? D_KEA1 : D_KEA2, keb = bond == 1 ? D_KEB1 : D_KEB2;
  const int kc = bond == 1 ? D_KC1 : D_KC2, tgk = bond == 1 ? D_TGK1 : D_TGK2;
  const int N = c->N;
  const DimExpr abound = bond == 1 ? dimc(c->ns) : dimv(D_R1NT);
  const DimExpr bbound = bond == 1 ? dimc(c->nt * c->np) : dimc(c->np);
  const int qcap = bond == 1 ? c->q1c : c->q2c;
  launch_mside(c->dims, ka, kb, km, side, abound, bbound, s);
  {
    Prof p(c, P_SMALL);
    GemmDesc g = gd(ea.V, N, 1, eb.V, N, 0, M, Rcap, dimv(ka), dimv(kb), dimv(Rdim));
    g.rowscale = ea.sq;
    g.colscale = eb.sq;
    gemm(g, Rcap, Rcap, 1, c->dims, s);
  }
  {
    // SVD of M (App. A.2) through the Golub-Kahan tridiagonal
    Prof p(c, bond == 1 ? P_EIGM1 : P_EIGM2);
    EigJob j{Cm, Rcap, tgk, em.lam, em.V, N, em.sq, em.isq, kc, 1.0, em.work};
    svd_short_side(M, Rcap, ka, kb, side, j, 2 * qcap, Rcap, c->dims, s);
  }
  RankArgs ra;
  ra.bond = bond; ra.km = km; ra.kc = kc; ra.ka = ka; ra.kb = kb;
  ra.rn = rn; ra.zero = zero; ra.kea = kea; ra.keb = keb;
  ra.replay = bond == 1 ? D_REPLAY1 : D_REPLAY2;
  ra.rnt = bond == 1 ? D_R1NT : -1;
  ra.nt = c->nt;
  ra.tol = tol;
  ra.eta = 1e-12;
  ra.rmax = std::min(rmax > 0 ? rmax : rcap, rcap);
  ra.rdim = Rdim;
  ra.g_tail = bond == 1 ? G_TAIL1 : G_TAIL2;
  ra.g_sr = bond == 1 ? G_SR1 : G_SR2;
  ra.g_srp = bond == 1 ? G_SR1P : G_SR2P;
  ra.g_rn = bond == 1 ? G_R1N : G_R2N;
  ra.g_ka = bond == 1 ? G_KA1 : G_KA2;
  ra.g_kb = bond == 1 ? G_KB1 : G_KB2;
  launch_rank(em.lam, c->dims, c->diag, ra, s);
  Prof p(c, P_SMALL);
  // side 0: W = M^T U~ ; side 1: U~ = M V~ S~^-1
  GemmDesc g0 = gd(M, Rcap, 1, em.V, N, 0, Wm, rcap, dimv(kb), dimv(rn), dimv(ka));
  g0.cond_idx = side; g0.cond_val = 0;
  gemm(g0, Rcap, rcap, 1, c->dims, s);
  GemmDesc g1 = gd(M, Rcap, 0, em.V, N, 0, Ur, rcap, dimv(ka), dimv(rn), dimv(kb));
  g1.cond_idx = side; g1.cond_val = 1;
  g1.colscale = em.isq;
  gemm(g1, Rcap, rcap, 1, c->dims, s);
  launch_svd_vectors(em.V, N, em.sq, Ur, rcap, Wm, rcap, c->dims, ka, kb, side, rn, zero, rcap, s);
  // P = V_A S_A^-1 U~  (R x r');  M_upd = (V_B S_B^-1 V~ S~)^T  (r' x R)
  GemmDesc gp = gd(ea.V, N, 0, Ur, rcap, 0, P, rcap, dimv(Rdim), dimv(rn), dimv(kea));
  gp.kscale = ea.isq;
  gemm(gp, Rcap, rcap, 1, c->dims, s);
  GemmDesc gm = gd(Wm, rcap, 1, eb.V, N, 1, Mupd, Rcap, dimv(rn), dimv(Rdim), dimv(keb));
  gm.kscale = eb.isq;
  gemm(gm, rcap, Rcap, 1, c->dims, s);
}

// Gram-SVD rounding (App. A Algorithm 1, d = 3) of the TT held in
// (xc, ldxc) / Thcat / Phcat with concatenated ranks dims[RC1], dims[RC2].
// xcf != nullptr: the FP32-mixed form (X_cat in FP32, sliced Gram and
// split-product update on FP32 MFMA, X' written to Xnf); else FP64 (X' to Xn).
void round_pipeline(tt_ctx* c, const double* xc, int ldxc, int ncap1, double tol, int rmax,
                    const float* xcf = nullptr) {
  hipStream_t s = c->st;
  const int nt = c->nt, np = c->np, R1c = c->R1c, R2c = c->R2c, N = c->N;
  {
    Prof p(c, P_SMALL);
    // backward sweep Grams: G_R3 = Phcat Phcat^T ; G_B1 = sum_l Thcat_l G_R3 Thcat_l^T
    gemm(gd(c->Phcat, np, 0, c->Phcat, np, 1, c->GR3, R2c, dimv(D_RC2), dimv(D_RC2), dimc(np)),
         R2c, R2c, 1, c->dims, s);
    gemm(gd(c->Thcat, R2c, 0, c->GR3, R2c, 0, c->T1, R2c, dimv(D_RC1, nt), dimv(D_RC2), dimv(D_RC2)),
         R1c * nt, R2c, 1, c->dims, s);
    // G_B1 = sum_l T1_l Thcat_l^T, one partial per ordinate l over the live
    // R2 (batched), then a fixed-order sum
    GemmDesc gb = gd(c->T1, nt * R2c, 0, c->Thcat, nt * R2c, 1, c->gpart, R1c, dimv(D_RC1),
                     dimv(D_RC1), dimv(D_RC2));
    gb.sA = gb.sB = R2c;
    gb.sC = (long long)R1c * R1c;
    gemm(gb, R1c, R1c, nt, c->dims, s);
    sum_partials(c->gpart, (long long)R1c * R1c, nt, c->GB1, R1c, R1c, dimv(D_RC1), dimv(D_RC1),
                 R1c, R1c, c->dims, s);
  }
  {
    GramPlan plan = gram_plan(c->ns, ncap1, ldxc);
    {
      Prof p(c, P_GRAM);
      if (xcf) gram_split_partial(plan, xcf, dimv(D_RC1), c->colmax, c->gpart, c->dims, s, c->gram_slices);
      else gram_tall_partial(plan, xc, dimv(D_RC1), c->gpart, c->dims, s);
    }
    Prof p(c, P_GRAMRED);
    if (xcf) gram_split_reduce(plan, dimv(D_RC1), c->gpart, c->GA, R1c, c->dims, s);
    else gram_tall_reduce(plan, dimv(D_RC1), c->gpart, c->GA, R1c, c->dims, s);
  }
  {
    Prof p(c, P_EIG1);
    EigJob jobs[3] = {
        {c->GA, R1c, D_RC1, c->E[0].lam, c->E[0].V, N, c->E[0].sq, c->E[0].isq, D_KA1, 1.0, c->E[0].work},
        {c->GB1, R1c, D_RC1, c->E[1].lam, c->E[1].V, N, c->E[1].sq, c->E[1].isq, D_KB1, 1.0, c->E[1].work},
        {c->GR3, R2c, D_RC2, c->E[2].lam, c->E[2].V, N, c->E[2].sq, c->E[2].isq, D_KB2, 1.0, c->E[2].work}};
    eig_batched(jobs, 3, N, c->dims, s);
  }
  truncate_bond(c, 1, c->E[0], c->E[1], c->E[3], c->M1, c->C1, c->Wm1, c->Ur1, c->P1, c->Mupd1,
                R1c, c->r1c, D_RC1, tol, rmax);
  {
    Prof p(c, P_XUPD);
    if (xcf)
      gemm_tall_f32(c->ns, xcf, ldxc, c->P1, c->r1c, c->Xnf, c->ldX, dimv(D_RC1), dimv(D_R1N),
                    c->r1c, c->dims, s);
    else
      gemm_tall(c->ns, xc, ldxc, c->P1, c->r1c, c->Xn, c->ldX, dimv(D_RC1), dimv(D_R1N), R1c,
                c->r1c, c->dims, s);
  }
  {
    Prof p(c, P_SMALL);
    gemm(gd(c->Mupd1, R1c, 0, c->Thcat, nt * R2c, 0, c->Thp, nt * R2c, dimv(D_R1N), dimc(nt * R2c),
            dimv(D_RC1)),
         c->r1c, nt * R2c, 1, c->dims, s);
    // bond 2: G_A2 = sum_l Theta'_l^T Theta'_l, one partial per ordinate l
    GemmDesc gl = gd(c->Thp, nt * R2c, 1, c->Thp, nt * R2c, 0, c->gpart, R2c, dimv(D_RC2),
                     dimv(D_RC2), dimv(D_R1N));
    gl.sA = gl.sB = R2c;
    gl.sC = (long long)R2c * R2c;
    gemm(gl, R2c, R2c, nt, c->dims, s);
    sum_partials(c->gpart, (long long)R2c * R2c, nt, c->GL2, R2c, R2c, dimv(D_RC2), dimv(D_RC2),
                 R2c, R2c, c->dims, s);
  }
  {
    Prof p(c, P_EIG2);
    EigJob j = {c->GL2, R2c, D_RC2, c->E[4].lam, c->E[4].V, N, c->E[4].sq, c->E[4].isq, D_KA2, 1.0, c->E[4].work};
    // sized by the bond-2 capacity: fewer divide-and-conquer levels than N
    eig_batched(&j, 1, R2c, c->dims, s);
  }
  truncate_bond(c, 2, c->E[4], c->E[2], c->E[5], c->M2, c->C2, c->Wm2, c->Ur2, c->P2, c->Mupd2,
                R2c, c->r2c, D_RC2, tol, rmax);
  {
    Prof p(c, P_SMALL);
    gemm(gd(c->Thp, R2c, 0, c->P2, c->r2c, 0, c->Th, c->r2c, dimv(D_R1NT), dimv(D_R2N), dimv(D_RC2)),
         c->r1c * nt, c->r2c, 1, c->dims, s);
    gemm(gd(c->Mupd2, R2c, 0, c->Phcat, np, 0, c->Ph, np, dimv(D_R2N), dimc(np), dimv(D_RC2)),
         c->r2c, np, 1, c->dims, s);
  }
}

// Ranks of the next replayed rounding: schedule entry dims[D_SCHEDPOS] (0
// past its end: the rank rule), then the position advances.
__global__ void k_set_replay(int* dims, const int* sched, int n) {
  if (threadIdx.x == 0) {
    const int k = dims[D_SCHEDPOS];
    dims[D_REPLAY1] = k < n ? sched[2 * k] : 0;
    dims[D_REPLAY2] = k < n ? sched[2 * k + 1] : 0;
    dims[D_SCHEDPOS] = k + 1;
  }
}

__global__ void k_set_dim(int* dims, int idx, int v) {
  if (threadIdx.x == 0) dims[idx] = v;
}

tt_status check_flags(tt_ctx* c) {
  int flag = 0;
  HIPCHK(c, hipMemcpyAsync(&flag, c->dims + D_FLAG, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (flag) {
    c->poisoned = true;
    std::string m = "numerical failure:";
    if (flag & FLAG_NONFINITE) m += " non-finite state";
    if (flag & FLAG_NEWTON) m += " Newton did not converge";
    if (flag & FLAG_EIG) m += " eigensolver produced a non-finite value";
    if (flag & FLAG_NOCONV) m += " the Jacobi SVD did not converge";
    if (flag & FLAG_BARRIER)
      m += " a grid barrier of a multi-block eigensolver timed out (blocks not co-resident)";
    return fail(c, TT_ERR_NUMERIC, m);
  }
  return TT_OK;
}

void energy_of_state(tt_ctx* c, double* E) {
  if (c->mixed) {
    launch_energy(c->Xf, c->ldX, c->ns, c->Th, c->nt, c->r2c, c->Ph, c->np, c->w, c->v, c->pv, c->z,
                  dimv(D_R1), dimv(D_R2), 1.0 / c->cfg.c, E, c->dims, c->r1c, c->r2c, c->st);
    return;
  }
  launch_energy(c->X, c->ldX, c->ns, c->Th, c->nt, c->r2c, c->Ph, c->np, c->w, c->v, c->pv, c->z,
                dimv(D_R1), dimv(D_R2), 1.0 / c->cfg.c, E, c->dims, c->r1c, c->r2c, c->st);
}

}  // namespace

namespace tt {

tt_status ctx_fail(tt_ctx* c, tt_status code, const std::string& msg) { return fail(c, code, msg); }

void step_body_frozen(tt_ctx* c) {
  hipStream_t s = c->st;
  launch_concat_dims(c->G, c->dims, s);
  launch_build_phcat(c->G, c->Ph, c->pfac, c->bc_p, c->Phcat, c->dims, s);
  launch_build_thcat(c->G, c->Th, c->tfac, c->bc_t, c->Thcat, c->dims, s);
  if (c->mixed) {
    launch_build_xcat(c->G, c->Xf, c->ldX, c->bc_e, c->d, c->s, c->Xcatf, c->ldC, c->dims, 1, s);
    round_pipeline(c, nullptr, c->ldC, c->R1c, c->cfg.tol, c->cfg.rmax, c->Xcatf);
  } else {
    launch_build_xcat(c->G, c->X, c->ldX, c->bc_e, c->d, c->s, c->Xcat, c->ldC, c->dims, 1, s);
    round_pipeline(c, c->Xcat, c->ldC, c->R1c, c->cfg.tol, c->cfg.rmax);
  }
}

}  // namespace tt

namespace {

// Every launch of one step on c->st, with its host bookkeeping (state
// buffer swaps, history count, schedule position).  No host synchronisation
// and no memset, so the sequence can be captured as a graph.
void step_once(tt_ctx* c) {
  hipStream_t s = c->st;
  const tt_config& cf = c->cfg;
  const bool coupled = cf.material == TT_MAT_COUPLED;
  // the source coefficients depend on this step's E* (Newton, or J^{m+1})
  const bool dyn = coupled || c->scatter;
  const double* ks = c->scatter ? c->kappa_s : nullptr;
  const bool twice = cf.schedule == TT_ROUND_TWICE;
  auto replay_next = [&]() {
    if (cf.rank_mode == TT_RANK_REPLAY) {
      k_set_replay<<<1, 64, 0, s>>>(c->dims, c->sched, c->nsched);
      c->sched_pos++;
    }
  };
  auto swap_state = [&]() {
    if (c->mixed) std::swap(c->Xf, c->Xnf);
    else std::swap(c->X, c->Xn);
  };
  replay_next();
  if (!twice) {
    {
      Prof p(c, P_CONCAT);
      launch_concat_dims(c->G, c->dims, s);
      launch_build_phcat(c->G, c->Ph, c->pfac, c->bc_p, c->Phcat, c->dims, s);
      launch_build_thcat(c->G, c->Th, c->tfac, c->bc_t, c->Thcat, c->dims, s);
    }
    if (dyn) {
      Prof p(c, P_MAT);
      // E* = (1/c) X_tr z over the transport columns (source column
      // excluded), X_tr formed from X on the fly, so that X_cat is written
      // once, with the source coefficients
      if (c->mixed)
        launch_energy_xcat(c->G, c->Xf, c->ldX, c->bc_e, c->Thcat, c->Phcat, c->w, c->v, c->pv,
                           c->z, dimv(D_RC2), 1.0 / cf.c, c->Estar, c->dims, s);
      else
        // Y in X_cat's buffer, free until the build below writes it
        launch_energy_xcat(c->G, c->X, c->ldX, c->bc_e, c->Thcat, c->Phcat, c->w, c->v, c->pv,
                           c->z, dimv(D_RC2), 1.0 / cf.c, c->Estar, c->Xcat, c->zt, c->dims, s);
      launch_material(c->ns, cf.c, c->dt, cf.a_r, coupled ? 1 : 0, c->kappa, ks, c->rho, c->cv,
                      c->T, c->Estar, c->Tdag, c->d, c->s, c->dims, s);
    }
    {
      Prof p(c, P_CONCAT);
      if (c->mixed)
        launch_build_xcat(c->G, c->Xf, c->ldX, c->bc_e, c->d, c->s, c->Xcatf, c->ldC, c->dims, 1, s);
      else
        launch_build_xcat(c->G, c->X, c->ldX, c->bc_e, c->d, c->s, c->Xcat, c->ldC, c->dims, 1, s);
    }
    if (c->mixed) round_pipeline(c, nullptr, c->ldC, c->R1c, cf.tol, cf.rmax, c->Xcatf);
    else round_pipeline(c, c->Xcat, c->ldC, c->R1c, cf.tol, cf.rmax);
  } else {
    // Sec. 4.2: round the transport sum, apply the source update to the
    // rounded state, round again
    StepGeom Gt = c->G;
    Gt.nem = 0;
    {
      Prof p(c, P_CONCAT);
      launch_transport_dims(Gt, c->dims, s);
      launch_build_phcat(Gt, c->Ph, c->pfac, c->bc_p, c->Phcat, c->dims, s);
      launch_build_thcat(Gt, c->Th, c->tfac, c->bc_t, c->Thcat, c->dims, s);
      if (c->mixed)
        launch_build_xcat(Gt, c->Xf, c->ldX, c->bc_e, c->d, c->s, c->Xcatf, c->ldC, c->dims, 0, s);
      else
        launch_build_xcat(Gt, c->X, c->ldX, c->bc_e, c->d, c->s, c->Xcat, c->ldC, c->dims, 0, s);
    }
    if (c->mixed) round_pipeline(c, nullptr, c->ldC, c->R1c, cf.tol, cf.rmax, c->Xcatf);
    else round_pipeline(c, c->Xcat, c->ldC, c->R1c, cf.tol, cf.rmax);
    launch_finish(c->dims, nullptr, 0, s);
    swap_state();
    if (dyn) {
      Prof p(c, P_MAT);
      energy_of_state(c, c->Estar);
      launch_material(c->ns, cf.c, c->dt, cf.a_r, coupled ? 1 : 0, c->kappa, ks, c->rho, c->cv,
                      c->T, c->Estar, c->Tdag, c->d, c->s, c->dims, s);
    }
    replay_next();
    {
      Prof p(c, P_CONCAT);
      if (c->mixed)
        launch_source_cat(c->G, c->Xf, c->ldX, c->d, c->s, c->Xcatf, c->ldC, c->Th, c->Ph,
                          c->Thcat, c->Phcat, c->dims, s);
      else
        launch_source_cat(c->G, c->X, c->ldX, c->d, c->s, c->Xcat, c->ldC, c->Th, c->Ph,
                          c->Thcat, c->Phcat, c->dims, s);
    }
    if (c->mixed) round_pipeline(c, nullptr, c->ldC, c->r1c + 1, cf.tol, cf.rmax, c->Xcatf);
    else round_pipeline(c, c->Xcat, c->ldC, c->r1c + 1, cf.tol, cf.rmax);
  }
  launch_finish(c->dims, c->hist, std::max(1, cf.max_steps), s);
  c->nhist = std::min(c->nhist + 1, std::max(1, cf.max_steps));
  swap_state();
  if (coupled) {
    Prof p(c, P_MAT);
    energy_of_state(c, c->Enew);
    launch_temperature(c->ns, c->rho, c->cv, c->Estar, c->Enew, c->T, s);
  }
}

void graphs_drop(tt_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) hipGraphExecDestroy(c->gexec[k]);
    c->gexec[k] = nullptr;
    c->gkey[k] = nullptr;
  }
}

// One step by graph replay.  The step's launches depend on the host state
// only through which buffer holds the state (the swaps alternate it), so
// one graph per buffer is captured on first use, on the context's own
// capture stream (the null stream cannot be captured), and launched on
// c->st.  The host bookkeeping the capture performed is undone and then
// applied after each launch, as step_once does.
hipError_t step_graph(tt_ctx* c) {
  const void* key = c->mixed ? (const void*)c->Xf : (const void*)c->X;
  int k = c->gkey[0] == key ? 0 : c->gkey[1] == key ? 1 : -1;
  if (k < 0) {
    k = c->gexec[0] ? 1 : 0;
    if (c->gexec[k]) {
      graphs_drop(c);
      k = 0;
    }
    hipError_t e = hipSuccess;
    if (!c->cap_st) {
      e = hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    hipStream_t st0 = c->st;
    double *X0 = c->X, *Xn0 = c->Xn;
    float *Xf0 = c->Xf, *Xnf0 = c->Xnf;
    const int nh0 = c->nhist, sp0 = c->sched_pos;
    c->st = c->cap_st;
    e = hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      c->st = st0;
      return e;
    }
    step_once(c);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap_st, &g);
    c->gafter[k][0] = c->X;
    c->gafter[k][1] = c->Xn;
    c->gafterf[k][0] = c->Xf;
    c->gafterf[k][1] = c->Xnf;
    c->gsched[k] = c->sched_pos - sp0;
    c->st = st0;
    c->X = X0;
    c->Xn = Xn0;
    c->Xf = Xf0;
    c->Xnf = Xnf0;
    c->nhist = nh0;
    c->sched_pos = sp0;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&c->gexec[k], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec[k] = nullptr;
      return e;
    }
    c->gkey[k] = key;
  }
  const hipError_t e = hipGraphLaunch(c->gexec[k], c->st);
  if (e != hipSuccess) return e;
  c->X = c->gafter[k][0];
  c->Xn = c->gafter[k][1];
  c->Xf = c->gafterf[k][0];
  c->Xnf = c->gafterf[k][1];
  c->sched_pos += c->gsched[k];
  c->nhist = std::min(c->nhist + 1, std::max(1, c->cfg.max_steps));
  return hipSuccess;
}

}  // namespace

// ============================================================================
extern "C" {

size_t tt_workspace_bytes(const tt_config* cfg, int32_t n_inflow) {
  std::string why;
  if (!validate(cfg, n_inflow, why)) {
    g_err = why;
    return 0;
  }
  tt_ctx tmp;
  geometry(&tmp, *cfg, n_inflow, 1);
  if (tmp.N > 1024) {
    g_err = "concatenated rank capacity above 1024 (lower rmax)";
    return 0;
  }
  return carve(&tmp, nullptr);
}

tt_status tt_create(const tt_config* cfg, const double* kappa, const double* rho, const double* cv,
                    const double* T0, const tt_inflow* inflow, int32_t n_inflow, const double* X0,
                    const double* Th0, const double* Ph0, int32_t r1, int32_t r2,
                    void* dev_workspace, size_t ws_bytes, void* hip_stream, tt_ctx** out) {
  if (!out) return fail(nullptr, TT_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  std::string why;
  if (!validate(cfg, n_inflow, why)) return fail(nullptr, TT_ERR_INVALID_ARG, why);
  if (!kappa || !T0 || !X0 || !Th0 || !Ph0 || (n_inflow > 0 && !inflow))
    return fail(nullptr, TT_ERR_INVALID_ARG, "null input array");
  tt_ctx* c = new tt_ctx();
  const int nz = cfg->dim == 3 ? cfg->nz : 1;
  const int ns = cfg->nx * cfg->ny * nz;
  geometry(c, *cfg, n_inflow, 1);  // emission slot always reserved
  const int nem = emission_flag(*cfg, T0, ns);
  c->nem = nem;
  c->nem_base = nem;
  c->G.nem = nem;
  c->st = (hipStream_t)hip_stream;
  for (int k = 0; k < n_inflow; ++k) {
    const int f = inflow[k].face;
    if (f < 0 || f >= 2 * cfg->dim || !inflow[k].face_w || !inflow[k].theta_w || !inflow[k].phi_w) {
      delete c;
      return fail(nullptr, TT_ERR_INVALID_ARG, "bad inflow term");
    }
    const int bc = (f % 2) ? cfg->bc_hi[f / 2] : cfg->bc_lo[f / 2];
    if (bc != TT_BC_INFLOW) {
      delete c;
      return fail(nullptr, TT_ERR_INVALID_ARG, "inflow term on a face whose bc is not TT_BC_INFLOW");
    }
    const size_t nface = face_cells(c, f).size();
    if (!all_finite(inflow[k].face_w, nface) || !all_finite(inflow[k].theta_w, c->nt) ||
        !all_finite(inflow[k].phi_w, c->np)) {
      delete c;
      return fail(nullptr, TT_ERR_INVALID_ARG, "non-finite inflow weights");
    }
  }
  if (r1 < 1 || r2 < 1 || r1 > c->r1c || r2 > c->r2c) {
    delete c;
    return fail(nullptr, TT_ERR_INVALID_ARG, "initial ranks exceed the rank capacity");
  }
  {
    // host inputs: finite, and in range, before any device work
    std::string bad;
    for (int i = 0; i < ns && bad.empty(); ++i) {
      if (!(kappa[i] >= 0 && kappa[i] <= 1.79e308)) bad = "kappa must be finite and >= 0";
      else if (rho && !(rho[i] > 0 && rho[i] <= 1.79e308)) bad = "rho must be finite and > 0";
      else if (cv && !(cv[i] > 0 && cv[i] <= 1.79e308)) bad = "cv must be finite and > 0";
      else if (!(T0[i] >= 0 && T0[i] <= 1.79e308)) bad = "T0 must be finite and >= 0";
    }
    if (bad.empty() && (!all_finite(X0, (size_t)ns * r1) || !all_finite(Th0, (size_t)r1 * c->nt * r2) ||
                        !all_finite(Ph0, (size_t)r2 * c->np)))
      bad = "non-finite initial cores";
    if (!bad.empty()) {
      delete c;
      return fail(nullptr, TT_ERR_INVALID_ARG, bad);
    }
  }
  if (c->N > 1024) {
    delete c;
    return fail(nullptr, TT_ERR_INVALID_ARG, "concatenated rank capacity above 1024 (lower rmax)");
  }
  c->ws_need = carve(c, nullptr);
  if (!dev_workspace || ws_bytes < c->ws_need) {
    delete c;
    return fail(nullptr, TT_ERR_OOM, "workspace too small: need " + std::to_string(tt_workspace_bytes(cfg, n_inflow)) + " bytes");
  }
  {
    // every eigensolver / SVD launch of a step must fit one CU's LDS
    const char *w1 = "", *w2 = "", *w3 = "", *w4 = "";
    const size_t l1 = eig_lds_bytes(c->N, true, &w1), l2 = eig_lds_bytes(c->R2c, true, &w2);
    const size_t l3 = svd_lds_bytes(2 * c->q1c, c->R1c, true, &w3);
    const size_t l4 = svd_lds_bytes(2 * c->q2c, c->R2c, true, &w4);
    const char* bad = !lds_fits(l1) ? w1 : !lds_fits(l2) ? w2 : !lds_fits(l3) ? w3 : !lds_fits(l4) ? w4 : nullptr;
    if (bad) {
      delete c;
      return fail(nullptr, TT_ERR_INVALID_ARG, std::string("LDS above 160 KiB in ") + bad);
    }
  }
  carve(c, (char*)dev_workspace);
  hipStream_t s = c->st;
  HIPCHK(nullptr, hipMemsetAsync(dev_workspace, 0, c->ws_need, s));
  std::vector<double> w, v, tf, pf, mu, sint, cosp, sinp;
  host_factors(c, w, v, tf, pf, mu, sint, cosp, sinp);
  HIPCHK(nullptr, hipMemcpyAsync(c->w, w.data(), w.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(nullptr, hipMemcpyAsync(c->v, v.data(), v.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(nullptr, hipMemcpyAsync(c->tfac, tf.data(), tf.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(nullptr, hipMemcpyAsync(c->pfac, pf.data(), pf.size() * 8, hipMemcpyHostToDevice, s));
  // inflow rank-1 terms: e (x) tpart (x) ppart
  const int nbk = std::max(1, c->nbc);
  std::vector<double> be((size_t)nbk * ns, 0.0), bt((size_t)nbk * c->nt, 0.0), bp((size_t)nbk * c->np, 0.0);
  // Dirichlet ghost value g = face_w (x) theta_w (x) phi_w of each entry: the
  // part of the flux through its face that the stencil blocks (ghost rows
  // zero) leave out, as rank-1 terms e_face (x) t (x) p (Sec. 4.5).
  // HLL: the ghost value enters F at the face with the face's weight, per
  // sign of n (term j = 0: n >= 0, j = 1: n < 0): + lam n alpha_lo g on a lo
  // face, - lam n beta_hi g on a hi face; the spatial part is weighted on
  // the device (k_hll_inflow, code = 4 axis + weight slot).
  const bool rus = cfg->flux == TT_FLUX_RUSANOV, dif = rusanov_diffusion(*cfg);
  const bool hll = cfg->flux == TT_FLUX_HLL;
  const int per = dif || hll ? 2 : 1;
  std::vector<int> code((size_t)nbk, 0);
  for (int k = 0; k < n_inflow; ++k) {
    const int f = inflow[k].face, a = f / 2, hi = f % 2;
    std::vector<int> cells = face_cells(c, f);
    const double lam = c->lam[a];
    for (int j = 0; j < per; ++j) {
      const size_t kb = (size_t)k * per + j;  // rank-1 term index
      for (size_t q = 0; q < cells.size(); ++q) be[kb * ns + cells[q]] = inflow[k].face_w[q];
      const bool neg = hll ? j == 1 : hi;  // upwind: the incoming sign only
      if (hll) code[kb] = 4 * a + (hi ? (j ? HLLW_AP_HI : HLLW_BP_HI) : (j ? HLLW_BP_LO : HLLW_AP_LO));
      for (int l = 0; l < c->nt; ++l) {
        double tfv;
        if (rus) tfv = j == 1 ? 1.0 : (a < 2 ? sint[l] : mu[l]);
        else tfv = a < 2 ? sint[l] : (neg ? std::min(mu[l], 0.0) : std::max(mu[l], 0.0));
        bt[kb * c->nt + l] = tfv * inflow[k].theta_w[l];
      }
      for (int p = 0; p < c->np; ++p) {
        const double n = a == 0 ? cosp[p] : a == 1 ? sinp[p] : 1.0;
        const double sl = hi ? -lam : lam;
        double pfv;
        if (rus) pfv = j == 1 ? 0.5 * lam * cfg->s_plus : (hi ? -0.5 : 0.5) * lam * n;
        else if (a < 2) pfv = sl * (neg ? std::min(n, 0.0) : std::max(n, 0.0));
        else pfv = sl;
        bp[kb * c->np + p] = pfv * inflow[k].phi_w[p];
      }
    }
  }
  if (n_inflow > 0) {
    HIPCHK(nullptr, hipMemcpyAsync(hll ? c->bc_e0 : c->bc_e, be.data(), be.size() * 8,
                                   hipMemcpyHostToDevice, s));
    if (hll) HIPCHK(nullptr, hipMemcpyAsync(c->bc_code, code.data(), code.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(nullptr, hipMemcpyAsync(c->bc_t, bt.data(), bt.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(nullptr, hipMemcpyAsync(c->bc_p, bp.data(), bp.size() * 8, hipMemcpyHostToDevice, s));
  }
  c->h_rho.assign(ns, 1.0);
  c->h_cv.assign(ns, 1.0);
  if (rho) std::copy(rho, rho + ns, c->h_rho.begin());
  if (cv) std::copy(cv, cv + ns, c->h_cv.begin());
  HIPCHK(nullptr, hipMemcpyAsync(c->kappa, kappa, ns * 8, hipMemcpyHostToDevice, s));
  HIPCHK(nullptr, hipMemcpyAsync(c->rho, c->h_rho.data(), ns * 8, hipMemcpyHostToDevice, s));
  HIPCHK(nullptr, hipMemcpyAsync(c->cv, c->h_cv.data(), ns * 8, hipMemcpyHostToDevice, s));
  HIPCHK(nullptr, hipMemcpyAsync(c->T, T0, ns * 8, hipMemcpyHostToDevice, s));
  hll_refresh(c);
  HIPCHK(nullptr, hipGetLastError());
  HIPCHK(nullptr, hipStreamSynchronize(s));
  const int32_t rr[2] = {r1, r2};
  tt_status st = tt_set_cores(c, X0, Th0, Ph0, rr);
  if (st != TT_OK) {
    g_err = c->err;
    delete c;
    return st;
  }
  *out = c;
  return TT_OK;
}

tt_status tt_set_cores(tt_ctx* c, const double* X, const double* Th, const double* Ph,
                       const int32_t r[2]) {
  if (!c || !X || !Th || !Ph || !r) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  if (r[0] < 1 || r[1] < 1 || r[0] > c->r1c || r[1] > c->r2c)
    return fail(c, TT_ERR_INVALID_ARG, "ranks exceed the rank capacity");
  if (!all_finite(X, (size_t)c->ns * r[0]) || !all_finite(Th, (size_t)r[0] * c->nt * r[1]) ||
      !all_finite(Ph, (size_t)r[1] * c->np))
    return fail(c, TT_ERR_INVALID_ARG, "non-finite cores");
  hipStream_t s = c->st;
  // the padded device layouts are filled from host staging copies by plain
  // 1D transfers (kept alive until the synchronisation below)
  const size_t xs = (size_t)c->ns * c->ldX, ths = (size_t)c->r1c * c->nt * c->r2c;
  std::vector<double> hx(xs, 0.0), ht(ths, 0.0);
  for (int i = 0; i < c->ns; ++i) memcpy(&hx[(size_t)i * c->ldX], X + (size_t)i * r[0], (size_t)r[0] * 8);
  for (size_t q = 0; q < (size_t)r[0] * c->nt; ++q)
    memcpy(&ht[q * c->r2c], Th + q * r[1], (size_t)r[1] * 8);
  HIPCHK(c, hipMemcpyAsync(c->X, hx.data(), xs * 8, hipMemcpyHostToDevice, s));
  if (c->mixed) launch_convert(c->X, c->ldX, c->Xf, c->ldX, c->ns, c->ldX, s);
  HIPCHK(c, hipMemcpyAsync(c->Th, ht.data(), ths * 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->Ph, Ph, (size_t)r[1] * c->np * 8, hipMemcpyHostToDevice, s));
  int hd[D_NDIMS];
  memset(hd, 0, sizeof(hd));
  hd[D_R1] = r[0];
  hd[D_R2] = r[1];
  hd[D_JAC_MAXSW] = c->jac_maxsw;
  HIPCHK(c, hipMemcpyAsync(c->dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  // frozen material without scattering: the source coefficients never change
  launch_material(c->ns, c->cfg.c, c->dt, c->cfg.a_r, 0, c->kappa, nullptr, c->rho, c->cv, c->T,
                  c->Estar, c->Tdag, c->d, c->s, c->dims, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(s));
  c->poisoned = false;
  c->nhist = 0;
  c->sched_pos = 0;
  c->gb.stale = false;
  return TT_OK;
}

tt_status tt_step(tt_ctx* c, int32_t nsteps) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (c->poisoned) return fail(c, TT_ERR_STATE, "context poisoned by an earlier numerical failure");
  if (nsteps < 0) return fail(c, TT_ERR_INVALID_ARG, "nsteps < 0");
  hipStream_t s = c->st;
  const tt_config& cf = c->cfg;
  if (c->gb.on && c->nhist + nsteps > std::max(1, cf.max_steps))
    return fail(c, TT_ERR_STATE, "tape full: more steps since tt_set_cores than max_steps");
  // graph replay unless a step needs host work of its own (event timing,
  // the gradient tape's checkpoints)
  const bool use_graph = c->graphs && !c->prof && !c->gb.on;
  for (int m = 0; m < nsteps; ++m) {
    if (use_graph) {
      const hipError_t e = step_graph(c);
      if (e == hipSuccess) continue;
      // capture unavailable here: eager steps from now on
      (void)hipGetLastError();
      graphs_drop(c);
      c->graphs = false;
    }
    Prof pstep(c, P_STEP);
    if (c->gb.on) HIPCHK(c, grad_record(c));
    step_once(c);
  }
  HIPCHK(c, hipGetLastError());
  launch_check_state(c->X, c->mixed ? c->Xf : nullptr, c->ldX, c->ns, c->Th, c->nt, c->r2c, c->Ph,
                     c->np, c->T, c->dims, s);
  return check_flags(c);
}

tt_status tt_round(tt_ctx* c, double tol, int32_t rmax, int32_t ranks_out[2]) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (c->poisoned) return fail(c, TT_ERR_STATE, "context poisoned");
  if (!(tol >= 0)) return fail(c, TT_ERR_INVALID_ARG, "tol must be >= 0");
  hipStream_t s = c->st;
  // the recorded steps no longer end in the stored state
  if (c->gb.on && c->nhist > 0) c->gb.stale = true;
  if (c->cfg.rank_mode == TT_RANK_REPLAY) {
    k_set_replay<<<1, 64, 0, s>>>(c->dims, c->sched, c->nsched);
    c->sched_pos++;
  }
  launch_round_dims(c->dims, s);
  launch_state_as_cat(c->G, c->Th, c->Ph, c->Thcat, c->Phcat, c->dims, s);
  if (c->mixed) round_pipeline(c, nullptr, c->ldX, c->r1c, tol, rmax, c->Xf);
  else round_pipeline(c, c->X, c->ldX, c->r1c, tol, rmax);
  launch_finish(c->dims, nullptr, 0, s);
  if (c->mixed) std::swap(c->Xf, c->Xnf);
  else std::swap(c->X, c->Xn);
  HIPCHK(c, hipGetLastError());
  tt_status st = check_flags(c);
  if (st != TT_OK) return st;
  if (ranks_out) {
    int r[2];
    HIPCHK(c, hipMemcpy(r, c->dims, 2 * sizeof(int), hipMemcpyDeviceToHost));
    ranks_out[0] = r[0];
    ranks_out[1] = r[1];
  }
  return TT_OK;
}

tt_status tt_energy(tt_ctx* c, double* E_dev, double* rad_total, double* mat_total) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  hipStream_t s = c->st;
  double* E = E_dev ? E_dev : c->Enew;
  energy_of_state(c, E);
  HIPCHK(c, hipGetLastError());
  const double dV = (c->cfg.lx / c->cfg.nx) * (c->cfg.ly / c->cfg.ny) *
                    (c->cfg.dim == 3 ? c->cfg.lz / c->cfg.nz : 1.0);
  if (rad_total || mat_total) {
    std::vector<double> hE(c->ns), hT(c->ns);
    HIPCHK(c, hipMemcpyAsync(hE.data(), E, c->ns * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(hT.data(), c->T, c->ns * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double er = 0.0, em = 0.0;
    for (int i = 0; i < c->ns; ++i) {
      er += hE[i];
      em += c->h_rho[i] * c->h_cv[i] * hT[i];
    }
    if (rad_total) *rad_total = er * dV;
    if (mat_total) *mat_total = em * dV;
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return TT_OK;
}

tt_status tt_set_kappa(tt_ctx* c, const double* kappa_dev) {
  if (!c || !kappa_dev) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  HIPCHK(c, hipMemcpyAsync(c->kappa, kappa_dev, c->ns * 8, hipMemcpyDeviceToDevice, c->st));
  if (c->nhist > 0) c->gb.stale = true;  // the taped steps used the old opacity
  launch_material(c->ns, c->cfg.c, c->dt, c->cfg.a_r, 0, c->kappa, nullptr, c->rho, c->cv, c->T,
                  c->Estar, c->Tdag, c->d, c->s, c->dims, c->st);
  hll_refresh(c);  // the HLL face weights depend on kappa
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  return TT_OK;
}

tt_status tt_set_scattering(tt_ctx* c, const double* kappa_s) {
  if (!c || !kappa_s) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  if (c->cfg.ckpt_every > 0)
    return fail(c, TT_ERR_INVALID_ARG, "scattering is not covered by the adjoint (ckpt_every > 0)");
  bool any = false;
  for (int i = 0; i < c->ns; ++i) {
    if (!(kappa_s[i] >= 0 && kappa_s[i] <= 1.79e308))
      return fail(c, TT_ERR_INVALID_ARG, "kappa_s must be finite and >= 0");
    any = any || kappa_s[i] > 0;
  }
  HIPCHK(c, hipMemcpyAsync(c->kappa_s, kappa_s, c->ns * 8, hipMemcpyHostToDevice, c->st));
  hll_refresh(c);  // the HLL face weights depend on kappa_s
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->scatter = any;
  // the isotropic source block carries the scattering term
  c->nem = (c->nem_base || any) ? 1 : 0;
  c->G.nem = c->nem;
  graphs_drop(c);  // the step's launch list changed
  return TT_OK;
}

tt_status tt_detector_loss(tt_ctx* c, const double* detector_w, double* loss_out) {
  if (!c || !detector_w || !loss_out) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  if (!all_finite(detector_w, c->ns)) return fail(c, TT_ERR_INVALID_ARG, "non-finite detector weights");
  hipStream_t s = c->st;
  HIPCHK(c, hipMemcpyAsync(c->wbuf, detector_w, c->ns * 8, hipMemcpyHostToDevice, s));
  energy_of_state(c, c->Enew);
  launch_wdot(c->wbuf, c->Enew, c->ns, c->lossbuf, s);
  HIPCHK(c, hipGetLastError());
  double L = 0.0;
  HIPCHK(c, hipMemcpyAsync(&L, c->lossbuf, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const double dV = (c->cfg.lx / c->cfg.nx) * (c->cfg.ly / c->cfg.ny) *
                    (c->cfg.dim == 3 ? c->cfg.lz / c->cfg.nz : 1.0);
  *loss_out = L * dV;
  return TT_OK;
}

tt_status tt_get_cores(tt_ctx* c, double* X, double* Th, double* Ph, int32_t r[2]) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  int rr[2];
  HIPCHK(c, hipMemcpyAsync(rr, c->dims, 2 * sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (r) { r[0] = rr[0]; r[1] = rr[1]; }
  hipStream_t s = c->st;
  // plain 1D transfers of the padded device layouts into host staging copies,
  // unpacked into the caller's buffers after the synchronisation
  std::vector<double> hx, ht;
  if (X && c->mixed) launch_convert(c->Xf, c->ldX, c->X, c->ldX, c->ns, rr[0], s);
  if (X) {
    hx.resize((size_t)c->ns * c->ldX);
    HIPCHK(c, hipMemcpyAsync(hx.data(), c->X, hx.size() * 8, hipMemcpyDeviceToHost, s));
  }
  if (Th) {
    ht.resize((size_t)rr[0] * c->nt * c->r2c);
    HIPCHK(c, hipMemcpyAsync(ht.data(), c->Th, ht.size() * 8, hipMemcpyDeviceToHost, s));
  }
  if (Ph) HIPCHK(c, hipMemcpyAsync(Ph, c->Ph, (size_t)rr[1] * c->np * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (X)
    for (int i = 0; i < c->ns; ++i) memcpy(X + (size_t)i * rr[0], &hx[(size_t)i * c->ldX], (size_t)rr[0] * 8);
  if (Th)
    for (size_t q = 0; q < (size_t)rr[0] * c->nt; ++q)
      memcpy(Th + q * rr[1], &ht[q * c->r2c], (size_t)rr[1] * 8);
  return TT_OK;
}

tt_status tt_get_temperature(tt_ctx* c, double* T) {
  if (!c || !T) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  HIPCHK(c, hipMemcpyAsync(T, c->T, c->ns * 8, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return TT_OK;
}

tt_status tt_get_rank_history(tt_ctx* c, int32_t* buf, int32_t cap, int32_t* n) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (n) *n = c->nhist;
  const int k = std::min(cap, c->nhist);
  if (buf && k > 0) {
    HIPCHK(c, hipMemcpyAsync(buf, c->hist, 2 * k * sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  return TT_OK;
}

tt_status tt_set_rank_schedule(tt_ctx* c, const int32_t* r1r2, int32_t nroundings) {
  if (!c || (nroundings > 0 && !r1r2)) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  const int per_step = c->cfg.schedule == TT_ROUND_TWICE ? 2 : 1;
  if (nroundings < 0 || nroundings > per_step * std::max(1, c->cfg.max_steps))
    return fail(c, TT_ERR_INVALID_ARG, "schedule longer than the roundings of max_steps steps");
  for (int k = 0; k < 2 * nroundings; ++k)
    if (r1r2[k] < 1 || r1r2[k] > (k % 2 ? c->r2c : c->r1c))
      return fail(c, TT_ERR_INVALID_ARG, "scheduled rank exceeds the rank capacity");
  if (nroundings > 0)
    HIPCHK(c, hipMemcpyAsync(c->sched, r1r2, 2 * nroundings * sizeof(int), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  k_set_dim<<<1, 64, 0, c->st>>>(c->dims, D_SCHEDPOS, 0);
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->nsched = nroundings;
  c->sched_pos = 0;
  graphs_drop(c);  // the replay launches carry the schedule length
  return TT_OK;
}

tt_status tt_get_round_info(tt_ctx* c, double out[16]) {
  if (!c || !out) return fail(c, TT_ERR_INVALID_ARG, "null argument");
  double dg[G_NDIAG];
  HIPCHK(c, hipMemcpyAsync(dg, c->diag, sizeof(dg), hipMemcpyDeviceToHost, c->st));
  int dm[D_NDIMS];
  HIPCHK(c, hipMemcpyAsync(dm, c->dims, sizeof(dm), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  out[0] = dg[G_NORM2]; out[1] = dg[G_DELTA2];
  out[2] = dm[D_KA1]; out[3] = dm[D_KB1]; out[4] = dm[D_KA2]; out[5] = dm[D_KB2];
  out[6] = dm[D_R1N]; out[7] = dm[D_R2N];
  out[8] = dg[G_TAIL1]; out[9] = dg[G_TAIL2];
  out[10] = dg[G_S1]; out[11] = dg[G_SR1]; out[12] = dg[G_SR1P];
  out[13] = dg[G_SR2]; out[14] = dg[G_SR2P]; out[15] = dm[D_RC1];
  return TT_OK;
}

tt_status tt_profile_enable(tt_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->prof = enable != 0;
  // 1: every class; otherwise bit k + 1 selects class k
  c->prof_mask = enable == 1 ? ~0u : ((unsigned)enable >> 1);
  c->ev_used = 0;
  return TT_OK;
}

tt_status tt_profile_read(tt_ctx* c, double* ms, int32_t* count, const char** names, int32_t cap,
                          int32_t* n) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  HIPCHK(c, hipStreamSynchronize(c->st));
  double tot[P_NCLS] = {0};
  int cnt[P_NCLS] = {0};
  for (size_t k = 0; k < c->ev_used; ++k) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->ev[k].second.first, c->ev[k].second.second) == hipSuccess) {
      tot[c->ev[k].first] += t;
      cnt[c->ev[k].first] += 1;
    }
  }
  const int k = std::min<int>(cap, P_NCLS);
  for (int i = 0; i < k; ++i) {
    if (ms) ms[i] = tot[i];
    if (count) count[i] = cnt[i];
    if (names) names[i] = kProfNames[i];
  }
  if (n) *n = P_NCLS;
  return TT_OK;
}

const char* tt_last_error(const tt_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

tt_status tt_set_gram_slices(tt_ctx* c, int32_t slices) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (slices < 1 || slices > 6) return fail(c, TT_ERR_INVALID_ARG, "gram slices must be 1 .. 6");
  HIPCHK(c, hipStreamSynchronize(c->st));
  graphs_drop(c);  // the captured launches name the kernel of the old count
  c->gram_slices = slices;
  return TT_OK;
}

tt_status tt_set_solver_limits(tt_ctx* c, int32_t jacobi_max_sweeps) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  if (jacobi_max_sweeps < 0) return fail(c, TT_ERR_INVALID_ARG, "jacobi_max_sweeps must be >= 0");
  c->jac_maxsw = jacobi_max_sweeps;
  // the kernels read the cap from the device table when they run, so the
  // captured step graphs stay valid
  HIPCHK(c, hipMemcpyAsync(c->dims + D_JAC_MAXSW, &c->jac_maxsw, sizeof(int), hipMemcpyHostToDevice,
                           c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return TT_OK;
}

tt_status tt_use_graphs(tt_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, TT_ERR_INVALID_ARG, "null context");
  HIPCHK(c, hipStreamSynchronize(c->st));
  graphs_drop(c);
  c->graphs = enable != 0;
  return TT_OK;
}

void tt_destroy(tt_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->st);
  graphs_drop(c);
  if (c->cap_st) hipStreamDestroy(c->cap_st);
  for (auto& e : c->ev) {
    hipEventDestroy(e.second.first);
    hipEventDestroy(e.second.second);
  }
  delete c;
}

}  // extern "C"
