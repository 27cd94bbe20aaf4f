// Symmetric FP64 eigensolver for the rank-sized Gram matrices of the
// Gram-SVD truncation (App. A.2: G_A = V_A S_A^2 V_A^T, G_B = V_B S_B^2 V_B^T,
// and the Gram of M for its SVD).
//
// Pipeline (one job per matrix, several jobs run side by side):
//   1. Householder tridiagonalisation A = Q T Q^T (the only step with O(n)
//      sequential dependences): the matrix in one block's registers up to
//      order 160, above that split by rows over 64 blocks' LDS.
//   2. Eigenpairs of T by divide and conquer from 8x8 leaves, all levels in
//      one persistent launch: the merges of a level run side by side, one
//      wavefront per secular root, and the eigenvector updates are tiled
//      products, with grid barriers between the phases.
//   3. Back-transformation V = Q Z, one wavefront per kept vector.
//   4. Descending order, sign gauge (largest |entry| positive), clip rule.
// The same divide and conquer also serves the small SVD of M (section 5).
#include <float.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "gemm_tile.h"
#include "tt_internal.h"

namespace tt {

namespace {

constexpr double U64 = 1.1102230246251565e-16;  // 2^-53

struct EigJobs {
  EigJob j[4];
};

struct Work {
  double *d, *e, *tau, *w, *H, *Z;
};
__device__ inline Work work_of(const EigJob& J, int N) {
  Work W;
  W.d = J.work;
  W.e = W.d + N;
  W.tau = W.e + N;
  W.w = W.tau + N;
  W.H = W.w + N;
  W.Z = W.H + (size_t)N * N;
  return W;
}

__host__ __device__ inline int next_pow2(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Work area of one job at capacity N, before the grid-barrier words: d, e,
// tau, w (4 N), reflectors (N x N), then the divide-and-conquer area.
// d, e, tau, w, H (N x N), then an area that the divide and conquer uses
// and, before it, the grid reductions' exchange buffers (k_gebrd_grid's
// double-buffered partials need 2 (N + 128 N + 128) doubles, more than the
// divide and conquer for small N).
__host__ __device__ inline size_t eig_work_main(int N) {
  const size_t N2 = next_pow2(N);
  const size_t dc = 3 * N2 * N2 + 17 * N2 + 64;
  const size_t grid = 2 * ((size_t)N + 128 * (size_t)N + 128) + 64;
  return 4 * (size_t)N + (size_t)N * N + N2 + (dc > grid ? dc : grid);
}

// Lane exchange inside rows of 16 lanes by DPP, on both halves of a double.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2);
}
__device__ inline double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront, returned on every lane, in a fixed
// order: inside each row of 16 lanes, pairs (lane ^ 1), quads (lane ^ 2),
// half rows (mirror of 8) and rows (mirror of 16), by DPP moves; then the four
// row sums, read from lanes 0, 16, 32 and 48.  At every stage the lanes of a
// row hold bitwise-equal sums (the two operands of each addition only swap),
// so every lane returns the same value.  Call with the whole wavefront active.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// Barrier that orders LDS only: waits for this wavefront's LDS accesses
// (lgkmcnt 0), not for its global stores, then s_barrier.  For loops whose
// global stores nothing in the kernel reads back; the signal fences keep the
// compiler from moving memory accesses across it.
__device__ inline void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt 63, expcnt 7, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Orders one wavefront's LDS accesses (its lanes' writes before their reads),
// for code that one wavefront runs alone (the leaves, the order-64 reduction).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Deterministic block-wide sum (fixed combination order).
template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------------------
// 1. Householder tridiagonalisation (lower form): for k = 0..n-3, H_k =
// I - tau_k v v^T with v = [1, x_2..]/(alpha - beta) annihilates A[k+2:, k].
constexpr int SYR_MAX = 160;  // orders reduced in registers by k_sytrd_reg

// Large orders (n > SYR_MAX): the matrix does not fit one CU's registers,
// and one block streaming the trailing matrix from L2 is bound by that CU's
// share of the memory system.  Instead P blocks per job (32 when their rows
// fit LDS, else SYTRD_GRID_P) each keep the rows i = b (mod P) of the full
// symmetric square in their own LDS
// (at most ceil(N / P) rows), and step k, which needs T_k (the matrix after
// reflectors 0..k-1), runs as:
//   - every block forms row k of T_k from row k of T_{k-1} (published by its
//     owner) and the previous reflector's (v, w), and v_k, tau_k from it,
//     redundantly (same data and fixed-order sums, so identical everywhere);
//   - each block applies T_k = T_{k-1} - v w^T - w v^T to its rows in LDS and
//     in the same pass forms p_k = tau_k T_k,22 v_k on them and its share of
//     p_k^T v_k; the owner of row k+1 publishes it;
//   - one grid barrier; w_k = p_k - (tau_k / 2)(p_k^T v_k) v_k then follows
//     from the published p_k and the partial dots summed in block order.
// Only p, the partial dots and one row cross blocks per step.  The grid (at
// most 4 x 64 blocks of 256 threads) is a small part of what the chip holds
// resident, so an ordinary launch has all blocks resident together (a
// cooperative launch would drain the queue on every call, also when all jobs
// are small and the kernel returns at once); every wait is bounded by
// SYTRD_SPIN_MAX polls, after which the barrier-timeout flag is raised and
// the kernel runs out.  Outputs (d, e, tau, reflectors in H): d, e the tridiagonal, row k of H and
// tau[k] the reflector H_k = I - tau_k v v^T (v_{k+1} = 1).
constexpr int SYTRD_GRID_P = 64;
constexpr int SYTRD_GRID_T = 256;
constexpr int SYTRD_GRID_NMAX = 1024;                          // largest order
constexpr int SYG_M = SYTRD_GRID_NMAX / SYTRD_GRID_T;          // columns per thread
constexpr int SYG_T = SYTRD_GRID_NMAX / 64;                    // columns per lane
constexpr unsigned SYTRD_SPIN_MAX = 1u << 24;

struct SytrdGridBufs {
  double *Rp, *Pv, *Dv;  // published rows (2 x N), p (2 x N), block partial dots (2 x P)
};
__device__ __host__ inline SytrdGridBufs sytrd_grid_bufs(double* work, int N) {
  // inside the divide-and-conquer area, which is free until the reduction ends
  const size_t N2 = next_pow2(N);
  double* z = work + 4 * (size_t)N + (size_t)N * N + N2;
  SytrdGridBufs B;
  B.Rp = z;
  B.Pv = z + 2 * (size_t)N;
  B.Dv = B.Pv + 2 * (size_t)N;
  return B;
}
// Blocks per job: the fewest of 32, 48, 64 whose rows fit LDS (fewer blocks
// make the grid barrier and the partial-dot sum cheaper).
constexpr size_t GRID_DYN_LDS_MAX = 158 * 1024;  // dynamic LDS a grid reduction may ask for
inline size_t sytrd_grid_lds_p(int N, int P) {
  return ((size_t)((N + P - 1) / P) * N + 3 * (size_t)N) * 8;
}
inline int sytrd_grid_blocks(int N) {
  for (int P = 32; P < SYTRD_GRID_P; P += 16)
    if (sytrd_grid_lds_p(N, P) <= GRID_DYN_LDS_MAX) return P;
  return SYTRD_GRID_P;
}
inline size_t sytrd_grid_lds(int N) { return sytrd_grid_lds_p(N, sytrd_grid_blocks(N)); }

// Grid barriers of the multi-block kernels.  A job's work area ends with one
// flag per block and a launch generation.  Each launch takes its barrier
// ordinals from gen * GRID_ORD_SPAN + 1, 2, ..., so they exceed every value
// an earlier launch left in the flags (compared in serial-number arithmetic,
// which survives the 32-bit wrap), and block 0 advances the generation at its
// end.  Every block reads the generation before its first barrier and block 0
// passes that barrier only after all have arrived, so no block can see the
// advanced value.  Nothing needs resetting between launches (the area starts
// zeroed with the rest of the workspace).
constexpr int SYNC_MAXP = 256;                 // blocks one barrier may join
constexpr unsigned GRID_ORD_SPAN = 1u << 16;   // barriers one launch may pass
constexpr size_t SYNC_DOUBLES = SYNC_MAXP / 2 + 8;
struct GridSync {
  unsigned* flag;  // SYNC_MAXP
  unsigned* gen;
};
__device__ inline GridSync grid_sync_of(double* work, int N) {
  GridSync g;
  g.flag = reinterpret_cast<unsigned*>(work + eig_work_main(N));
  g.gen = g.flag + SYNC_MAXP;
  return g;
}
__device__ inline unsigned grid_gen(const GridSync& g) {
  return __hip_atomic_load(g.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// At the end of a launch that passed at least one barrier: block 0 advances
// the generation (gen0 as read at the start).
__device__ inline void grid_launch_end(const GridSync& g, unsigned gen0, bool used) {
  if (used && blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(g.gen, gen0 + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier with ordinal `ordinal` over the P <= SYNC_MAXP blocks of one launch:
// each block stores its ordinal into its own flag (a release store after the
// block barrier, which orders the block's earlier stores before it); one wave
// polls all P flags with coherent loads, then an acquire fence.  No
// read-modify-write, so no serialisation on one address.
__device__ inline void grid_barrier(unsigned* flag, unsigned ordinal, int P, int* s_abort,
                                    int* dims) {
  __syncthreads();
  if (threadIdx.x < 64 && !*s_abort) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(&flag[blockIdx.x], ordinal, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (true) {
      bool ok = true;
      for (int q = lane; q < P; q += 64)
        ok = ok && (int)(__hip_atomic_load(&flag[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                         ordinal) >= 0;
      if (__all(ok)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SYTRD_SPIN_MAX) {
        if (lane == 0) {
          *s_abort = 1;
          atomicOr(&dims[D_FLAG], FLAG_BARRIER);
        }
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

__global__ __launch_bounds__(SYTRD_GRID_T) void k_sytrd_grid(EigJobs jobs, int* __restrict__ dims,
                                                             int N) {
  const int b = blockIdx.x, P = gridDim.x;
  const EigJob J = jobs.j[blockIdx.y];
  const int n = dims[J.n_idx];
  if (n <= SYR_MAX) return;  // k_sytrd_reg (the same decision on all blocks of the job)
  Work W = work_of(J, N);
  const SytrdGridBufs G = sytrd_grid_bufs(J.work, N);
  const double* A = J.A;
  const long long lda = J.lda;
  extern __shared__ double lds[];
  const int RB = (N + P - 1) / P;
  double* Lr = lds;                   // own rows: row i at Lr + (i / P) N
  double* sv = Lr + (size_t)RB * N;   // v_k (and row k of T_k before scaling)
  double* svp = sv + N;               // v_{k-1}
  double* swp = svp + N;              // w_{k-1}
  __shared__ double red[16];
  __shared__ double s_tau, s_scal, s_taup, s_d;
  __shared__ int s_abort;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int li = wave; li * P + b < n; li += 4) {
    const double* ra = A + (long long)(li * P + b) * lda;
    for (int j = lane; j < n; j += 64) Lr[(size_t)li * N + j] = ra[j];
  }
  for (int i = tid; i < N; i += SYTRD_GRID_T) svp[i] = swp[i] = 0.0;
  if (tid == 0) { s_taup = 0.0; s_abort = 0; }
  __syncthreads();
  const GridSync gs = grid_sync_of(J.work, N);
  const unsigned gen0 = grid_gen(gs);
  unsigned ordinal = gen0 * GRID_ORD_SPAN;
  for (int k = 0; k <= n - 2; ++k) {
    // w_{k-1} on indices >= k from the published p_{k-1} and partial dots
    // (every wave sums the P partials the same way), fused with row k of T_k.
    // Every load of the step is issued before the first use: one round trip.
    const int par = (k - 1) & 1;
    const double* pp = G.Pv + (size_t)par * N;
    const double* src = k == 0 ? A : G.Rp + (size_t)par * N;
    const double dpv = (k >= 1 && lane < P) ? G.Dv[(size_t)par * SYTRD_GRID_P + lane] : 0.0;
    const double ppk = k >= 1 ? pp[k] : 0.0;
    double ppv[SYG_M], srv[SYG_M];
#pragma unroll
    for (int m = 0; m < SYG_M; ++m) {
      const int j = k + tid + SYTRD_GRID_T * m;
      ppv[m] = (k >= 1 && j < n) ? pp[j] : 0.0;
      srv[m] = j < n ? src[j] : 0.0;
    }
    const double hc = k >= 1 ? 0.5 * s_taup * wave_sum(dpv) : 0.0;
    const double vk0 = svp[k];
    const double wk0 = k >= 1 ? ppk - hc * vk0 : 0.0;
    if (k == n - 2) {
#pragma unroll
      for (int m = 0; m < SYG_M; ++m) {
        const int j = k + tid + SYTRD_GRID_T * m;
        if (j < n) swp[j] = ppv[m] - hc * svp[j];
      }
      __syncthreads();
    } else {
      // row k of T_k (columns >= k)
      double part = 0.0;
#pragma unroll
      for (int m = 0; m < SYG_M; ++m) {
        const int j = k + tid + SYTRD_GRID_T * m;
        if (j >= n) continue;
        const double wj = k >= 1 ? ppv[m] - hc * svp[j] : 0.0;
        swp[j] = wj;
        const double r = srv[m] - vk0 * wj - wk0 * svp[j];
        if (j == k) s_d = r;
        sv[j] = r;
        if (j >= k + 2) part += r * r;
      }
      const double sumsq = block_sum<SYTRD_GRID_T>(part, red);
      if (tid == 0) {
        const double alpha = sv[k + 1];
        double e;
        if (sumsq == 0.0) {
          s_tau = 0.0;
          s_scal = 0.0;
          e = alpha;
        } else {
          const double beta = -copysign(sqrt(alpha * alpha + sumsq), alpha);
          s_tau = (beta - alpha) / beta;
          s_scal = 1.0 / (alpha - beta);
          e = beta;
        }
        if (b == 0) {
          W.d[k] = s_d;
          W.e[k] = e;
          W.tau[k] = s_tau;
        }
      }
      __syncthreads();
      const double tau = s_tau, scal = s_scal;
      for (int j = k + 1 + tid; j < n; j += SYTRD_GRID_T) {
        const double v = j == k + 1 ? 1.0 : sv[j] * scal;
        sv[j] = v;
        if (b == 0) W.H[(long long)k * N + j] = v;
      }
      __syncthreads();
      // own rows: T_k = T_{k-1} - v w^T - w v^T, and p_k = tau T_k,22 v_k.
      // Lane l handles the columns j = k + 1 + l + 64 t of every row it
      // updates, so it keeps v_{k-1}, w_{k-1} and v_k at those columns in
      // registers: per element only the row entry moves through LDS.
      double* pk = G.Pv + (size_t)(k & 1) * N;
      double* rpub = G.Rp + (size_t)(k & 1) * N;
      const int i0 = k + 1 + ((b - (k + 1)) % P + P) % P;
      const int j0 = k + 1 + lane;
      double cv[SYG_T], cw[SYG_T], cs[SYG_T];
#pragma unroll
      for (int t = 0; t < SYG_T; ++t) {
        const int j = j0 + 64 * t;
        const bool ok = j < n;
        cv[t] = ok ? svp[j] : 0.0;
        cw[t] = ok ? swp[j] : 0.0;
        cs[t] = ok ? sv[j] : 0.0;
      }
      double wpart = 0.0;
      for (int i = i0 + wave * P; i < n; i += 4 * P) {
        const double vi = svp[i], wi = swp[i];
        double* r = Lr + (size_t)(i / P) * N;
        const bool publish = i == k + 1;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < SYG_T; ++t) {
          if (k + 1 + 64 * t >= n) break;
          const int j = j0 + 64 * t;
          if (j < n) {
            const double x = r[j] - vi * cw[t] - wi * cv[t];
            r[j] = x;
            if (publish) rpub[j] = x;
            acc += x * cs[t];
          }
        }
        acc = wave_sum(acc);
        const double pv = tau * acc;
        if (lane == 0) pk[i] = pv;
        wpart += pv * sv[i];
      }
      __syncthreads();
      if (lane == 0) red[wave] = wpart;
      __syncthreads();
      if (tid == 0) {
        G.Dv[(size_t)(k & 1) * SYTRD_GRID_P + b] = ((red[0] + red[1]) + red[2]) + red[3];
        s_taup = tau;
      }
      for (int j = k + 1 + tid; j < n; j += SYTRD_GRID_T) svp[j] = sv[j];
      grid_barrier(gs.flag, ++ordinal, P, &s_abort, dims);
    }
    if (k == n - 2 && tid == 0) {
      // the last 2 x 2 block of T_{n-2}, from its owners' rows of T_{n-3}
      const int i0 = n - 2, i1 = n - 1;
      if (i0 % P == b) {
        const double* r = Lr + (size_t)(i0 / P) * N;
        W.d[i0] = r[i0] - 2.0 * svp[i0] * swp[i0];
        W.e[i0] = r[i1] - svp[i0] * swp[i1] - swp[i0] * svp[i1];
        W.tau[i0] = 0.0;
      }
      if (i1 % P == b) {
        const double* r = Lr + (size_t)(i1 / P) * N;
        W.d[i1] = r[i1] - 2.0 * svp[i1] * swp[i1];
      }
    }
  }
  grid_launch_end(gs, gen0, ordinal != gen0 * GRID_ORD_SPAN);
}

// The same reduction with the matrix in registers (n <= SYR_MAX), one block
// per matrix.  Orders up to SYW_MAX run on one wavefront (sytrd_one_wave);
// larger ones on SYP_WAVES wavefronts with each row split over two lanes:
// lane l of wavefront w holds row r = 32 w + l % 32 and, with h = l / 32,
// the columns of parity h, shifted: before step k, a[c] = A(r, 2 (c + s) + h)
// with s = floor(k / 2), so column k is a[0] on the lanes of parity k % 2 and
// column k + 1 is a[k % 2] on the others; the update of an odd step writes
// A(r, 2 (c + 1 + s) + h) into a[c] (the shift costs nothing), and no
// register is ever picked by a run-time index.  The two halves of a row are
// lanes l and l ^ 32 of one wavefront, and the columns still live at step k
// are spread evenly over both.  A Householder step k, with two block barriers:
//   the lanes of parity k % 2 publish column k in LDS (zero at rows <= k + 1)
//   and each wavefront its share of the column norm; (B1)
//   every wavefront forms tau, beta, scal from the partial norms (summed in
//   a fixed order) and its rows' v_r; the matrix-vector product over the
//   lane's columns p_r = tau (A(r, k+1) + scal sum_{j > k+1} A(r, j) x_j)
//   (x the published column), the two halves combined by a lane exchange;
//   p and each wavefront's share of p.v to LDS; (B2)
//   with K = tau p.v / 2 and u_r = p_r - 2 K v_r, each lane applies
//   A(r, j) -= v_r p_j + u_r v_j = v_r w_j + w_r v_j (w = p - K v) to its
//   columns, v_j = scal x_j from the published column and column k + 1
//   (v = 1 there) separately.
// The published column and p sit at positions relative to s, once at c and
// once at c + 1, so that the unshifted and the shifted update both read
// aligned pairs; the last row of each parity also zeroes the positions past
// its own, which the step two before had filled.  Columns are taken in
// groups of 8 per lane (16 of the matrix); a group wholly past n is skipped
// by a scalar branch.  The published arrays and the partial sums are double
// buffered by the parity of k, so step k + 1 may publish while a slower
// wavefront still reads step k's.  The matrix is the lower triangle of A:
// entries above the diagonal come from coalesced loads of its columns, those
// on and below from rows staged in LDS 64 at a time.
// The loop issues no global memory access: the reflectors and d, e, tau stay
// in LDS (the reflectors where the staged rows were) and are written out
// after it.  A global store in flight holds its data registers until the
// write is acknowledged, so a wavefront that stored inside the loop would
// stall there on its next use of them, on every step.  Barriers inside the
// loop therefore order LDS only (lds_barrier).
constexpr int SYP_C = SYR_MAX / 2;       // columns per lane
constexpr int SYP_PUB = SYP_C + 8;       // positions of each published array
constexpr int SYP_WAVES = SYR_MAX / 32;  // 32 rows per wavefront
constexpr int SYR_T = 64 * SYP_WAVES;
constexpr int SYR_LD = SYR_MAX + 1;      // LDS row stride of the staged rows
// LDS of the staged rows, then of the packed reflectors
constexpr int SYR_BIG = 64 * SYR_LD > SYR_MAX * (SYR_MAX - 1) / 2 ? 64 * SYR_LD : SYR_MAX * (SYR_MAX - 1) / 2;
// offset of v_k (n - 1 - k entries) in the packed reflector store
__device__ inline int refl_off(int k, int n) { return k * (n - 1) - k * (k - 1) / 2; }


// Orders n <= SYW_MAX: the whole reduction on one wavefront, no block
// barrier and no cross-wavefront sum.  Lane i holds row i of the full
// symmetric matrix in registers, shifted so that at step k a[c] = A(i, k + c)
// (zero past n): column k is always a[0].  Each step's update writes the
// updated A(i, k + 1 + c) into a[c], so the shift costs nothing, and no
// register is ever picked by a run-time index (a tree of scalar branches
// costs hundreds of cycles per pick).  Step k: alpha and A(k, k) are read
// from lanes k + 1 and k; the Householder vector costs one wavefront sum;
// v goes to LDS by position relative to k; each lane forms
// p_i = tau sum_c A(i, k + c) v_{k+c} with v read as broadcast pairs;
// K = tau p.v / 2 is the second wavefront sum; w = p - K v goes to LDS; each
// lane applies A(i, j) -= v_i w_j + w_i v_j to its row while shifting it.
// v and w are stored twice, at positions c and c + 1, so that both passes
// read aligned pairs; the lane of row n - 1 also zeroes the position past
// the end, which the previous step had filled.  Columns are taken in groups
// of 8; a group wholly past n is skipped by a scalar branch.  Reflectors and
// d, e, tau go to LDS and are written out after the loop.
constexpr int SYW_MAX = 64;
constexpr int SYW_LD = SYW_MAX + 1;  // LDS row stride of the staged matrix
constexpr int SYW_PUB = SYW_MAX + 8; // entries of each published copy of v, w
static_assert(SYW_MAX * SYW_LD <= SYR_BIG &&
                  SYW_MAX * (SYW_MAX - 1) / 2 + 3 * SYW_PUB <= SYR_BIG,
              "the one-wavefront staging fits the block's LDS array");


__device__ void sytrd_one_wave(const EigJob& J, int n, int N, const Work& W, double* lds,
                               double (*sde)[SYR_MAX]) {
  const int lane = threadIdx.x & 63;
  const double* A = J.A;
  const long long lda = J.lda;
  // the lower triangle, staged through LDS: coalesced row reads, 8 in flight
  for (int i0 = 0; i0 < n; i0 += 8) {
    double t[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i = i0 + r;
      t[r] = (i < n && lane <= i) ? A[(long long)i * lda + lane] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i = i0 + r;
      if (i < n && lane <= i) lds[i * SYW_LD + lane] = t[r];
    }
  }
  wave_sync();
  double a[SYW_MAX];
#pragma unroll
  for (int j = 0; j < SYW_MAX; ++j) {
    double t = 0.0;
    if (lane < n && j < n) t = j <= lane ? lds[lane * SYW_LD + j] : lds[j * SYW_LD + lane];
    a[j] = t;
  }
  wave_sync();  // the staging area becomes the reflectors and v, w
  double* refl = lds;                                // packed reflectors
  double* sva = lds + SYW_MAX * (SYW_MAX - 1) / 2;   // v_{k+c} at c (16-byte aligned)
  double* svb = sva + SYW_PUB;                       // v_{k+c} at c + 1
  double* swb = svb + SYW_PUB;                       // w_{k+c} at c + 1
  for (int e = lane; e < 3 * SYW_PUB; e += 64) sva[e] = 0.0;
  wave_sync();
  for (int k = 0; k + 2 < n; ++k) {
    const int o = k + 1, c = lane - k;  // this lane's row, as a position
    const double x = a[0];              // A(lane, k)
    const double alpha = lane_d(x, o), dkk = lane_d(x, k);
    const double sumsq = wave_sum(lane > o && lane < n ? x * x : 0.0);
    double tau, scal, beta;
    if (sumsq == 0.0) {
      tau = 0.0;
      scal = 0.0;
      beta = alpha;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sumsq), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double v = lane == o ? 1.0 : (lane > o && lane < n ? x * scal : 0.0);
    if (lane >= o && lane < n) refl[refl_off(k, n) + lane - o] = v;
    if (lane == 0) {
      sde[0][k] = dkk;
      sde[1][k] = beta;
      sde[2][k] = tau;
    }
    if (c >= 0 && lane < n) {
      sva[c] = v;
      svb[c + 1] = v;
    }
    if (lane == n - 1) {  // the previous step's last entries, one position on
      sva[c + 1] = 0.0;
      svb[c + 2] = 0.0;
      swb[c + 2] = 0.0;
    }
    wave_sync();
    double pa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < SYW_MAX / 8; ++g) {
      if (8 * g >= n - k) continue;
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        const double2 vj = *reinterpret_cast<const double2*>(sva + 8 * g + t);
        pa[t / 2] = fma(a[8 * g + t], vj.x, pa[t / 2]);
        pa[t / 2] = fma(a[8 * g + t + 1], vj.y, pa[t / 2]);
      }
    }
    const double p = lane > k ? tau * ((pa[0] + pa[1]) + (pa[2] + pa[3])) : 0.0;
    const double K = 0.5 * tau * wave_sum(p * v);
    const double w = p - K * v;
    if (c >= 0 && lane < n) swb[c + 1] = w;
    wave_sync();
    // a[c] <- A(lane, k + 1 + c) - v w_{k+1+c} - w v_{k+1+c}
#pragma unroll
    for (int g = 0; g < SYW_MAX / 8; ++g) {
      if (8 * g >= n - k) continue;
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        const int q = 8 * g + t;
        const double2 vj = *reinterpret_cast<const double2*>(svb + q + 2);
        const double2 wj = *reinterpret_cast<const double2*>(swb + q + 2);
        const double nxt = q + 2 < SYW_MAX ? a[q + 2] : 0.0;
        a[q] = fma(-v, wj.x, fma(-w, vj.x, a[q + 1]));
        a[q + 1] = fma(-v, wj.y, fma(-w, vj.y, nxt));
      }
    }
    wave_sync();  // v, w are rewritten by the next step
  }
  // the last 2 x 2 block, at positions 0 and 1: d[n-2], e[n-2] = A(n-1, n-2), d[n-1]
  const int kl = n >= 2 ? n - 2 : 0;
  const double dn2 = lane_d(a[0], kl), en2 = lane_d(a[0], kl + 1 < n ? kl + 1 : kl);
  const double dn1 = lane_d(n >= 2 ? a[1] : a[0], n - 1);
  if (lane == 0) {
    if (n >= 2) {
      W.d[n - 2] = dn2;
      W.e[n - 2] = en2;
      W.tau[n - 2] = 0.0;
    }
    W.d[n - 1] = dn1;
  }
  for (int k = lane; k + 2 < n; k += 64) {
    W.d[k] = sde[0][k];
    W.e[k] = sde[1][k];
    W.tau[k] = sde[2][k];
  }
  // reflector k: rows k + 1 .. n - 1 of H's row k (one lane per row)
#pragma unroll 8
  for (int k = 0; k + 2 < n; ++k) {
    const int i = k + 1 + lane;
    if (i < n) W.H[(long long)k * N + i] = refl[refl_off(k, n) + lane];
  }
}

__global__ __launch_bounds__(SYR_T) void k_sytrd_reg(EigJobs jobs, int* __restrict__ dims, int N) {
  const EigJob J = jobs.j[blockIdx.x];
  const int n = dims[J.n_idx];
  if (n > SYR_MAX) return;  // k_sytrd_grid
  // staged rows during the load, then the reflectors: v_k (rows k+1 .. n-1)
  // packed from refl_off(k), written to H once after the loop
  __shared__ __align__(16) double big[SYR_BIG];
  double* const stage = big;
  double* const refl = big;
  __shared__ double sde[3][SYR_MAX];  // d, e, tau of the loop's steps
  // published column x and p, [parity of k][parity of the row][position]:
  // A at the row's position, S one further on (read by the shifting update)
  __shared__ __align__(16) double xA[2][2][SYP_PUB], xS[2][2][SYP_PUB];
  __shared__ __align__(16) double pA[2][2][SYP_PUB], pS[2][2][SYP_PUB];
  __shared__ double red[2][SYP_WAVES], red2[2][SYP_WAVES];
  __shared__ double s_ad[2][2];  // A(k+1, k), A(k, k)
  const double* A = J.A;
  const long long lda = J.lda;
  Work W = work_of(J, N);
  const int tid = threadIdx.x, l = tid & 63;
  // the wavefront index is uniform: in a scalar register
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (n <= SYW_MAX) {  // one wavefront; the others leave before any barrier
    if (wave == 0 && n >= 1) sytrd_one_wave(J, n, N, W, big, sde);
    return;
  }
  const int h = l >> 5, r = 32 * wave + (l & 31);
  const bool row = r < n;
  // the last row of this lane's row parity
  const bool lastp = row && (r == n - 1 || r == n - 2);
  for (int e = tid; e < 2 * 2 * SYP_PUB; e += SYR_T) {
    (&xA[0][0][0])[e] = 0.0;
    (&xS[0][0][0])[e] = 0.0;
    (&pA[0][0][0])[e] = 0.0;
    (&pS[0][0][0])[e] = 0.0;
  }
  double a[SYP_C];
  // above the diagonal (j > r): L(j, r), column r of the lower triangle
#pragma unroll
  for (int c = 0; c < SYP_C; ++c) {
    const int j = 2 * c + h;
    a[c] = (row && j < n && j > r) ? A[(long long)j * lda + r] : 0.0;
  }
  // on and below the diagonal (j <= r): L(r, j), rows staged 64 at a time
  for (int r0 = 0; r0 < n; r0 += 64) {
    __syncthreads();
    for (int rr = wave; rr < 64 && r0 + rr < n; rr += SYP_WAVES)
      for (int j = l; j <= r0 + rr; j += 64) stage[rr * SYR_LD + j] = A[(long long)(r0 + rr) * lda + j];
    __syncthreads();
    if (row && r >= r0 && r < r0 + 64) {
      const double* sr = stage + (r - r0) * SYR_LD;
#pragma unroll
      for (int c = 0; c < SYP_C; ++c)
        if (2 * c + h <= r) a[c] = sr[2 * c + h];
    }
  }
  __syncthreads();  // stage is reused for the reflectors
  // step k; SHIFT (k odd) writes the updated A(r, 2 (c + 1 + s) + h) into
  // a[c], so the row moves down one register at no cost.  Steps run in pairs
  // (even, odd) so that the register array has one layout at the loop's back
  // edge.
  auto step = [&](const int k, auto shift_tag) {
    constexpr bool SHIFT = decltype(shift_tag)::value;
    const int o = k + 1, buf = k & 1, hk = k & 1, sh = k >> 1;
    const int pos = (r >> 1) - sh;  // this row's position in the published arrays
    // column k: a[0] on the lanes of parity k % 2
    const double x = a[0];
    const bool own = row && h == hk;
    if (own) {
      const double xv = r > o ? x : 0.0;
      if (pos >= 0) {
        xA[buf][r & 1][pos] = xv;
        xS[buf][r & 1][pos + 1] = xv;
      }
      if (lastp) {  // the step two before wrote one position further on
        xA[buf][r & 1][pos + 1] = 0.0;
        xS[buf][r & 1][pos + 2] = 0.0;
      }
      if (r == o) s_ad[buf][0] = x;
      if (r == k) s_ad[buf][1] = x;
    }
    const double ss = wave_sum(own && r > o ? x * x : 0.0);
    if (l == 0) red[buf][wave] = ss;
    lds_barrier();  // (B1)
    double sumsq = 0.0;
#pragma unroll
    for (int w = 0; w < SYP_WAVES; ++w) sumsq += red[buf][w];
    const double alpha = s_ad[buf][0], dkk = s_ad[buf][1];
    double tau, scal, beta;
    if (sumsq == 0.0) {
      tau = 0.0;
      scal = 0.0;
      beta = alpha;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sumsq), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      sde[0][k] = dkk;
      sde[1][k] = beta;
      sde[2][k] = tau;
    }
    const double xr = row && pos >= 0 ? xA[buf][r & 1][pos] : 0.0;  // A(r, k) below row k + 1
    const double vr = r == o ? 1.0 : xr * scal;
    if (row && h == 0 && r >= o) refl[refl_off(k, n) + r - o] = vr;
    // p over this lane's columns (both halves: one lane exchange)
    double pa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < SYP_C / 8; ++g) {
      if (2 * (8 * g + sh) >= n) continue;
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        const double2 xs = *reinterpret_cast<const double2*>(&xA[buf][h][8 * g + t]);
        pa[t / 2] = fma(a[8 * g + t], xs.x, pa[t / 2]);
        pa[t / 2] = fma(a[8 * g + t + 1], xs.y, pa[t / 2]);
      }
    }
    const bool ocol = h == (o & 1);  // lanes holding column k + 1 (at position k % 2)
    double pp = scal * ((pa[0] + pa[1]) + (pa[2] + pa[3]));
    if (ocol) pp += SHIFT ? a[1] : a[0];  // A(r, k + 1), v = 1 there
    const double pr = row && r > k ? tau * (pp + __shfl_xor(pp, 32)) : 0.0;
    if (row && h == 0 && pos >= 0) {
      pA[buf][r & 1][pos] = pr;
      pS[buf][r & 1][pos + 1] = pr;
    }
    if (lastp && h == 0) {
      pA[buf][r & 1][pos + 1] = 0.0;
      pS[buf][r & 1][pos + 2] = 0.0;
    }
    const double kp = wave_sum(h == 0 ? pr * vr : 0.0);
    if (l == 0) red2[buf][wave] = kp;
    lds_barrier();  // (B2)
    double kd = 0.0;
#pragma unroll
    for (int w = 0; w < SYP_WAVES; ++w) kd += red2[buf][w];
    const double K = 0.5 * tau * kd;
    const double ur = pr - 2.0 * K * vr, us = ur * scal;
#pragma unroll
    for (int g = 0; g < SYP_C / 8; ++g) {
      if (2 * (8 * g + sh) >= n) continue;  // a group wholly past n holds zeros
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        const int q = 8 * g + t;
        if (SHIFT) {  // positions q + 1, q + 2 into q, q + 1
          const double2 xs = *reinterpret_cast<const double2*>(&xS[buf][h][q + 2]);
          const double2 ps = *reinterpret_cast<const double2*>(&pS[buf][h][q + 2]);
          const double nxt = q + 2 < SYP_C ? a[q + 2] : 0.0;
          a[q] = fma(-vr, ps.x, fma(-us, xs.x, a[q + 1]));
          a[q + 1] = fma(-vr, ps.y, fma(-us, xs.y, nxt));
        } else {
          const double2 xs = *reinterpret_cast<const double2*>(&xA[buf][h][q]);
          const double2 ps = *reinterpret_cast<const double2*>(&pA[buf][h][q]);
          a[q] = fma(-vr, ps.x, fma(-us, xs.x, a[q]));
          a[q + 1] = fma(-vr, ps.y, fma(-us, xs.y, a[q + 1]));
        }
      }
    }
    if (ocol) a[0] -= ur;  // column k + 1 (v = 1), now at position 0
  };
  int k0 = 0;
  for (; k0 + 3 < n; k0 += 2) {
    step(k0, std::false_type());
    step(k0 + 1, std::true_type());
  }
  if (k0 + 2 < n) step(k0, std::false_type());
  // the last 2 x 2 block: d[n-2] and e[n-2] = A(n-1, n-2) at position 0 on
  // parity (n - 2) % 2, d[n-1] at position n % 2 on parity (n - 1) % 2
  {
    const double y1 = (n & 1) ? a[1] : a[0];
    if (h == (n & 1)) {
      if (r == n - 2) W.d[n - 2] = a[0];
      if (r == n - 1) W.e[n - 2] = a[0];
    }
    if (h == ((n - 1) & 1) && r == n - 1) W.d[n - 1] = y1;
    if (tid == 0) W.tau[n - 2] = 0.0;
  }
  // the loop's outputs, kept in LDS so that no global store was in flight
  // across its barriers
  __syncthreads();
  for (int k = tid; k + 2 < n; k += SYR_T) {
    W.d[k] = sde[0][k];
    W.e[k] = sde[1][k];
    W.tau[k] = sde[2][k];
  }
  for (int k = wave; k + 2 < n; k += SYP_WAVES) {
    const int off = refl_off(k, n);
    for (int i = k + 1 + l; i < n; i += 64) W.H[(long long)k * N + i] = refl[off + i - k - 1];
  }
}

// ---------------------------------------------------------------------------
// 2. Tridiagonal eigenproblem by divide and conquer (Cuppen), bottom-up from
// 1x1 leaves.  T is torn at every off-diagonal e_m into blocks coupled by
// rank-one terms |e_m| w w^T, w = e_m + sign(e_m) e_{m+1}; each merge of two
// solved halves solves  D + rho z z^T  (z = last row of Q_left, sign-scaled
// first row of Q_right).  Deflation removes tiny z_j and near-equal d_j
// (Givens); the remaining roots come from the secular equation
//   1 + rho sum_j z_j^2 / (d_j - lambda) = 0,
// solved in the shifted variable lambda = d_origin + tau; the eigenvectors
// use the Loewner-recomputed z^ so that they are orthogonal to working
// accuracy.  Vector updates Q <- Q_rot U are tiled products (dc_merge_tile).
struct DC {
  double *lam, *Qa, *Qb, *U, *dsl, *zsl, *rc, *rs, *rtau, *zhat, *dK, *zK, *mrho;
  int *perm, *Kslot, *rp, *rq, *ro, *mk, *mnrot, *mm2;
};
__device__ inline DC dc_of(const Work& W, int N) {
  const int N2 = next_pow2(N);
  DC D;
  double* p = W.Z;  // the D&C area starts where the inverse-iteration area was
  D.lam = p; p += N2;
  D.Qa = p; p += (size_t)N2 * N2;
  D.Qb = p; p += (size_t)N2 * N2;
  D.U = p; p += (size_t)N2 * N2;
  double** dv[] = {&D.dsl, &D.zsl, &D.rc, &D.rs, &D.rtau, &D.zhat, &D.dK, &D.zK, &D.mrho};
  for (double** q : dv) { *q = p; p += N2; }
  int** iv[] = {&D.perm, &D.Kslot, &D.rp, &D.rq, &D.ro, &D.mk, &D.mnrot, &D.mm2};
  for (int** q : iv) { *q = reinterpret_cast<int*>(p); p += N2; }
  return D;
}

// Q = I (both buffers' live blocks) and the torn diagonal, over blocks b of P.
__device__ void dc_init_job(const EigJob& J, const int* __restrict__ dims, int N, int b, int P) {
  const int n = max(0, dims[J.n_idx]);  // -1: an SVD solved by k_svd_jacobi
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int N2 = next_pow2(N);
  // only the live n x n block of Q is ever read
  const long long tot = (long long)n * n;
  for (long long e = b * 256LL + threadIdx.x; e < tot; e += (long long)P * 256) {
    const int i = (int)(e / n), j = (int)(e % n);
    D.Qa[(size_t)i * N2 + j] = i == j ? 1.0 : 0.0;
    D.Qb[(size_t)i * N2 + j] = 0.0;
  }
  for (int i = b * 256 + threadIdx.x; i < N2; i += P * 256) {
    double v = 0.0;
    if (i < n) {
      v = W.d[i];
      if (i > 0) v -= fabs(W.e[i - 1]);
      if (i + 1 < n) v -= fabs(W.e[i]);
    }
    D.lam[i] = v;
  }
}

// Leaves of DC_LEAF rows, solved directly: block b holds rows
// [DC_LEAF b, DC_LEAF (b + 1)) of
// T torn only at its two boundary off-diagonals (its diagonal loses |e| at a
// torn boundary; inside the block T keeps its off-diagonals).  Each block
// is diagonalised in LDS by parallel cyclic Jacobi (round-robin pairs, all
// rotations of a round applied together), its eigenvalues sorted ascending
// with their vectors, and written where the merges up to blocks of 32
// would have left them: lam[block] and the diagonal block of Q.  One
// wavefront per leaf, a lane per entry: with R the round's rotations
// (R[a][a] = R[b][b] = c, R[a][b] = -s, R[b][a] = s on each pair a < b), a
// round forms A' = R A R^T and V' = V R^T entry by entry into a second
// buffer, each entry from the two coefficients of its row's and its
// column's pair, so a round is one pass between two barriers.
constexpr int DC_LEAF = 8;

// A wavefront's LDS for one leaf.
struct LeafLds {
  double A[2][DC_LEAF][DC_LEAF + 1], V[2][DC_LEAF][DC_LEAF + 1];
  double al[DC_LEAF], be[DC_LEAF];  // index i: row i of R is al_i e_i + be_i e_pi(i)
  int pi[DC_LEAF];
  int ord[DC_LEAF];
};


// Leaf `leaf` of job J, by the calling wavefront (lane = threadIdx.x % 64).
__device__ void dc_leaf_wave(const EigJob& J, int* __restrict__ dims, int N, int leaf, LeafLds& L) {
  const int n = max(0, dims[J.n_idx]);
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int N2 = next_pow2(N);
  const int r0 = leaf * DC_LEAF;
  if (r0 >= n) return;
  const int nb = min(DC_LEAF, n - r0);
  const int nbe = nb + (nb & 1);  // even count for the pairing (a decoupled pad)
  auto& A = L.A;
  auto& V = L.V;
  double* s_al = L.al;
  double* s_be = L.be;
  int* s_pi = L.pi;
  int* s_ord = L.ord;
  const int tid = threadIdx.x & 63, ti = tid / DC_LEAF, tj = tid % DC_LEAF;
  double a0 = 0.0;
  if (ti < nb && tj < nb) {
    const int gi = r0 + ti, gj = r0 + tj;
    if (ti == tj) {
      a0 = W.d[gi];
      if (ti == 0 && gi > 0) a0 -= fabs(W.e[gi - 1]);
      if (ti == nb - 1 && gi + 1 < n) a0 -= fabs(W.e[gi]);
    } else if (tj == ti + 1) {
      a0 = W.e[gi];
    } else if (ti == tj + 1) {
      a0 = W.e[gj];
    }
  }
  A[0][ti][tj] = a0;
  V[0][ti][tj] = ti == tj ? 1.0 : 0.0;
  if (tid < DC_LEAF) {
    s_al[tid] = 1.0;
    s_be[tid] = 0.0;
    s_pi[tid] = tid;
  }
  const double tiny = U64 * sqrt(wave_sum(a0 * a0));
  wave_sync();
  const int npair = nbe / 2, m1 = nbe - 1;
  int cur = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    int rot = 0;
    for (int round = 0; round < m1; ++round) {
      // round-robin: position 0 fixed, the others rotate
      if (tid < npair) {
        const int k = tid;
        int xa = k - 1 + round, xb = nbe - 2 - k + round;
        if (xa >= m1) xa -= m1;
        if (xb >= m1) xb -= m1;
        int a = k == 0 ? 0 : 1 + xa, b = 1 + xb;
        if (a > b) { const int t = a; a = b; b = t; }
        double c = 1.0, sn = 0.0;
        if (b < nb) {
          const double apq = A[cur][a][b], app = A[cur][a][a], aqq = A[cur][b][b];
          // tan(theta) = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = a_qq - a_pp,
          // e = 2 a_pq; then c = D / q, s = sign(d) e / q with D = |d| + r,
          // q = sqrt(D^2 + e^2): two square roots and one division, on d and e
          // scaled by a power of two (exact; c and s do not change)
          const double dd = aqq - app, ee = 2.0 * apq;
          const int ex = ilogb(fmax(fabs(dd), fabs(ee)));
          const double ds = ldexp(dd, -ex), es = ldexp(ee, -ex);
          const double r = sqrt(ds * ds + es * es);
          const double Dq = fabs(ds) + r;
          const double inv = 1.0 / sqrt(Dq * Dq + es * es);
          // absolute threshold: the merges above deflate at 8 u ||T|| anyway, and a
          // relative one would chase rounding noise next to near-zero diagonals
          if (apq != 0.0 && fabs(apq) > 0.125 * tiny && fabs(apq) > U64 * sqrt(fabs(app) * fabs(aqq))) {
            c = Dq * inv;
            sn = (dd < 0.0 ? -es : es) * inv;
            rot = 1;
          }
        }
        s_al[a] = c;
        s_be[a] = -sn;
        s_pi[a] = b;
        s_al[b] = c;
        s_be[b] = sn;
        s_pi[b] = a;
      }
      wave_sync();
      {
        const double ai = s_al[ti], bi = s_be[ti], aj = s_al[tj], bj = s_be[tj];
        const int pi = s_pi[ti], pj = s_pi[tj];
        const double x00 = A[cur][ti][tj], x01 = A[cur][ti][pj];
        const double x10 = A[cur][pi][tj], x11 = A[cur][pi][pj];
        A[cur ^ 1][ti][tj] = ai * (aj * x00 + bj * x01) + bi * (aj * x10 + bj * x11);
        V[cur ^ 1][ti][tj] = aj * V[cur][ti][tj] + bj * V[cur][ti][pj];
      }
      cur ^= 1;
      wave_sync();
    }
    if (!__any(rot)) break;
  }
  // ascending order of the eigenvalues (stable: index breaks ties); the
  // identity first, so a NaN (flagged below) cannot leave a slot unset
  if (tid < DC_LEAF) s_ord[tid] = tid < nb ? tid : 0;
  wave_sync();
  if (tid < nb) {
    const double v = A[cur][tid][tid];
    int pos = 0;
    for (int j = 0; j < nb; ++j) {
      const double w = A[cur][j][j];
      pos += (w < v) || (w == v && j < tid);
    }
    s_ord[pos] = tid;
  }
  wave_sync();
  for (int e = tid; e < nb * nb; e += 64) {
    const int i = e / nb, c = e % nb;
    D.Qa[(size_t)(r0 + i) * N2 + r0 + c] = V[cur][i][s_ord[c]];
  }
  if (tid < nb) {
    const double v = A[cur][s_ord[tid]][s_ord[tid]];
    if (!(v == v)) atomicOr(&dims[D_FLAG], FLAG_EIG);
    D.lam[r0 + tid] = v;
  }
}

// Dynamic shared-memory bytes per merge element of the sort and deflation
// (4 doubles, 2 ints) and of the vectors phase (6 doubles and 4 ints with the
// permutation and the rotations staged, up to VEC_STAGE_MAX rows; 4 doubles
// and 1 int above), which also uses 32 KB of fixed arrays (VecLds).
constexpr int PREP_BYTES_PER = 4 * 8 + 2 * 4;
constexpr int VEC_STAGE_MAX = 1024;
constexpr int VEC_BYTES_STAGED = 6 * 8 + 4 * 4;
constexpr int VEC_BYTES_GLOBAL = 4 * 8 + 1 * 4;

// Sort of two ascending halves and deflation of merge m; one 256-thread
// block, the merge's arrays staged in LDS.  The halves are merged in
// parallel (each element's rank in the other half by binary search; ties
// put the left element first); the deflation sweep, which carries the last
// kept entry along, runs on one lane over LDS.  The eigenvector blocks of
// a level live in one of two buffers (par: 0 reads Qa and writes Qb, 1 the
// reverse); a block with no merge at this level is copied across.
__device__ void dc_prep_merge(const EigJob& J, int* __restrict__ dims, int N, int S, int par, int m,
                              double* smem) {
  const int n = dims[J.n_idx];
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int N2 = next_pow2(N);
  const double* Qs = par ? D.Qb : D.Qa;
  double* Qd = par ? D.Qa : D.Qb;
  const int b0 = m * 2 * S;
  if (b0 + S >= n) {
    if (threadIdx.x == 0) D.mk[m] = -1;
    const int nb = max(0, min(2 * S, n - b0));
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
      const size_t o = (size_t)(b0 + e / nb) * N2 + b0 + e % nb;
      Qd[o] = Qs[o];
    }
    return;
  }
  const int nL = S, nR = min(S, n - b0 - S), m2 = nL + nR;
  double* dt = smem;            // original local order
  double* zt = dt + 2 * S;
  double* ds = zt + 2 * S;      // sorted
  double* zs = ds + 2 * S;
  int* perm = reinterpret_cast<int*>(zs + 2 * S);
  int* defl = perm + 2 * S;
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const double beta = W.e[b0 + S - 1];
  const double sgn = beta < 0.0 ? -1.0 : 1.0;
  double part = 0.0, pmax = 0.0;
  for (int c = tid; c < m2; c += 256) {
    const double zq = c < nL ? Qs[(size_t)(b0 + S - 1) * N2 + b0 + c]
                             : sgn * Qs[(size_t)(b0 + S) * N2 + b0 + c];
    const double dv = D.lam[b0 + c];
    zt[c] = zq;
    dt[c] = dv;
    part += zq * zq;
    pmax = fmax(pmax, fabs(dv));
  }
  const double nz2 = block_sum<256>(part, red);
  for (int o = 32; o > 0; o >>= 1) pmax = fmax(pmax, __shfl_xor(pmax, o));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = pmax;
  __syncthreads();
  const double dmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double nz = sqrt(nz2);
  const double rho = fabs(beta) * nz2;
  // parallel merge by ranks
  for (int c = tid; c < m2; c += 256) {
    const double x = dt[c];
    int pos;
    if (c < nL) {  // count right entries strictly below x
      int lo = 0, hi = nR;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dt[nL + mid] < x) lo = mid + 1;
        else hi = mid;
      }
      pos = c + lo;
    } else {       // count left entries at or below x
      int lo = 0, hi = nL;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dt[mid] <= x) lo = mid + 1;
        else hi = mid;
      }
      pos = (c - nL) + lo;
    }
    perm[pos] = c;
    ds[pos] = x;
    zs[pos] = nz > 0.0 ? zt[c] / nz : 0.0;  // rows of orthogonal blocks: nz^2 = 2
  }
  __syncthreads();
  const double tol = 8.0 * U64 * fmax(dmax, rho);
  if (tid == 0) {
    int nrot = 0, p = -1;
    double dp = 0.0, zp = 0.0;  // current values of entry p
    for (int s0 = 0; s0 < m2; s0 += 8) {
      double dd[8], zz[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        dd[t] = s0 + t < m2 ? ds[s0 + t] : 0.0;
        zz[t] = s0 + t < m2 ? zs[s0 + t] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int sI = s0 + t;
        if (sI >= m2) break;
        if (rho * fabs(zz[t]) <= tol) {
          defl[sI] = 1;
          continue;
        }
        defl[sI] = 0;
        double dcur = dd[t], zcur = zz[t];
        if (p >= 0) {
          // |t c s| <= tol with c = z_cur / r, s = z_p / r, r^2 = z_p^2 + z_cur^2,
          // tested without a square root or a division (the z are normalised
          // and above tol / rho, so r^2 neither overflows nor underflows)
          const double tt = dcur - dp;
          const double r2 = zp * zp + zcur * zcur;
          if (fabs(tt * zcur * zp) <= tol * r2) {
            const double r = sqrt(r2);
            const double ir = 1.0 / r;
            const double c = zcur * ir, sn = zp * ir;
            D.rp[b0 + nrot] = p;
            D.rq[b0 + nrot] = sI;
            D.rc[b0 + nrot] = c;
            D.rs[b0 + nrot] = sn;
            ++nrot;
            const double dpn = c * c * dp + sn * sn * dcur;
            const double dqn = sn * sn * dp + c * c * dcur;
            ds[p] = dpn;
            zs[p] = 0.0;
            defl[p] = 1;
            dcur = dqn;
            zcur = r;
            ds[sI] = dcur;
            zs[sI] = zcur;
          }
        }
        p = sI;
        dp = dcur;
        zp = zcur;
      }
    }
    D.mnrot[m] = nrot;
  }
  __syncthreads();
  // K list (non-deflated slots in order) by a block prefix count
  __shared__ int wcnt[4];
  __shared__ int s_nk;
  int base = 0;
  for (int c0 = 0; c0 < m2; c0 += 256) {
    const int c = c0 + tid;
    const int keep = c < m2 && !defl[c];
    const unsigned long long bal = __ballot(keep);
    const int lane = tid & 63, wv = tid >> 6;
    const int before = __popcll(bal & ((1ULL << lane) - 1ULL));
    if (lane == 0) wcnt[wv] = __popcll(bal);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wv; ++w) off += wcnt[w];
    if (keep) {
      const int q = off + before;
      D.dK[b0 + q] = ds[c];
      D.zK[b0 + q] = zs[c];
      D.Kslot[b0 + q] = c;
    }
    base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  for (int c = tid; c < m2; c += 256) {
    D.perm[b0 + c] = perm[c];
    D.dsl[b0 + c] = ds[c];
    D.zsl[b0 + c] = zs[c];
  }
  if (tid == 0) {
    D.mk[m] = base;
    D.mrho[m] = rho;
    D.mm2[m] = m2;
  }
}

// Secular function on LDS-staged d and z^2 (the merge's K entries).
__device__ inline double secular(const double* d, const double* z2, int k, int o, double tau,
                                 double rho, int lane) {
  double s = 0.0;
  const double dor = d[o];
  for (int j = lane; j < k; j += 64) s += z2[j] / ((d[j] - dor) - tau);
  return 1.0 + rho * wave_sum(s);
}

// Roots of the secular equation f(tau) = 1 + rho sum_j z_j^2 / (delta_j - tau)
// (delta_j = d_j - d_o, o the nearer end of the root's interval), one
// wavefront per root, the merge's d and z^2 staged in LDS (roots 4 grp ..
// 4 grp + 3 of merge m on one block).  f is increasing between the poles delta_i < tau < delta_{i+1};
// the root is kept in a bracket [lo, hi] with f(lo) < 0 < f(hi).  Each
// iteration fits the two-pole rational model of Bunch, Nielsen and Sorensen
// (1978): the terms left of the root, psi, and right of it, phi, are each
// replaced by a / (delta - tau) + b matching value and slope at the current
// iterate at their nearest pole; the model's root in the bracket is the
// next iterate (bisection when it falls outside).  When an iteration leaves
// f's sign unchanged and reduces |f| by less than 10x, the next step swaps to
// the fixed-weight model (exact weight on the origin pole, fitted weight on
// the other neighbour), and back, as LAPACK's dlaed4 does between its
// middle-way and fixed-weight steps (Li, 1993).  Stops when |f| is at the
// level of its evaluation error, 8u (1 + rho sum |terms|), or at a relative
// change of 2u.
__device__ void dc_secular_roots(const EigJob& J, int* __restrict__ dims, int N, int S, int m, int grp,
                                 double* smem) {
  const int n = dims[J.n_idx];
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int b0 = m * 2 * S;
  if (b0 + S >= n) return;
  const int nk = D.mk[m];
  if (grp * 4 >= nk) return;
  double* d = smem;
  double* z2 = smem + 2 * S;
  for (int j = threadIdx.x; j < nk; j += 256) {
    d[j] = D.dK[b0 + j];
    const double zj = D.zK[b0 + j];
    z2[j] = zj * zj;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = grp * 4 + wave;
  if (i >= nk) return;
  const double rho = D.mrho[m];
  int o;
  double lo, hi;
  if (i < nk - 1) {
    const double gap = d[i + 1] - d[i];
    const double mid = 0.5 * gap;
    const double g = secular(d, z2, nk, i, mid, rho, lane);
    // Safe brackets from the secular function itself: for the root on the
    // origin's right, g(tau) <= 1 + 2 rho / gap - rho z_o^2 / tau, so
    // tau* >= rho z_o^2 / (1 + 2 rho / gap); symmetrically on the left.
    if (g >= 0.0) {
      o = i;
      hi = mid;
      lo = 0.5 * rho * z2[o] / (1.0 + 2.0 * rho / gap);
    } else {
      o = i + 1;
      lo = -(gap - mid);
      hi = -0.5 * rho * z2[o] / fmax(1.0, 2.0 * rho / gap);
    }
  } else {
    // last root: all other terms are negative, so tau* >= rho z_o^2
    o = nk - 1;
    hi = rho;
    lo = 0.5 * rho * z2[o];
  }
  // an end that underflowed to zero would sit on the origin's pole
  if (lo == 0.0) lo = hi * 0x1p-60;
  if (hi == 0.0) hi = lo * 0x1p-60;
  const double dor = d[o];
  // nearest poles left and right of the root, in the shifted variable
  const double pl = d[i] - dor;
  const bool has_right = i < nk - 1;
  const double pr = has_right ? d[i + 1] - dor : 0.0;
  double tau = 0.0;
  bool done = false;
  {
    // the bracket ends themselves may already be the root to working accuracy
    const double glo = secular(d, z2, nk, o, lo, rho, lane);
    const double ghi = secular(d, z2, nk, o, hi, rho, lane);
    if (glo >= 0.0) { tau = lo; done = true; }
    else if (ghi <= 0.0) { tau = hi; done = true; }
  }
  double x = (lo > 0.0 && hi > 4.0 * lo) ? sqrt(lo) * sqrt(hi)
           : (hi < 0.0 && lo < 4.0 * hi) ? -sqrt(-lo) * sqrt(-hi) : 0.5 * (lo + hi);
  bool fw = false;
  double fprev = 0.0;
  for (int it = 0; it < 100 && !done; ++it) {
    // psi, psi', phi, phi' at x
    double ps = 0.0, dps = 0.0, ph = 0.0, dph = 0.0;
    for (int j = lane; j < nk; j += 64) {
      const double r = 1.0 / ((d[j] - dor) - x);
      const double t = z2[j] * r;
      if (j <= i) { ps += t; dps += t * r; }
      else { ph += t; dph += t * r; }
    }
    ps = wave_sum(ps);
    dps = wave_sum(dps);
    ph = wave_sum(ph);
    dph = wave_sum(dph);
    const double f = 1.0 + rho * (ps + ph);
    // converged once f is at the level of its own rounding error
    if (f == 0.0 || fabs(f) <= 8.0 * U64 * (1.0 + rho * (ph - ps))) { tau = x; break; }
    if (f < 0.0) lo = x;
    else hi = x;
    if (hi - lo <= 4.0 * U64 * fmax(fabs(lo), fabs(hi))) { tau = 0.5 * (lo + hi); break; }
    // when f keeps its sign and falls by less than a factor of 10, the
    // other model takes the next step
    if (it > 0 && f * fprev > 0.0 && fabs(f) > 0.1 * fabs(fprev)) fw = !fw;
    fprev = f;
    // model: a0 + al / (pl - t) + ga / (pr - t) = 0
    double xn;
    if (has_right) {
      double al, ga, a0;
      if (fw) {
        // fixed weight: the origin pole keeps its exact weight rho z_o^2; the
        // other neighbouring pole's weight and the constant match f and f'
        // at x.  It converges where the two-pole fit above does not: a root
        // next to a pole of tiny weight, beside a heavy pole one step away.
        const double fp = rho * (dps + dph);
        const double po = o == i ? pl : pr, pq = o == i ? pr : pl;
        const double wo = rho * z2[o];
        const double wq = (fp - wo / ((po - x) * (po - x))) * (pq - x) * (pq - x);
        a0 = f - wo / (po - x) - wq / (pq - x);
        al = o == i ? wo : wq;
        ga = o == i ? wq : wo;
      } else {
        al = rho * dps * (pl - x) * (pl - x);
        a0 = 1.0 + rho * (ps - dps * (pl - x));
        ga = rho * dph * (pr - x) * (pr - x);
        a0 += rho * (ph - dph * (pr - x));
      }
      // a0 t^2 - b t + c = 0
      const double b = a0 * (pl + pr) + al + ga;
      const double c = a0 * pl * pr + al * pr + ga * pl;
      const double disc = b * b - 4.0 * a0 * c;
      xn = NAN;
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double qq = b >= 0.0 ? b + sq : b - sq;  // no cancellation
        const double r1 = qq != 0.0 ? 2.0 * c / qq : NAN;
        const double r2 = a0 != 0.0 ? qq / (2.0 * a0) : NAN;
        if (r1 > lo && r1 < hi) xn = r1;
        else if (r2 > lo && r2 < hi) xn = r2;
      }
    } else {
      // a0 + al / (pl - t) = 0  ->  t = pl + al / a0 (phi is empty)
      const double al = rho * dps * (pl - x) * (pl - x);
      double a0 = 1.0 + rho * (ps - dps * (pl - x));
      a0 += rho * ph;
      xn = a0 != 0.0 ? pl + al / a0 : NAN;
    }
    if (!(xn > lo && xn < hi)) {
      xn = (lo > 0.0 && hi > 4.0 * lo) ? sqrt(lo) * sqrt(hi)
         : (hi < 0.0 && lo < 4.0 * hi) ? -sqrt(-lo) * sqrt(-hi) : 0.5 * (lo + hi);
      if (!(xn > lo && xn < hi)) { tau = 0.5 * (lo + hi); break; }
    }
    if (fabs(xn - x) <= 2.0 * U64 * fabs(xn)) { tau = xn; break; }
    x = xn;
    tau = x;
  }
  if (lane == 0) {
    if (!(tau == tau) || tau == 0.0) {
      atomicOr(&dims[D_FLAG], FLAG_EIG);
      tau = o == i ? hi : lo;
    }
    D.ro[b0 + i] = o;
    D.rtau[b0 + i] = tau;
  }
}

// Loewner z^, eigenvectors of D + rho z^ z^^T, sorted output, and the
// merge's update matrix W = P G U: U (slot rows, output columns) with the
// deflation's Givens rotations G = G_0 ... G_{r-1} (which act on the slot
// columns of the merge block) applied to its rows, and the slot-to-local
// permutation P applied to its rows, so that the new eigenvector block is
// the old block times W.  A thread owns whole columns of W, so the
// rotations need no barrier.  Everything the per-column loops read (the K
// arrays, the permutation, the rotations) is staged in LDS first, so they
// wait on LDS only; merges of more than VEC_STAGE_MAX rows (the SVD's
// Golub-Kahan order above 1024) read the permutation and the rotations from
// global memory instead, to stay within the CU's LDS.
//
// The rotations are applied without reading W back.  Rotation t acts on
// slots p_t < q_t, the q_t strictly increase with t and p_t >= q_{t-1}
// (the deflation carries its last kept slot along).  Applied last first,
// rotation t therefore meets slot p_t untouched (its U entry), and slot q_t
// untouched or as the output of rotation t + 1 on its p side, carried in a
// register; q_t is final after rotation t, and the carried slot is final
// once the next rotation does not take it.
// Fixed LDS of the vectors phase (one allocation for both of its forms):
// sort keys and tags of up to 2048 outputs, the slot-to-K map.
struct VecLds {
  double sv[2048];
  int st[2048];
  int kix[2048];
  int wcnt[4];
  int bad;
};
__device__ inline VecLds& vec_lds() {
  __shared__ VecLds L;
  return L;
}

template <bool STAGE>
__device__ void dc_vectors_merge(const EigJob& J, int* __restrict__ dims, int N, int S, int m,
                                 double* smem) {
  const int n = dims[J.n_idx];
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int b0 = m * 2 * S;
  const int S2 = 2 * S;
  double* Ub = D.U + (size_t)m * S2 * S2;
  const int tid = threadIdx.x;
  if (b0 + S >= n) return;  // no merge in this block; its GEMM batch is skipped
  const int nk = D.mk[m];
  const int m2 = D.mm2[m];
  const int nrot = D.mnrot[m];
  double* d = smem;
  double* dro = d + S2;
  double* rt = dro + S2;
  double* zh = rt + S2;
  double* rcs_s = zh + S2;        // rotation cosines (staged)
  double* rsn_s = rcs_s + S2;     // rotation sines (staged)
  int* ks = reinterpret_cast<int*>(STAGE ? rsn_s + S2 : zh + S2);  // K index -> slot
  int* pm_s = ks + S2;            // slot -> local row (staged)
  int* rp_s = pm_s + S2;          // rotation t acts on slots rp[t] < rq[t] (staged)
  int* rq_s = rp_s + S2;
  const int* pm = STAGE ? pm_s : D.perm + b0;
  const int* rp = STAGE ? rp_s : D.rp + b0;
  const int* rq = STAGE ? rq_s : D.rq + b0;
  const double* rcs = STAGE ? rcs_s : D.rc + b0;
  const double* rsn = STAGE ? rsn_s : D.rs + b0;
  VecLds& L = vec_lds();
  double* sv = L.sv;
  int* st = L.st;
  int* kix = L.kix;  // slot -> K index + 1, 0 for a deflated slot
  int* wcnt = L.wcnt;
  int& s_bad = L.bad;
  if (tid == 0) s_bad = 0;
  for (long long e = tid; e < (long long)m2 * S2; e += 256) Ub[e] = 0.0;
  for (int c = tid; c < m2; c += 256) {
    if (STAGE) pm_s[c] = D.perm[b0 + c];
    kix[c] = 0;
  }
  for (int j = tid; j < nk; j += 256) {
    d[j] = D.dK[b0 + j];
    rt[j] = D.rtau[b0 + j];
    ks[j] = D.Kslot[b0 + j];
  }
  if (STAGE)
    for (int t = tid; t < nrot; t += 256) {
      rp_s[t] = D.rp[b0 + t];
      rq_s[t] = D.rq[b0 + t];
      rcs_s[t] = D.rc[b0 + t];
      rsn_s[t] = D.rs[b0 + t];
    }
  __syncthreads();
  for (int j = tid; j < nk; j += 256) {
    dro[j] = d[D.ro[b0 + j]];
    kix[ks[j]] = j + 1;
  }
  __syncthreads();
  const double rho = D.mrho[m];
  for (int j = tid; j < nk; j += 256) {
    const double dj = d[j];
    double prod = -((dj - dro[j]) - rt[j]) / rho;
#pragma unroll 4
    for (int i = 0; i < nk; ++i)
      if (i != j) prod *= ((dj - dro[i]) - rt[i]) / (dj - d[i]);
    zh[j] = copysign(sqrt(fmax(prod, 0.0)), D.zK[b0 + j]);
  }
  // sort all outputs: roots (tag i) and deflated slots (tag m2 + slot); the
  // deflated slots enter in slot order, after the roots, by a block prefix
  // count
  int base = 0;
  for (int c0 = 0; c0 < m2; c0 += 256) {
    const int c = c0 + tid;
    const int defl = c < m2 && kix[c] == 0;
    const unsigned long long bal = __ballot(defl);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) wcnt[wv] = __popcll(bal);
    __syncthreads();
    int off = base + __popcll(bal & ((1ULL << lane) - 1ULL));
    for (int w = 0; w < wv; ++w) off += wcnt[w];
    if (defl) {
      const double v = D.dsl[b0 + c];
      if (!(v == v)) s_bad = 1;
      sv[nk + off] = v == v ? v : DBL_MAX;
      st[nk + off] = m2 + c;
    }
    base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  for (int i = tid; i < nk; i += 256) {
    const double v = dro[i] + rt[i];
    if (!(v == v)) s_bad = 1;
    sv[i] = v == v ? v : DBL_MAX;
    st[i] = i;
  }
  const int P2 = next_pow2(m2);
  for (int e = m2 + tid; e < P2; e += 256) {
    sv[e] = DBL_MAX;
    st[e] = 0x7fffffff;
  }
  __syncthreads();
  // bitonic sort by (value, tag)
  for (int k2 = 2; k2 <= P2; k2 <<= 1)
    for (int jj = k2 >> 1; jj > 0; jj >>= 1) {
      for (int e = tid; e < P2; e += 256) {
        const int x = e ^ jj;
        if (x > e) {
          const bool up = (e & k2) == 0;
          const bool gt = sv[e] > sv[x] || (sv[e] == sv[x] && st[e] > st[x]);
          if (gt == up) {
            const double tv = sv[e]; sv[e] = sv[x]; sv[x] = tv;
            const int tt2 = st[e]; st[e] = st[x]; st[x] = tt2;
          }
        }
      }
      __syncthreads();
    }
  if (tid == 0 && s_bad) atomicOr(&dims[D_FLAG], FLAG_EIG);
  for (int pos = tid; pos < m2; pos += 256) {
    D.lam[b0 + pos] = sv[pos];
    const int tag = st[pos];
    double* col = Ub + pos;
    if (tag < 0 || tag >= 2 * m2) {
      atomicOr(&dims[D_FLAG], FLAG_EIG);
      continue;
    }
    const bool root = tag < m2;
    const int dslot = root ? -1 : tag - m2;
    double di = 0.0, ti = 0.0, inv = 0.0;
    if (root) {
      di = dro[tag];
      ti = rt[tag];
      double nrm = 0.0;
#pragma unroll 4
      for (int j = 0; j < nk; ++j) {
        const double u = zh[j] / ((d[j] - di) - ti);
        nrm += u * u;
      }
      if (!(nrm > 0.0) || !(nrm < DBL_MAX)) {
        atomicOr(&dims[D_FLAG], FLAG_EIG);
        continue;
      }
      inv = 1.0 / sqrt(nrm);
#pragma unroll 4
      for (int j = 0; j < nk; ++j) col[(size_t)pm[ks[j]] * S2] = zh[j] / ((d[j] - di) - ti) * inv;
    } else {
      col[(size_t)pm[dslot] * S2] = 1.0;
    }
    // U entry of this column at slot s, before any rotation
    auto u0 = [&](int s) -> double {
      if (!root) return s == dslot ? 1.0 : 0.0;
      const int j = kix[s] - 1;
      return j < 0 ? 0.0 : zh[j] / ((d[j] - di) - ti) * inv;
    };
    int crow = -1;
    double cval = 0.0;
    for (int t = nrot - 1; t >= 0; --t) {
      const int p = rp[t], q = rq[t];
      const double c = rcs[t], sn = rsn[t];
      double xq;
      if (q == crow) {
        xq = cval;
      } else {
        if (crow >= 0) col[(size_t)pm[crow] * S2] = cval;
        xq = u0(q);
      }
      const double xp = u0(p);
      col[(size_t)pm[q] * S2] = c * xq - sn * xp;
      crow = p;
      cval = c * xp + sn * xq;
    }
    if (crow >= 0) col[(size_t)pm[crow] * S2] = cval;
  }
}

// One 64 x 64 tile of a merge product: half h of merge m at level S takes
// rows [b0 + h S, b0 + h S + mh) of the new eigenvector block as the old
// block's h-th diagonal block (mh x mh, one solved half) times rows
// [h S, h S + mh) of the merge's update matrix W (2 S x 2 S, row-major).
__device__ void dc_merge_tile(const EigJob& J, const int* __restrict__ dims, int N, int S, int par,
                              int m, int h, int ti, int tj, double* smem) {
  const int n = dims[J.n_idx];
  const int b0 = m * 2 * S, lim = n - b0;
  if (lim <= S) return;  // no merge in this block
  const int n2 = min(2 * S, lim);
  const int mh = h == 0 ? S : min(S, lim - S);
  const int i0 = ti * 64, j0 = tj * 64;
  if (i0 >= mh || j0 >= n2) return;
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int N2 = next_pow2(N);
  const double* Qs = par ? D.Qb : D.Qa;
  double* Qd = par ? D.Qa : D.Qb;
  const int r0 = b0 + h * S;
  const double* A = Qs + (size_t)r0 * N2 + r0;
  const double* B = D.U + (size_t)m * 4 * S * S + (size_t)h * S * 2 * S;
  double* C = Qd + (size_t)r0 * N2 + b0;
  double(*As)[65] = reinterpret_cast<double(*)[65]>(smem);
  double(*Bs)[65] = reinterpret_cast<double(*)[65]>(smem + GEMM_GK * 65);
  double acc[4][4];
  gemm_tile_acc<0, 0>(acc, A, B, N2, 2 * S, nullptr, i0, j0, mh, n2, mh, As, Bs);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty + 16 * r;
    if (i >= mh) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx + 16 * c;
      if (j < n2) C[(size_t)i * N2 + j] = acc[r][c];
    }
  }
}

// Levels of the divide and conquer at order n (merges of blocks S = 8, 16,
// ... while S < n), and which buffer holds its eigenvectors at the end
// (0: Qa, 1: Qb): the leaves write Qa and each level swaps.
__host__ __device__ inline int dc_par(int n) {
  int L = 0;
  for (int S = DC_LEAF; S < n; S *= 2) ++L;
  return L & 1;
}

// Job q's item t of a phase whose job q has cnt[q] items (t counts across
// the jobs in order).
__device__ inline bool dc_item(const int* cnt, int njobs, int t, int& q, int& r) {
  for (q = 0; q < njobs; ++q) {
    if (t < cnt[q]) {
      r = t;
      return true;
    }
    t -= cnt[q];
  }
  return false;
}

// The whole divide and conquer of up to 4 jobs in one launch of P
// persistent 256-thread blocks: Q = I and the leaves, then per level the
// sort and deflation of every merge, its secular roots (4 per item), its
// vectors and update matrix, and the tiles of its products, each phase
// spread over the blocks and ended by a grid barrier.  A job stops at its
// own live order (dims), so its levels follow n, not the capacity N.  LDS:
// the phases' arrays share the dynamic buffer (dc_fused_dyn_lds(N) bytes).
constexpr int DCF_MAXP = 128;
__global__ __launch_bounds__(256) void k_dc_fused(EigJobs jobs, int njobs, int* __restrict__ dims,
                                                  int N) {
  extern __shared__ double smem[];
  __shared__ LeafLds leaf_lds[4];
  __shared__ int s_abort;
  const int b = blockIdx.x, P = gridDim.x, wave = threadIdx.x >> 6;
  const GridSync gs = grid_sync_of(jobs.j[0].work, N);
  if (threadIdx.x == 0) s_abort = 0;
  const unsigned gen0 = grid_gen(gs);
  unsigned ord = gen0 * GRID_ORD_SPAN;
  int nq[4] = {0, 0, 0, 0}, nmax = 0;
  for (int q = 0; q < njobs; ++q) {
    nq[q] = max(0, dims[jobs.j[q].n_idx]);  // -1: an SVD solved by k_svd_jacobi
    nmax = max(nmax, nq[q]);
  }
  if (nmax == 0) return;  // nothing to solve (every block sees the same sizes)
  for (int q = 0; q < njobs; ++q) dc_init_job(jobs.j[q], dims, N, b, P);
  grid_barrier(gs.flag, ++ord, P, &s_abort, dims);
  int cnt[4] = {0, 0, 0, 0}, tot = 0;
  for (int q = 0; q < njobs; ++q) tot += cnt[q] = (nq[q] + DC_LEAF - 1) / DC_LEAF;
  for (int t = b * 4 + wave; t < tot; t += 4 * P) {
    int q, r;
    if (dc_item(cnt, njobs, t, q, r)) dc_leaf_wave(jobs.j[q], dims, N, r, leaf_lds[wave]);
  }
  for (int S = DC_LEAF, par = 0; S < nmax; S *= 2, par ^= 1) {
    int nm[4] = {0, 0, 0, 0}, tm = 0;
    for (int q = 0; q < njobs; ++q) tm += nm[q] = nq[q] > S ? (nq[q] + 2 * S - 1) / (2 * S) : 0;
    grid_barrier(gs.flag, ++ord, P, &s_abort, dims);
    for (int t = b; t < tm; t += P) {
      int q, r;
      __syncthreads();  // the previous item's LDS reads are done
      if (dc_item(nm, njobs, t, q, r)) dc_prep_merge(jobs.j[q], dims, N, S, par, r, smem);
    }
    grid_barrier(gs.flag, ++ord, P, &s_abort, dims);
    const int X = (2 * S + 3) / 4;  // groups of 4 roots of a merge
    for (int q = 0; q < njobs; ++q) cnt[q] = nm[q] * X;
    for (int t = b; t < tm * X; t += P) {
      int q, r;
      __syncthreads();
      if (dc_item(cnt, njobs, t, q, r)) dc_secular_roots(jobs.j[q], dims, N, S, r / X, r % X, smem);
    }
    grid_barrier(gs.flag, ++ord, P, &s_abort, dims);
    for (int t = b; t < tm; t += P) {
      int q, r;
      __syncthreads();
      if (!dc_item(nm, njobs, t, q, r)) continue;
      if (2 * S <= VEC_STAGE_MAX) dc_vectors_merge<true>(jobs.j[q], dims, N, S, r, smem);
      else dc_vectors_merge<false>(jobs.j[q], dims, N, S, r, smem);
    }
    grid_barrier(gs.flag, ++ord, P, &s_abort, dims);
    const int TI = (S + 63) / 64, TJ = (2 * S + 63) / 64, TM = 2 * TI * TJ;
    for (int q = 0; q < njobs; ++q) cnt[q] = nm[q] * TM;
    for (int t = b; t < tm * TM; t += P) {
      int q, r;
      __syncthreads();
      if (!dc_item(cnt, njobs, t, q, r)) continue;
      const int m = r / TM, e = r % TM, h = e / (TI * TJ), ti = (e / TJ) % TI, tj = e % TJ;
      dc_merge_tile(jobs.j[q], dims, N, S, par, m, h, ti, tj, smem);
    }
  }
  grid_launch_end(gs, gen0, true);
}

// Threshold of the clip rule: eigenvalues above it are kept.
__device__ inline double keep_threshold(const EigJob& J, const double* w, int n) {
  const double lmax = n > 0 ? w[n - 1] : 0.0;
  return fmax(J.clip * (double)n * U64 * lmax, 0.0);
}

// ---------------------------------------------------------------------------
// 3. Back-transformation V[:, n-1-j] = H_0 H_1 ... H_{n-3} q_j for the kept
// eigenvectors q_j of T (columns of the D&C result), a wavefront per vector,
// the vector in registers (lane l holds rows l + 64 c, c < NCH; row chunks
// past n are skipped by a scalar branch).  The reflectors are applied four
// at a time in compact WY form: G = H_k H_{k+1} H_{k+2} H_{k+3} = I - V T V^T
// with V = [v_k .. v_{k+3}] and T upper triangular (T_jj = tau_j,
// T(0:j-1, j) = -tau_j T(0:j-1, 0:j-1) V(:, 0:j-1)^T v_j), so G y = y - V (T
// (V^T y)): four dot products whose wavefront sums run side by side, a 4 x 4
// triangular product, one pass of axpys.  The reflectors are staged through
// LDS in chunks of whole groups (one cooperative load per chunk, every load
// in flight before the first store; rows zero outside each reflector, up to
// n rounded to 64), one wavefront forms each group's T there, and the
// sequential loop over the groups reads only LDS.
constexpr int ORM_G = 4;   // reflectors per compact WY group
constexpr int ORM_CH = 64;
// reflector doubles staged per chunk, and of them per thread: one block per
// CU (a launch has one block per four kept vectors, well under the CU
// count at the orders that matter), so a chunk may take most of the LDS;
// ch * ld stays within it for every capacity up to 1024 (ch >= 4)
constexpr int ORM_LDS_DBL = 18432;
constexpr int ORM_PER = (ORM_LDS_DBL + 255) / 256;
constexpr int ORM_BATCH = 24;  // staged doubles a thread loads before storing them
static_assert(ORM_PER % ORM_BATCH == 0, "whole staging batches");
__host__ __device__ inline int ormtr_ld(int N) { return ((N > 0 ? N : 1) + 63) & ~63; }
__host__ __device__ inline int ormtr_chunk(int N) {
  int c = ORM_LDS_DBL / ormtr_ld(N);
  c = c < ORM_G ? ORM_G : (c > ORM_CH ? ORM_CH : c);
  return c - c % ORM_G;
}
__host__ __device__ inline size_t ormtr_lds_doubles(int N) {
  const int ch = ormtr_chunk(N);
  return (size_t)ch * ormtr_ld(N) + (size_t)(ch / ORM_G) * 16 + ch;
}

// VPW vectors per wavefront (4 VPW per block): every block stages all the
// reflectors, so at large orders (capacity above 640), where the blocks
// outnumber the CUs and the staging traffic (blocks x reflector bytes) bounds
// the launch, each wavefront carries four vectors through the same staged
// chunks; below that one vector a wavefront is faster.
template <int NCH, int VPW>
__global__ __launch_bounds__(256) void k_ormtr(EigJobs jobs, int* __restrict__ dims, int N) {
  const EigJob J = jobs.j[blockIdx.y];
  const int n = dims[J.n_idx];
  const int par = dc_par(n);
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int N2 = next_pow2(N);
  const int ch = ormtr_chunk(N), ld = ormtr_ld(N), gpc = ch / ORM_G;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j0 = blockIdx.x * 4 * VPW;
  if (j0 >= n) return;
  const double thr = keep_threshold(J, D.lam, n);
  // eigenvalues ascend, so the block's last vector is its largest
  if (!(D.lam[min(j0 + 4 * VPW - 1, n - 1)] > thr)) return;
  // vector v of this wavefront: j = j0 + 4 v + wave
  bool active[VPW];
  bool any = false;
#pragma unroll
  for (int v = 0; v < VPW; ++v) {
    const int j = j0 + 4 * v + wave;
    active[v] = j < n && D.lam[j] > thr;
    any = any || active[v];
  }
  extern __shared__ double hs[];  // ch reflectors (rows 0 .. ld - 1), each group's T, the taus
  double* Ts = hs + (size_t)ch * ld;
  double* taus = Ts + (size_t)gpc * 16;
  double y[VPW][NCH];
#pragma unroll
  for (int v = 0; v < VPW; ++v)
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int i = lane + 64 * c, j = j0 + 4 * v + wave;
      y[v][c] = active[v] && i < n ? (par ? D.Qb : D.Qa)[(size_t)i * N2 + j] : 0.0;
    }
  const int nref = n - 2;  // reflectors 0 .. n - 3
  const int ngrp = nref > 0 ? (nref + ORM_G - 1) / ORM_G : 0;
  for (int g1 = ngrp - 1; g1 >= 0; g1 -= gpc) {
    const int g0 = max(0, g1 - gpc + 1), kbase = ORM_G * g0, nr = ORM_G * (g1 - g0 + 1);
    __syncthreads();  // the previous chunk is no longer read
    // flat over (reflector, row), in batches of ORM_BATCH elements a thread:
    // every load of a batch in flight before its first store
    const int tot = nr * ld;
    const double tv = threadIdx.x < nr && kbase + (int)threadIdx.x < nref ? W.tau[kbase + threadIdx.x] : 0.0;
    for (int u0 = 0; u0 < ORM_PER; u0 += ORM_BATCH) {
      if (256 * u0 >= tot) break;
      double t[ORM_BATCH];
#pragma unroll
      for (int u = 0; u < ORM_BATCH; ++u) {
        const int e = threadIdx.x + 256 * (u0 + u), q = e / ld, i = e - q * ld, kk = kbase + q;
        t[u] = (e < tot && kk < nref && i > kk && i < n) ? W.H[(size_t)kk * N + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < ORM_BATCH; ++u) {
        const int e = threadIdx.x + 256 * (u0 + u);
        if (e < tot) hs[e] = t[u];
      }
    }
    if (threadIdx.x < nr) taus[threadIdx.x] = tv;
    __syncthreads();
    for (int gq = wave; gq <= g1 - g0; gq += 4) {
      const double* v = hs + (size_t)(ORM_G * gq) * ld;
      const int kb = kbase + ORM_G * gq;
      double d01 = 0.0, d02 = 0.0, d03 = 0.0, d12 = 0.0, d13 = 0.0, d23 = 0.0;
      for (int i = kb + 1 + lane; i < n; i += 64) {
        const double a0 = v[i], a1 = v[ld + i], a2 = v[2 * ld + i], a3 = v[3 * ld + i];
        d01 = fma(a0, a1, d01);
        d02 = fma(a0, a2, d02);
        d03 = fma(a0, a3, d03);
        d12 = fma(a1, a2, d12);
        d13 = fma(a1, a3, d13);
        d23 = fma(a2, a3, d23);
      }
      d01 = wave_sum(d01);
      d02 = wave_sum(d02);
      d03 = wave_sum(d03);
      d12 = wave_sum(d12);
      d13 = wave_sum(d13);
      d23 = wave_sum(d23);
      const double t0 = taus[ORM_G * gq], t1 = taus[ORM_G * gq + 1];
      const double t2 = taus[ORM_G * gq + 2], t3 = taus[ORM_G * gq + 3];
      const double T01 = -t1 * t0 * d01;
      const double T02 = -t2 * (t0 * d02 + T01 * d12), T12 = -t2 * t1 * d12;
      const double T03 = -t3 * ((t0 * d03 + T01 * d13) + T02 * d23);
      const double T13 = -t3 * (t1 * d13 + T12 * d23), T23 = -t3 * t2 * d23;
      if (lane < 16) {
        const int rr = lane >> 2, cc = lane & 3;
        double tv = 0.0;
        if (rr == cc) tv = rr == 0 ? t0 : rr == 1 ? t1 : rr == 2 ? t2 : t3;
        else if (rr < cc)
          tv = rr == 0 ? (cc == 1 ? T01 : cc == 2 ? T02 : T03) : rr == 1 ? (cc == 2 ? T12 : T13) : T23;
        Ts[gq * 16 + lane] = tv;
      }
    }
    __syncthreads();
    if (!any) continue;
    for (int gq = g1 - g0; gq >= 0; --gq) {
      const double* v = hs + (size_t)(ORM_G * gq) * ld;
      const int kb = kbase + ORM_G * gq;
      // one vector: the group's rows stay in registers for the update; more:
      // they are read from LDS again (registers hold the vectors)
      constexpr bool KEEP = VPW == 1;
      double vv[ORM_G][KEEP ? NCH : 1];
      double sv[VPW][ORM_G];
#pragma unroll
      for (int w = 0; w < VPW; ++w)
#pragma unroll
        for (int q = 0; q < ORM_G; ++q) sv[w][q] = 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int ck = KEEP ? c : 0;
#pragma unroll
        for (int q = 0; q < ORM_G; ++q) vv[q][ck] = 0.0;
        if (64 * c >= n || 64 * c + 63 <= kb) continue;  // no rows of the group here
        const int i = lane + 64 * c;
#pragma unroll
        for (int q = 0; q < ORM_G; ++q) vv[q][ck] = v[(size_t)q * ld + i];
#pragma unroll
        for (int w = 0; w < VPW; ++w)
#pragma unroll
          for (int q = 0; q < ORM_G; ++q) sv[w][q] = fma(vv[q][ck], y[w][c], sv[w][q]);
      }
      const double* T = Ts + gq * 16;
#pragma unroll
      for (int w = 0; w < VPW; ++w) {
        const double s0 = wave_sum(sv[w][0]), s1 = wave_sum(sv[w][1]);
        const double s2 = wave_sum(sv[w][2]), s3 = wave_sum(sv[w][3]);
        const double u0 = ((T[0] * s0 + T[1] * s1) + T[2] * s2) + T[3] * s3;
        const double u1 = (T[5] * s1 + T[6] * s2) + T[7] * s3;
        const double u2 = T[10] * s2 + T[11] * s3;
        const double u3 = T[15] * s3;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if (64 * c >= n || 64 * c + 63 <= kb) continue;
          const int i = lane + 64 * c;
          const double a0 = KEEP ? vv[0][KEEP ? c : 0] : v[i];
          const double a1 = KEEP ? vv[1][KEEP ? c : 0] : v[(size_t)ld + i];
          const double a2 = KEEP ? vv[2][KEEP ? c : 0] : v[2 * (size_t)ld + i];
          const double a3 = KEEP ? vv[3][KEEP ? c : 0] : v[3 * (size_t)ld + i];
          y[w][c] -= ((a0 * u0 + a1 * u1) + a2 * u2) + a3 * u3;
        }
      }
    }
  }
#pragma unroll
  for (int w = 0; w < VPW; ++w) {
    if (!active[w]) continue;
    const int col = n - 1 - (j0 + 4 * w + wave);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int i = lane + 64 * c;
      if (i < n) J.V[(size_t)i * J.ldv + col] = y[w][c];
    }
  }
}

// Sign gauge of columns c < ncol of V (rows < nrow): the largest-magnitude
// entry (first on ties) made positive; a wavefront per column (256-thread
// block, four columns at a time).
__device__ void gauge_columns(double* V, int ldv, int nrow, int ncol) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = wave; c < ncol; c += 4) {
    double best = -1.0, val = 0.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < nrow; i += 64) {
      const double v = V[(size_t)i * ldv + c];
      if (fabs(v) > best) { best = fabs(v); val = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double b2 = __shfl_xor(best, o), v2 = __shfl_xor(val, o);
      const int i2 = __shfl_xor(bi, o);
      if (b2 > best || (b2 == best && i2 < bi)) { best = b2; val = v2; bi = i2; }
    }
    if (val < 0.0)
      for (int i = lane; i < nrow; i += 64) V[(size_t)i * ldv + c] = -V[(size_t)i * ldv + c];
  }
}

// ---------------------------------------------------------------------------
// 4. Descending eigenvalues, kept count, sqrt scalings and sign gauge.  Each
// block takes 16 columns of the gauge (and recounts the kept eigenvalues from
// an LDS copy of them); block 0 also writes the count and the scalings.
constexpr int FINAL_COLS = 4;  // one column per wavefront: the gauge is latency-bound
__global__ __launch_bounds__(256) void k_eig_final(EigJobs jobs, int* __restrict__ dims, int N) {
  const EigJob J = jobs.j[blockIdx.y];
  const int n = dims[J.n_idx];
  const int c0 = blockIdx.x * FINAL_COLS;
  if (c0 >= n && blockIdx.x > 0) return;  // block 0 always writes the count
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  __shared__ int s_low, s_bad;
  __shared__ double sl[1024];
  const int tid = threadIdx.x;
  const double thr = keep_threshold(J, D.lam, n);
  if (tid == 0) {
    s_low = -1;
    s_bad = 0;
  }
  for (int c = tid; c < n; c += 256) sl[c] = D.lam[c];
  __syncthreads();
  // ascending eigenvalues: the kept ones are those above the highest index
  // whose value is not above the threshold (a NaN counts as not above)
  int low = -1, bad = 0;
  for (int j = tid; j < n; j += 256) {
    if (!(sl[j] == sl[j])) bad = 1;
    if (!(sl[j] > thr)) low = j;
  }
  if (low >= 0) atomicMax(&s_low, low);
  if (bad) s_bad = 1;
  __syncthreads();
  const int kept = n - 1 - s_low;
  if (tid == 0 && blockIdx.x == 0) {
    dims[J.kept_idx] = kept;
    if (s_bad) atomicOr(&dims[D_FLAG], FLAG_EIG);
  }
  if (blockIdx.x == 0) {
    for (int c = tid; c < n; c += 256) {
      const double l = sl[n - 1 - c];
      J.lam[c] = l;
      if (c < kept) {
        const double s = sqrt(l);
        J.sq[c] = s;
        J.isq[c] = 1.0 / s;
      }
    }
  }
  const int c1 = min(c0 + FINAL_COLS, kept);
  if (c0 < c1) gauge_columns(J.V + c0, J.ldv, n, c1 - c0);
}

// ---------------------------------------------------------------------------
// 5. Small SVD through the Golub-Kahan tridiagonal.  With M = Q_L B Q_R^T
// (B upper bidiagonal, diagonal d_i, superdiagonal e_i), the symmetric
// tridiagonal of order 2q with zero diagonal and off-diagonal
// (d_0, e_0, d_1, e_1, ..., d_{q-1}) has eigenvalues +-sigma_j, and the
// eigenvector of +sigma_j interleaves (v_j, u_j) / sqrt 2.  Its eigenpairs
// come from the divide and conquer above, so sigma_j is accurate to
// ~u sigma_1 absolutely and the vectors to ~u sigma_1 / gap.

constexpr int GEBRD_LDS_MAX = 16384;  // p q doubles held in LDS by k_gebrd_lds
// Longer side from which k_gebrd_grid takes a matrix that does not fit
// k_gebrd_lds.  With p >= q, a p x q matrix with p < 128 always fits
// (p (q | 1) <= 127^2 < GEBRD_LDS_MAX), so every other one goes to the grid.
constexpr int GEBRD_GRID_MIN = 128;
constexpr int GEBRD_GRID_PMAX = 128;  // blocks of k_gebrd_grid at most
static_assert(GEBRD_GRID_PMAX <= 128, "eig_work_main sizes the grid partials for 128 blocks");
constexpr int GBG_M = 4;   // columns per thread in k_gebrd_grid's partial sums (q <= 1024)
constexpr int GBG_U = 16;  // block partials loaded together
__device__ inline int gebrd_ld(int q) { return q | 1; }
__device__ inline bool gebrd_fits(int p, int q) {
  return (long long)p * gebrd_ld(q) <= GEBRD_LDS_MAX && p <= 1024;
}

// The taller orientation of M into the work matrix (side 0: M^T, b x a);
// only for matrices too large for k_gebrd_lds.
__global__ __launch_bounds__(256) void k_svd_load(const double* __restrict__ M, int ldm,
                                                  EigJobs jobs, int* __restrict__ dims,
                                                  int a_idx, int b_idx, int side_idx) {
  const EigJob J = jobs.j[0];
  const int a = dims[a_idx], b = dims[b_idx], side = dims[side_idx];
  const int p = side ? a : b, q = side ? b : a;
  if (blockIdx.x == 0 && threadIdx.x == 0) dims[J.n_idx] = 2 * q;
  if (gebrd_fits(p, q)) return;  // k_gebrd_lds loads M itself
  const long long tot = (long long)p * q;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / q), j = (int)(e % q);
    J.A[(long long)i * J.lda + j] = side ? M[(long long)i * ldm + j] : M[(long long)j * ldm + i];
  }
}

// Small SVDs by one-sided Jacobi (Hestenes), in one 512-thread block: when
// the short side q <= JAC_QMAX and the p x q work matrix B (B = M for side 1,
// M^T for side 0; p >= q) fits LDS, its columns are orthogonalised by plane
// rotations, B V = U S, and the right vectors V (the vectors of M's short
// side) and S come out directly, with no bidiagonalisation and no
// tridiagonal eigensolve.  The q columns are paired round-robin (q - 1
// rounds of q / 2 disjoint pairs per sweep); each pair belongs to one row of
// 16 lanes, whose sums need only the four in-row DPP steps, so the up to 32
// pairs of a round run side by side on at most eight wavefronts, and a
// wavefront whose rows all lack a pair skips the round.  (The step is bound
// by instruction issue: every wave64 VALU instruction holds its SIMD for four
// cycles, so the work per round is kept on as few wavefronts as the pairs
// need.)  A pair (i, j) with a = |b_i|^2, b = |b_j|^2, g = b_i . b_j is
// rotated when g^2 > (p u)^2 a b, by the angle that zeroes g: with d = b - a,
// t = sign(d) 2 g / (|d| + sqrt(d^2 + 4 g^2)) (the smaller root of
// t^2 + (d / g) t - 1 = 0), c = 1 / sqrt(1 + t^2), s = c t.  A sweep without
// a rotation ends the iteration (at most JAC_MAXSW sweeps; more raises the
// eigensolver flag).  Singular values are the final column norms, sorted
// descending (index breaks ties); the kept count, the scalings and the sign
// gauge follow the same rules as the Golub-Kahan path, whose launches then
// return at once: the Golub-Kahan order dims[J.n_idx] is set to -1 to say so.
constexpr int JAC_QMAX = 64;
constexpr int JAC_PQ = 12288;   // doubles of B in LDS (96 KB: q columns of p rows padded to 16), plus V
constexpr int JAC_PMAX = 512;
constexpr int JAC_MAXSW = 40;
constexpr int JAC_T = 512;
constexpr int JAC_WAVES = JAC_T / 64;
__device__ inline int jacobi_ld(int p) { return (p + 15) & ~15; }
__device__ inline bool jacobi_fits(int p, int q) {
  return q >= 1 && q <= JAC_QMAX && p <= JAC_PMAX && jacobi_ld(p) * q <= JAC_PQ;
}

// Sum over each row of 16 lanes, returned on every lane of the row (the
// first four steps of wave_sum).
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

__global__ __launch_bounds__(JAC_T) void k_svd_jacobi(const double* __restrict__ M, int ldm,
                                                      EigJobs jobs, int* __restrict__ dims,
                                                      int a_idx, int b_idx, int side_idx) {
  const EigJob J = jobs.j[0];
  const int a = dims[a_idx], b = dims[b_idx], side = dims[side_idx];
  const int p = side ? a : b, q = side ? b : a;
  if (!jacobi_fits(p, q)) return;  // the Golub-Kahan path
  __shared__ double Bs[JAC_PQ];
  __shared__ double Vs[JAC_QMAX * JAC_QMAX];
  __shared__ double ssig[JAC_QMAX];
  __shared__ int spos[JAC_QMAX];
  __shared__ int s_rot[2];
  __shared__ int s_kept;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rl = lane & 15;              // lane within the row of 16
  const int k = 4 * wave + (lane >> 4);  // the pair of this row
  // B column-major (column j at Bs + j ld, rows p .. ld - 1 zero), V = I
  const int ld = jacobi_ld(p);
  for (int e = tid; e < ld * q; e += JAC_T) {
    const int i = e % ld, j = e / ld;
    Bs[e] = i >= p ? 0.0 : side ? M[(long long)i * ldm + j] : M[(long long)j * ldm + i];
  }
  for (int e = tid; e < q * q; e += JAC_T) Vs[e] = (e % q) == (e / q) ? 1.0 : 0.0;
  if (tid < 2) s_rot[tid] = 0;
  __syncthreads();
  const int qe = q + (q & 1), npair = qe / 2, m1 = qe - 1;
  const int nch = ld / 16;
  const double tol2 = ((double)p * U64) * ((double)p * U64);
  // sweeps allowed: JAC_MAXSW, or fewer when the host caps them (a test of
  // the failure path: the rotations stay finite, only convergence is lost)
  const int capsw = dims[D_JAC_MAXSW];
  const int maxsw = capsw > 0 && capsw < JAC_MAXSW ? capsw : JAC_MAXSW;
  int sw = 0;
  for (; sw < maxsw; ++sw) {
    const int flag = sw & 1;
    for (int rnd = 0; rnd < m1; ++rnd) {
      if (4 * wave < npair) {
        // round-robin: position 0 fixed, the others rotate
        int xa = k - 1 + rnd, xb = qe - 2 - k + rnd;
        if (xa >= m1) xa -= m1;
        if (xb >= m1) xb -= m1;
        int ci = k == 0 ? 0 : 1 + xa, cj = 1 + xb;
        if (ci > cj) { const int t = ci; ci = cj; cj = t; }
        // a row without a pair this round (k >= npair, or the padding
        // column of an odd q) reads column 0 and never rotates; every load is
        // in bounds and unconditional (the columns are zero-padded to ld)
        const bool live = k < npair && cj < q;
        double* bi = Bs + (size_t)(live ? ci : 0) * ld;
        double* bj = Bs + (size_t)(live ? cj : 0) * ld;
        double pa = 0.0, pb = 0.0, pg = 0.0;
#pragma unroll 8
        for (int c = 0; c < nch; ++c) {
          const double xv = bi[rl + 16 * c], yv = bj[rl + 16 * c];
          pa = fma(xv, xv, pa);
          pb = fma(yv, yv, pb);
          pg = fma(xv, yv, pg);
        }
        const double aa = row16_sum(pa), bb = row16_sum(pb), g = row16_sum(pg);
        if (live && g != 0.0 && g * g > tol2 * aa * bb) {
          const double d = bb - aa, g2 = 2.0 * g;
          const double t = (d >= 0.0 ? g2 : -g2) / (fabs(d) + sqrt(d * d + g2 * g2));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          // the columns are read again from LDS: holding them in registers
          // costs more instructions than the reads (and spills at p = 512)
#pragma unroll 8
          for (int c = 0; c < nch; ++c) {
            const int i = rl + 16 * c;
            const double xv = bi[i], yv = bj[i];
            bi[i] = cs * xv - sn * yv;  // padding rows stay zero
            bj[i] = sn * xv + cs * yv;
          }
          double* vi = Vs + (size_t)ci * q;
          double* vj = Vs + (size_t)cj * q;
          for (int r = rl; r < q; r += 16) {
            const double u = vi[r], w = vj[r];
            vi[r] = cs * u - sn * w;
            vj[r] = sn * u + cs * w;
          }
          if (rl == 0) s_rot[flag] = 1;
        }
      }
      __syncthreads();
    }
    const int any = s_rot[flag];
    if (tid == 0) s_rot[flag ^ 1] = 0;  // the next sweep's flag
    __syncthreads();
    if (!any) break;
  }
  if (sw == maxsw && tid == 0) atomicOr(&dims[D_FLAG], FLAG_NOCONV);
  // singular values: column norms; descending order (index breaks ties)
  for (int j = wave; j < q; j += JAC_WAVES) {
    double part = 0.0;
    for (int i = lane; i < p; i += 64) part = fma(Bs[(size_t)j * ld + i], Bs[(size_t)j * ld + i], part);
    const double s2 = wave_sum(part);
    if (lane == 0) ssig[j] = sqrt(s2);
  }
  __syncthreads();
  if (tid < q) {
    const double v = ssig[tid];
    if (!(v == v)) atomicOr(&dims[D_FLAG], FLAG_EIG);
    int pos = 0;
    for (int kk = 0; kk < q; ++kk) {
      const double w = ssig[kk];
      pos += (w > v) || (w == v && kk < tid);
    }
    spos[tid] = pos;
  }
  __syncthreads();
  for (int j = tid; j < q; j += JAC_T) J.lam[spos[j]] = ssig[j];
  for (int e = tid; e < q * q; e += JAC_T) {
    const int i = e % q, j = e / q;
    J.V[(size_t)i * J.ldv + spos[j]] = Vs[e];
  }
  if (tid == 0) {
    // the Golub-Kahan path's clip rule at its order 2q: sigma > clip 2q u sigma_1
    double smax = 0.0;
    for (int j = 0; j < q; ++j) smax = fmax(smax, ssig[j]);
    const double thr = fmax(J.clip * (double)(2 * q) * U64 * smax, 0.0);
    int kk = 0;
    for (int j = 0; j < q; ++j) kk += ssig[j] > thr;
    s_kept = kk;
    dims[J.kept_idx] = kk;
    dims[J.n_idx] = -1;
  }
  __syncthreads();  // J.V and J.lam written by this block
  const int kept = s_kept;
  for (int c = tid; c < kept; c += JAC_T) {
    const double sg = J.lam[c];
    J.sq[c] = sg;
    J.isq[c] = 1.0 / sg;
  }
  if (tid < 256) gauge_columns(J.V, J.ldv, q, kept);
}

// Householder bidiagonalisation of the p x q work matrix (p >= q): left
// reflectors zero column k below the diagonal (d_k), right reflectors zero
// row k right of the superdiagonal (e_k).  Only the right reflectors are kept
// (W.H rows, W.tau): the vectors of the short side are Q_R times the v-part
// of the tridiagonal's eigenvectors.  Two kernels: k_gebrd_lds when the
// matrix fits one block's LDS, else k_gebrd_grid.
//
// k_gebrd_grid: P blocks, each holding the rows i = b (mod P) in LDS (row
// stride q), with one grid barrier per step.  The left reflector of column k is
// u = e_k + s_L c, c = A(k+1:, k), and its product with the trailing matrix is
// y = tau_L (A(k, k+1:) + s_L sum_{i > k} A(i, k) A(i, k+1:)): each block can
// form its share of that sum, and of |c|^2, from its own rows before the
// reflector exists.  So before the barrier that opens step k every block
// publishes those two partials over its own rows i > k, and the owner of row
// k publishes the row; step k then runs without another barrier:
//   every block sums the P partials in block order, forms the left reflector
//   (alpha = A(k, k)), y, row k after it, and from that row the right
//   reflector v_k, tau_R, e_k, redundantly; it applies both reflectors to its
//   own rows in LDS (A_i -= s_L A(i, k) y, then A_i -= tau_R (A_i . v) v) and
//   publishes the partials of step k + 1 (double-buffered by step parity: a
//   block may write step k + 1's while another still reads step k's).
// Outputs: W.e[2k] = d_k, W.e[2k+1] = e_k, W.tau, right reflectors in W.H.
// Launch and barrier as k_sytrd_grid.

struct GebrdGridBufs {
  double *R, *Y, *S;  // published rows (2 x N), partial sums (2 x P x N), |c|^2 partials (2 x P)
};
__device__ __host__ inline GebrdGridBufs gebrd_grid_bufs(double* work, int N) {
  const size_t N2 = next_pow2(N);
  double* z = work + 4 * (size_t)N + (size_t)N * N + N2;
  GebrdGridBufs B;
  B.R = z;
  B.Y = z + 2 * (size_t)N;
  B.S = B.Y + 2 * (size_t)GEBRD_GRID_PMAX * N;
  return B;
}
// blocks and dynamic LDS for rows up to pcap and columns up to qcap: the
// fewest blocks (16, 32, 64, 128) whose rows fit LDS, since the barrier and
// the partial sums cost more with more blocks
inline size_t gebrd_grid_lds_p(int pcap, int qcap, int P) {
  return ((size_t)((pcap + P - 1) / P) * qcap + (size_t)pcap + 3 * (size_t)qcap) * 8;
}
inline int gebrd_grid_blocks(int pcap, int qcap) {
  for (int P = 16; P < GEBRD_GRID_PMAX; P *= 2)
    if (gebrd_grid_lds_p(pcap, qcap, P) <= GRID_DYN_LDS_MAX) return P;
  return GEBRD_GRID_PMAX;
}
inline size_t gebrd_grid_lds(int pcap, int qcap) {
  return gebrd_grid_lds_p(pcap, qcap, gebrd_grid_blocks(pcap, qcap));
}

// The launch is sized for the capacities (pcap, qcap); the live p x q matrix
// runs on the fewest of 16, 32, ... launched blocks whose rows of stride q,
// with y and v after them, fit the lds_doubles the launch provides, and the
// other blocks return at once.
__device__ inline int gebrd_grid_live_blocks(int p, int q, int qcap, int launched,
                                             int lds_doubles) {
  for (int P = 16; P < launched; P *= 2)
    if ((long long)((p + P - 1) / P) * q + 2LL * qcap <= lds_doubles) return P;
  return launched;
}

__global__ __launch_bounds__(256) void k_gebrd_grid(EigJobs jobs, int* __restrict__ dims, int N,
                                                    int a_idx, int b_idx, int side_idx, int qcap,
                                                    int lds_doubles) {
  const EigJob J = jobs.j[0];
  if (dims[J.n_idx] < 0) return;  // solved by k_svd_jacobi
  const int a = dims[a_idx], bb = dims[b_idx], side = dims[side_idx];
  const int p = side ? a : bb, q = side ? bb : a;
  if (gebrd_fits(p, q) || p < GEBRD_GRID_MIN) return;  // k_gebrd_lds
  const int P = gebrd_grid_live_blocks(p, q, qcap, gridDim.x, lds_doubles);
  const int b = blockIdx.x;
  if (b >= P) return;
  const double* A = J.A;
  const long long lda = J.lda;
  Work W = work_of(J, N);
  const GebrdGridBufs G = gebrd_grid_bufs(J.work, N);
  extern __shared__ double lds[];
  const int RB = (p + P - 1) / P;
  double* Lr = lds;                 // own rows: row i at Lr + (i / P) q
  double* sy = Lr + (size_t)RB * q; // y (q)
  double* sv = sy + qcap;           // row k, then v_k (q)
  __shared__ double red[16];
  __shared__ double s_tr, s_sr;
  __shared__ int s_abort;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int li = wave; li * P + b < p; li += 4) {
    const double* ra = A + (long long)(li * P + b) * lda;
    for (int j = lane; j < q; j += 64) Lr[(size_t)li * q + j] = ra[j];
  }
  if (b == 0)
    for (int i = tid; i < 2 * q; i += 256) W.d[i] = 0.0;
  if (tid == 0) s_abort = 0;
  __syncthreads();
  // partials of step k over the own rows i > k (rows already in LDS), and
  // row k from its owner
  auto publish = [&](int k) {
    const int par = k & 1;
    double* yp = G.Y + ((size_t)par * GEBRD_GRID_PMAX + b) * N;
    const int ifirst = k + 1 + ((b - (k + 1)) % P + P) % P;
    for (int j = tid; j < q - k - 1; j += 256) {
      double acc = 0.0;
      for (int i = ifirst; i < p; i += P) {
        const double* r = Lr + (size_t)(i / P) * q;
        acc += r[k] * r[k + 1 + j];
      }
      yp[j] = acc;
    }
    if (wave == 0) {
      double part = 0.0;
      for (int i = ifirst + lane * P; i < p; i += 64 * P) {
        const double c = Lr[(size_t)(i / P) * q + k];
        part += c * c;
      }
      part = wave_sum(part);
      if (lane == 0) G.S[(size_t)par * GEBRD_GRID_PMAX + b] = part;
    }
    if (k % P == b) {
      const double* r = Lr + (size_t)(k / P) * q;
      double* rpub = G.R + (size_t)par * N;
      for (int j = k + tid; j < q; j += 256) rpub[j] = r[j];
    }
  };
  const GridSync gs = grid_sync_of(J.work, N);
  const unsigned gen0 = grid_gen(gs);
  unsigned ordinal = gen0 * GRID_ORD_SPAN;
  publish(0);
  grid_barrier(gs.flag, ++ordinal, P, &s_abort, dims);
  for (int k = 0; k < q; ++k) {
    const int nc = q - k - 1, par = k & 1;
    const double* rk = G.R + (size_t)par * N;
    const double* S = G.S + (size_t)par * GEBRD_GRID_PMAX;
    // left reflector of column k (every thread forms the same scalars)
    const double sumsq =
        wave_sum((lane < P ? S[lane] : 0.0) + (lane + 64 < P ? S[lane + 64] : 0.0));
    const double alpha = rk[k];
    double tl, sl, bl;
    if (sumsq == 0.0) {
      tl = 0.0;
      sl = 0.0;
      bl = alpha;
    } else {
      bl = -copysign(sqrt(alpha * alpha + sumsq), alpha);
      tl = (bl - alpha) / bl;
      sl = 1.0 / (alpha - bl);
    }
    if (b == 0 && tid == 0) {
      W.e[2 * k] = bl;
      if (nc <= 0) W.tau[k] = 0.0;
    }
    if (nc <= 0) break;  // the last column: no right reflector
    // y, and row k after the left reflector
    // (the P partials of a column are summed in block order; the loads of up
    // to GBG_M columns times GBG_U blocks are issued together)
    const double* Yp = G.Y + (size_t)par * GEBRD_GRID_PMAX * N;
    double acc[GBG_M];
#pragma unroll
    for (int m = 0; m < GBG_M; ++m) acc[m] = 0.0;
    for (int q0 = 0; q0 < P; q0 += GBG_U) {
      double v[GBG_M][GBG_U];
#pragma unroll
      for (int m = 0; m < GBG_M; ++m) {
        const int j = tid + 256 * m;
#pragma unroll
        for (int u = 0; u < GBG_U; ++u)
          v[m][u] = (j < nc && q0 + u < P) ? Yp[(size_t)(q0 + u) * N + j] : 0.0;
      }
#pragma unroll
      for (int m = 0; m < GBG_M; ++m)
#pragma unroll
        for (int u = 0; u < GBG_U; ++u) acc[m] += v[m][u];
    }
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < GBG_M; ++m) {
      const int j = tid + 256 * m;
      if (j >= nc) continue;
      const double rkj = rk[k + 1 + j];
      const double y = tl * (rkj + sl * acc[m]);
      sy[j] = y;
      const double r = rkj - y;
      sv[j] = r;
      if (j > 0) part += r * r;
    }
    const double sumr = block_sum<256>(part, red);
    if (tid == 0) {
      const double alpha_r = sv[0];
      double beta;
      if (sumr == 0.0) {
        s_tr = 0.0;
        s_sr = 0.0;
        beta = alpha_r;
      } else {
        beta = -copysign(sqrt(alpha_r * alpha_r + sumr), alpha_r);
        s_tr = (beta - alpha_r) / beta;
        s_sr = 1.0 / (alpha_r - beta);
      }
      if (b == 0) {
        W.e[2 * k + 1] = beta;
        W.tau[k] = s_tr;
      }
    }
    __syncthreads();
    const double tr = s_tr, sr = s_sr;
    for (int j = tid; j < nc; j += 256) {
      const double v = j == 0 ? 1.0 : sv[j] * sr;
      sv[j] = v;
      if (b == 0) W.H[(long long)k * N + k + 1 + j] = v;
    }
    __syncthreads();
    // own rows: lane l handles the columns k + 1 + l + 64 t of every row, so y
    // and v at those columns stay in registers, and so does the row between
    // the two reflectors: one LDS read and one write per element
    const int i0 = k + 1 + ((b - (k + 1)) % P + P) % P;
    double cy[SYG_T], cv[SYG_T];
#pragma unroll
    for (int t = 0; t < SYG_T; ++t) {
      const int j = lane + 64 * t;
      cy[t] = j < nc ? sy[j] : 0.0;
      cv[t] = j < nc ? sv[j] : 0.0;
    }
    for (int i = i0 + wave * P; i < p; i += 4 * P) {
      double* rowp = Lr + (size_t)(i / P) * q;
      double* r = rowp + k + 1;
      const double ui = sl * rowp[k];
      double x[SYG_T];
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < SYG_T; ++t) {
        if (64 * t >= nc) break;
        const int j = lane + 64 * t;
        x[t] = j < nc ? r[j] - ui * cy[t] : 0.0;
        acc += x[t] * cv[t];
      }
      const double z = tr * wave_sum(acc);
#pragma unroll
      for (int t = 0; t < SYG_T; ++t) {
        if (64 * t >= nc) break;
        const int j = lane + 64 * t;
        if (j < nc) r[j] = x[t] - z * cv[t];
      }
    }
    __syncthreads();
    publish(k + 1);
    grid_barrier(gs.flag, ++ordinal, P, &s_abort, dims);
  }
  grid_launch_end(gs, gen0, ordinal != gen0 * GRID_ORD_SPAN);
}

// k_gebrd_lds: the p x q matrix in LDS (p ldq <= GEBRD_LDS_MAX, ldq = q
// rounded up to odd so a thread per row reads distinct banks; p <= 1024),
// loaded in the taller orientation from M directly; outputs as k_gebrd_grid.
// Householder
// vectors are formed by one wavefront; the left reflector is applied by
// column partial sums, the right one by a thread per row.

__global__ __launch_bounds__(1024) void k_gebrd_lds(const double* __restrict__ M, int ldm,
                                                    EigJobs jobs, int* __restrict__ dims, int N,
                                                    int a_idx, int b_idx, int side_idx) {
  const EigJob J = jobs.j[0];
  if (dims[J.n_idx] < 0) return;  // solved by k_svd_jacobi
  const int a = dims[a_idx], b = dims[b_idx], side = dims[side_idx];
  const int p = side ? a : b, q = side ? b : a;
  if (!gebrd_fits(p, q)) return;
  const int lq = gebrd_ld(q);
  __shared__ double A[GEBRD_LDS_MAX];
  __shared__ double sv[1024], sp[8][128];
  __shared__ double s_tau;
  Work W = work_of(J, N);
  const int tid = threadIdx.x, cj = tid & 127, g = tid >> 7;
  const int wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < p * q; e += 1024) {
    const int i = e / q, j = e - i * q;
    A[i * lq + j] = side ? M[(long long)i * ldm + j] : M[(long long)j * ldm + i];
  }
  for (int i = tid; i < 2 * q; i += 1024) W.d[i] = 0.0;
  __syncthreads();
  for (int k = 0; k < q; ++k) {
    const int mr = p - k, nc = q - k - 1;
    if (wave == 0) {
      // left reflector of column k (rows k..p-1)
      double part = 0.0;
      for (int i = 1 + lane; i < mr; i += 64) {
        const double x = A[(k + i) * lq + k];
        part += x * x;
      }
      const double sumsq = wave_sum(part);
      const double alpha = A[k * lq + k];
      double tau, scal, beta;
      if (sumsq == 0.0) {
        tau = 0.0;
        scal = 0.0;
        beta = alpha;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sumsq), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      if (lane == 0) {
        W.e[2 * k] = beta;
        s_tau = tau;
      }
      for (int i = lane; i < mr; i += 64) sv[i] = i == 0 ? 1.0 : A[(k + i) * lq + k] * scal;
    }
    __syncthreads();
    double tau = s_tau;
    if (tau != 0.0 && nc > 0) {
      if (cj < nc) {
        double acc = 0.0;
        for (int i = g; i < mr; i += 8) acc += A[(k + i) * lq + k + 1 + cj] * sv[i];
        sp[g][cj] = acc;
      }
      __syncthreads();
      if (cj < nc) {
        double wj = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) wj += sp[t][cj];
        wj *= tau;
        for (int i = g; i < mr; i += 8) A[(k + i) * lq + k + 1 + cj] -= sv[i] * wj;
      }
      __syncthreads();
    }
    if (nc <= 0) {
      if (tid == 0) W.tau[k] = 0.0;
      continue;
    }
    if (wave == 0) {
      // right reflector of row k (columns k+1..q-1)
      double part = 0.0;
      for (int j = 1 + lane; j < nc; j += 64) {
        const double x = A[k * lq + k + 1 + j];
        part += x * x;
      }
      const double sumsq = wave_sum(part);
      const double alpha = A[k * lq + k + 1];
      double tr, scal, beta;
      if (sumsq == 0.0) {
        tr = 0.0;
        scal = 0.0;
        beta = alpha;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sumsq), alpha);
        tr = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      if (lane == 0) {
        W.e[2 * k + 1] = beta;
        W.tau[k] = tr;
        s_tau = tr;
      }
      for (int j = lane; j < nc; j += 64) {
        const double v = j == 0 ? 1.0 : A[k * lq + k + 1 + j] * scal;
        sv[j] = v;
        W.H[(long long)k * N + k + 1 + j] = v;
      }
    }
    __syncthreads();
    tau = s_tau;
    if (tau != 0.0) {
      // rows k+1..p-1: A[i, k+1:] -= tau (A[i, k+1:] . v) v^T; 128 rows at a
      // time, each row's dot product split over 8 column groups
      for (int r0 = k + 1; r0 < p; r0 += 128) {
        const int i = r0 + cj;
        double* row = A + i * lq + k + 1;
        if (i < p) {
          double acc = 0.0;
          for (int j = g; j < nc; j += 8) acc += row[j] * sv[j];
          sp[g][cj] = acc;
        }
        __syncthreads();
        if (i < p) {
          double sdot = 0.0;
#pragma unroll
          for (int t = 0; t < 8; ++t) sdot += sp[t][cj];
          sdot *= tau;
          for (int j = g; j < nc; j += 8) row[j] -= sdot * sv[j];
        }
        __syncthreads();
      }
    } else {
      __syncthreads();
    }
  }
}

// Vectors of the short side for the kept singular values, one wavefront per
// vector: y = the even entries of the tridiagonal's eigenvector, normalised,
// then y <- G_0 G_1 ... G_{q-2} y with the right reflectors.
__global__ __launch_bounds__(256) void k_svd_back(EigJobs jobs, int* __restrict__ dims, int N) {
  const EigJob J = jobs.j[0];
  const int n = dims[J.n_idx], q = n / 2;
  if (n < 0) return;  // solved by k_svd_jacobi
  const int par = dc_par(n);
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  const int N2 = next_pow2(N);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave;
  __shared__ double ys[4][1024];
  if (c >= q) return;
  const double thr = keep_threshold(J, D.lam, n);
  const int col = n - 1 - c;
  if (!(D.lam[col] > thr)) return;
  double* y = ys[wave];
  // mixing of the +-sigma pair only rescales the v-part: normalise it
  double part0 = 0.0;
  for (int i = lane; i < q; i += 64) {
    const double x = (par ? D.Qb : D.Qa)[(size_t)(2 * i) * N2 + col];
    y[i] = x;
    part0 += x * x;
  }
  const double nrm = sqrt(wave_sum(part0));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = lane; i < q; i += 64) y[i] *= inv;
  for (int k = q - 2; k >= 0; --k) {
    const double tau = W.tau[k];
    if (tau == 0.0) continue;
    const double* v = W.H + (size_t)k * N;
    double part = 0.0;
    for (int i = k + 1 + lane; i < q; i += 64) part += v[i] * y[i];
    const double dot = wave_sum(part) * tau;
    for (int i = k + 1 + lane; i < q; i += 64) y[i] -= dot * v[i];
  }
  for (int i = lane; i < q; i += 64) J.V[(size_t)i * J.ldv + c] = y[i];
}

// Descending singular values, kept count, scalings and sign gauge.
__global__ __launch_bounds__(256) void k_svd_final(EigJobs jobs, int* __restrict__ dims, int N) {
  const EigJob J = jobs.j[0];
  const int n = dims[J.n_idx], q = n / 2;
  if (n < 0) return;  // solved by k_svd_jacobi
  Work W = work_of(J, N);
  DC D = dc_of(W, N);
  __shared__ int s_kept;
  const int tid = threadIdx.x;
  const double thr = keep_threshold(J, D.lam, n);
  if (tid == 0) {
    int k = 0, bad = 0, run = 1;
    for (int c = 0; c < q; ++c) {
      const double sg = D.lam[n - 1 - c];
      if (!(sg == sg)) bad = 1;
      if (run && sg > thr) ++k;
      else run = 0;
    }
    s_kept = k;
    dims[J.kept_idx] = k;
    if (bad) atomicOr(&dims[D_FLAG], FLAG_EIG);
  }
  __syncthreads();
  const int kept = s_kept;
  for (int c = tid; c < q; c += 256) {
    const double sg = D.lam[n - 1 - c];
    J.lam[c] = sg;
    if (c < kept) {
      J.sq[c] = sg;
      J.isq[c] = 1.0 / sg;
    }
  }
  gauge_columns(J.V, J.ldv, q, kept);
}

// Dynamic LDS of k_dc_fused at capacity N: the largest of its phases' needs
// at the top level (sort and deflation, secular roots, vectors, product tiles).
size_t dc_fused_dyn_lds(int N) {
  size_t need = (size_t)2 * GEMM_GK * 65 * 8;
  for (int S = DC_LEAF; S < N; S *= 2) {
    const size_t m2 = (size_t)2 * S;
    need = std::max(need, m2 * PREP_BYTES_PER);
    need = std::max(need, m2 * 16);
    need = std::max(need, m2 * (m2 <= VEC_STAGE_MAX ? VEC_BYTES_STAGED : VEC_BYTES_GLOBAL));
  }
  return need;
}
int dc_fused_blocks(int N) { return std::min(DCF_MAXP, std::max(8, (N + 3) / 4)); }

}  // namespace

// ---- LDS budget of the launches with dynamic LDS -----------------------------
// A CU has 160 KiB of LDS; a launch asking for more static + dynamic LDS than
// that fails to dispatch.  These are the static sizes of the kernels launched
// with dynamic LDS as compiled for gfx950; at run time the larger of this and
// the runtime's own figure is used.
namespace {
constexpr size_t LDS_CU = 160 * 1024;
constexpr size_t ST_SYTRD_GRID = 168, ST_DC_FUSED = 42832, ST_ORMTR = 0, ST_GEBRD_GRID = 168,
                 ST_SVD_JACOBI = 131856;

size_t static_lds(const void* fn, size_t table, bool runtime) {
  if (!runtime) return table;
  hipFuncAttributes a;
  if (hipFuncGetAttributes(&a, fn) == hipSuccess && (size_t)a.sharedSizeBytes > table)
    return (size_t)a.sharedSizeBytes;
  return table;
}

void lds_note(size_t bytes, const char* name, size_t& worst, const char** which) {
  if (bytes > worst) {
    worst = bytes;
    if (which) *which = name;
  }
}

// divide and conquer at order N (eigensolve N, or Golub-Kahan order 2q)
void dc_lds(int N, bool rt, size_t& worst, const char** which) {
  lds_note(static_lds((const void*)k_dc_fused, ST_DC_FUSED, rt) + dc_fused_dyn_lds(N), "k_dc_fused",
           worst, which);
}
}  // namespace

size_t eig_lds_bytes(int N, bool runtime, const char** which) {
  size_t worst = 0;
  if (N > SYR_MAX)
    lds_note(static_lds((const void*)k_sytrd_grid, ST_SYTRD_GRID, runtime) + sytrd_grid_lds(N),
             "k_sytrd_grid", worst, which);
  dc_lds(N, runtime, worst, which);
  lds_note(static_lds((const void*)k_ormtr<16, 4>, ST_ORMTR, runtime) + ormtr_lds_doubles(N) * 8,
           "k_ormtr", worst, which);
  return worst;
}

size_t svd_lds_bytes(int ncap2, int pcap, bool runtime, const char** which) {
  size_t worst = 0;
  lds_note(static_lds((const void*)k_svd_jacobi, ST_SVD_JACOBI, runtime), "k_svd_jacobi", worst, which);
  const int qcap = ncap2 / 2;
  if (pcap >= GEBRD_GRID_MIN) {
    const int qc = qcap < pcap ? qcap : pcap;
    lds_note(static_lds((const void*)k_gebrd_grid, ST_GEBRD_GRID, runtime) + gebrd_grid_lds(pcap, qc),
             "k_gebrd_grid", worst, which);
  }
  dc_lds(ncap2, runtime, worst, which);
  return worst;
}

bool lds_fits(size_t bytes) { return bytes <= LDS_CU; }

size_t eig_work_doubles(int N) { return eig_work_main(N) + SYNC_DOUBLES; }

namespace {

// Divide and conquer of the tridiagonals (W.d, W.e) of the jobs; the
// eigenvectors end in buffer dc_par(n) of each job.
void dc_solve(const EigJobs& J, int njobs, int N, int* dims, hipStream_t s) {
  k_dc_fused<<<dc_fused_blocks(N), 256, dc_fused_dyn_lds(N), s>>>(J, njobs, dims, N);
}

}  // namespace

void eig_batched(const EigJob* jobs, int njobs, int N, int* dims, hipStream_t s) {
  if (njobs <= 0 || N <= 0) return;
  EigJobs J;
  for (int i = 0; i < njobs && i < 4; ++i) J.j[i] = jobs[i];
  k_sytrd_reg<<<njobs, SYR_T, 0, s>>>(J, dims, N);
  if (N > SYR_MAX) {
    const int nj = njobs < 4 ? njobs : 4;
    k_sytrd_grid<<<dim3(sytrd_grid_blocks(N), nj), SYTRD_GRID_T, sytrd_grid_lds(N), s>>>(J, dims,
                                                                                         N);
  }
  dc_solve(J, njobs < 4 ? njobs : 4, N, dims, s);
  {
    const dim3 g((N + 3) / 4, njobs), g4((N + 15) / 16, njobs);
    const size_t lds = ormtr_lds_doubles(N) * 8;
    if (N <= 192) k_ormtr<3, 1><<<g, 256, lds, s>>>(J, dims, N);
    else if (N <= 384) k_ormtr<6, 1><<<g, 256, lds, s>>>(J, dims, N);
    else if (N <= 640) k_ormtr<10, 1><<<g, 256, lds, s>>>(J, dims, N);
    else k_ormtr<16, 4><<<g4, 256, lds, s>>>(J, dims, N);
  }
  k_eig_final<<<dim3((N + FINAL_COLS - 1) / FINAL_COLS, njobs), 256, 0, s>>>(J, dims, N);
}

void svd_short_side(const double* M, int ldm, int a_idx, int b_idx, int side_idx,
                    const EigJob& job, int N, int pcap, int* dims, hipStream_t s) {
  if (N < 2) return;
  EigJobs J;
  J.j[0] = job;
  const int qcap = N / 2;
  int lb = (int)(((long long)2 * qcap * qcap + 255) / 256);
  if (lb > 1024) lb = 1024;
  if (lb < 1) lb = 1;
  k_svd_load<<<lb, 256, 0, s>>>(M, ldm, J, dims, a_idx, b_idx, side_idx);
  k_svd_jacobi<<<1, JAC_T, 0, s>>>(M, ldm, J, dims, a_idx, b_idx, side_idx);
  k_gebrd_lds<<<1, 1024, 0, s>>>(M, ldm, J, dims, N, a_idx, b_idx, side_idx);
  if (pcap >= GEBRD_GRID_MIN) {
    const int qc = qcap < pcap ? qcap : pcap;
    const int P = gebrd_grid_blocks(pcap, qc);
    const size_t lds = gebrd_grid_lds(pcap, qc);
    k_gebrd_grid<<<P, 256, lds, s>>>(J, dims, N, a_idx, b_idx, side_idx, qc, (int)(lds / 8));
  }
  dc_solve(J, 1, N, dims, s);
  k_svd_back<<<(qcap + 3) / 4, 256, 0, s>>>(J, dims, N);
  k_svd_final<<<1, 256, 0, s>>>(J, dims, N);
}

}  // namespace tt
