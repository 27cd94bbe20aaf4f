/*
 * tt_kernels.h -- kernel-level entry points of libtt.so.
 *
 * These expose the individual contractions and the eigensolver used inside
 * one Gram-SVD rounding (paper App. A.2) so that each can be checked
 * against a plain reference on random inputs.  All matrix pointers are
 * device memory, row-major float64, caller-owned.  `ws` is caller-owned
 * device scratch of at least the bytes returned by the matching
 * *_workspace() query.  Each call runs on `stream` (a hipStream_t, NULL =
 * default) and returns after a stream synchronisation.  Errors:
 * TT_ERR_INVALID_ARG (sizes, null pointers), TT_ERR_OOM (ws too small),
 * TT_ERR_DEVICE (HIP failure); messages via tt_last_error(NULL).
 */
#ifndef TT_KERNELS_H
#define TT_KERNELS_H

#include "tt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Symmetric eigendecomposition of A (n x n, lda; not modified) for
 * 1 <= n <= 1024 (App. A.2: G = V S^2 V^T).  lam (n): eigenvalues in
 * descending order.  V (n x n, ldv): columns = eigenvectors of the kept
 * eigenvalues, each signed so that its largest-magnitude entry is positive.
 * Kept: lambda > clip * n * 2^-53 * lambda_max and lambda > 0 (clip = 1 is
 * the Gram clip rule; clip = 0 keeps every positive eigenvalue).
 * kept (host int) receives the number kept. */
size_t tt_kernel_eigh_workspace(int32_t n);
tt_status tt_kernel_eigh(const double* A, int32_t n, int32_t lda, double clip, double* lam,
                         double* V, int32_t ldv, int32_t* kept, void* ws, size_t ws_bytes,
                         void* stream);

/* Singular values and the singular vectors of the short side of the
 * a x b matrix M (row-major, ldm >= b, device), as the Gram-SVD truncation
 * needs them for M = S_A V_A^T V_B S_B (App. A.2): Householder
 * bidiagonalisation, then divide and conquer on the order-2q Golub-Kahan
 * tridiagonal (q = min(a, b)), whose eigenvalues are +-sigma.
 * sig (q, device) receives sigma descending; V (device, ldv >= q) receives
 * the left singular vectors (a x q) when a <= b, else the right ones
 * (b x q), each column signed so its largest |entry| is positive.  kept
 * (host int) = number with sigma > 2q * 2^-53 * sigma_1 (vectors beyond it
 * are not written).  1 <= a, b <= 1024. */
size_t tt_kernel_svd_workspace(int32_t a, int32_t b);
tt_status tt_kernel_svd(const double* M, int32_t a, int32_t b, int32_t ldm, double* sig, double* V,
                        int32_t ldv, int32_t* kept, void* ws, size_t ws_bytes, void* stream);

/* G (n x n, ldg) = A^T A for A of K rows and n columns (lda >= n):
 * the left Gram of a tall core on MFMA, split over K with a fixed-order
 * (deterministic) reduction. */
size_t tt_kernel_gram_workspace(int32_t K, int32_t n, int32_t lda);
tt_status tt_kernel_gram(const double* A, int32_t K, int32_t n, int32_t lda, double* G,
                         int32_t ldg, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * G = A^T A as tt_kernel_gram, with no workspace argument.  Its scratch (a
 * 64-int size table and the per-block partial Gram tiles) lives in a
 * library-owned 32 MiB device array per GPU, held until the process ends;
 * the call allocates nothing.  Sizes whose partial tiles do not fit (about
 * 256 row blocks x ceil(n/32)(ceil(n/32)+1)/2 tiles of 8 KiB for n <= 384,
 * e.g. every K for n <= 160) return TT_ERR_INVALID_ARG.  All calls on one
 * GPU share the array and every call overwrites it: calls that overlap on
 * one GPU (other streams, other threads) race and must be serialised by the
 * caller. */
tt_status tt_kernel_gram_noalloc(const double* A, int32_t K, int32_t n, int32_t lda, double* G,
                                 int32_t ldg, void* stream);

/* G (n x n, ldg, FP64) = A^T A for an FP32 matrix A (K rows, n <= 1024
 * columns, lda >= n): the Gram formation of the FP32-mixed precision form.
 * Each entry is split on its column's exponent grid into four 11-bit integer
 * slices; slice products are summed four rows at a time on FP32 MFMA, where
 * the sums are exact, and accumulated in FP64.  G is therefore the Gram of
 * A to within 2^-44 of the product of the two columns' largest entries per
 * term (compensated split products; App. A.2 needs the Gram accurate down
 * to the truncation tolerance squared). */
size_t tt_kernel_gram_f32_workspace(int32_t K, int32_t n, int32_t lda);
tt_status tt_kernel_gram_f32(const float* A, int32_t K, int32_t n, int32_t lda, double* G,
                             int32_t ldg, void* ws, size_t ws_bytes, void* stream);

/* C (K x n, ldc) = A (K x k, lda) B (k x n, ldb) on MFMA (the core update
 * A' = A P of App. A.2). */
size_t tt_kernel_gemm_tall_workspace(void);
tt_status tt_kernel_gemm_tall(const double* A, int32_t K, int32_t k, int32_t lda, const double* B,
                              int32_t n, int32_t ldb, double* C, int32_t ldc, void* ws,
                              size_t ws_bytes, void* stream);

/* C (m x n, ldc) = op(A) op(B), op = transpose when ta / tb != 0; the
 * generic rank-sized product.  ws: tt_kernel_gemm_tall_workspace() bytes. */
tt_status tt_kernel_gemm(const double* A, int32_t lda, int32_t ta, const double* B, int32_t ldb,
                         int32_t tb, double* C, int32_t ldc, int32_t m, int32_t n, int32_t k,
                         void* ws, size_t ws_bytes, void* stream);

/* LDS budget check (host only, no device work): the largest static + dynamic
 * LDS of any launch of the symmetric eigensolver at order n and of the SVD
 * at Golub-Kahan order ncap2 (= 2 min(a, b)) with longer side pcap (0
 * skips either), written to max_bytes.  TT_OK when every launch fits the
 * 160 KiB of one CU, else TT_ERR_INVALID_ARG naming the kernel.  Every
 * context and every eigh/svd call applies the same check, with the HIP
 * runtime's static sizes, before launching. */
tt_status tt_kernel_lds_check(int32_t n, int32_t ncap2, int32_t pcap, size_t* max_bytes);

/* Peak microbenchmarks of this GPU, for roofline fractions against what it
 * delivers: which = 0, HBM streaming copy of copy_bytes (16-byte loads and
 * stores), repeated `iters` times, result in GB/s counting read + write;
 * which = 1 / 2, dense FP64 / FP32 MFMA (16x16x4 on register operands,
 * `iters` rounds of four independent products per wavefront on 2048 blocks
 * of four wavefronts), result in TFLOP/s.  ws: device scratch of
 * tt_kernel_microbench_workspace(which, copy_bytes) bytes.  Timed with HIP
 * events on `stream` after one untimed launch. */
size_t tt_kernel_microbench_workspace(int32_t which, size_t copy_bytes);
tt_status tt_kernel_microbench(int32_t which, size_t copy_bytes, int32_t iters, void* ws,
                               size_t ws_bytes, double* result, void* stream);

/* Message of the last failed kernel-level call on this thread. */
const char* tt_kernel_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TT_KERNELS_H */
