/*
 * mlk_host.h -- C ABI of the host (CPU) kernels: the multi-core OpenMP form of
 * the paper's two kernels, with a searched tiling and unroll factor.
 *
 * The paper lowers its convolution's parallel loops to OpenMP worksharing
 * loops (Sec. 4.2, the end-to-end OpenMP pipeline) and tunes tile sizes and an
 * unroll factor by black-box search over measured run time (Sec. 4.3, where
 * the OpenMP variant is one of the measured targets).  These entry points are
 * that CPU path for linalg.matmul (Sec. 2.1, listing "linalg-matmul") and
 * linalg.conv_2d_nchw_fchw (Sec. 4.1, listing "2dnchwconv") in fp32.
 *
 * This library is separate from the GPU library (libmlk.so): no GPU entry
 * point calls it, and it calls no GPU code.  Every pointer is a HOST pointer;
 * the caller owns every buffer.  Calls block until the result is written.
 * Results are fp32 sums in a tiled order (not the plain nest's order): within
 * the usual fp32 bound of the exact result.
 */
#ifndef MLK_HOST_H
#define MLK_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes: the values of mlk_status in mlk.h. */
enum { MLKH_OK = 0, MLKH_ERR_NULL = 1, MLKH_ERR_SHAPE = 2, MLKH_ERR_LAYOUT = 3, MLKH_ERR_CONFIG = 5,
       MLKH_ERR_ARG = 9 };

/*
 * Host tiling.  Matmul: the output is cut into mb x nb blocks (one OpenMP
 * work item each, scheduled over `threads` threads), the depth into kb-deep
 * slabs; `unroll` rows of C are updated together per step of k (each loaded
 * row slice of B feeds `unroll` rows; 1, 2, 4 or 8).  Conv: mb is the number
 * of filters per work item (work items are (image, filter block, output
 * row)), `unroll` filters share each loaded input row (1, 2, 4 or 8); nb and
 * kb are unused (0).  threads = 0 uses every thread OpenMP offers.
 * A zeroed configuration means "choose" (a built-in default).
 */
typedef struct {
    int32_t mb, nb, kb;
    int32_t unroll;
    int32_t threads;
} mlkh_config;

/* C[M,N] (+)= A[M,K] * B[K,N], row-major fp32 (lda >= K, ldb >= N, ldc >= N);
 * accumulate = 0 overwrites C.  M, N, K >= 0. */
int mlkh_matmul_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B, int64_t ldb,
                    float* C, int64_t ldc, int accumulate, const mlkh_config* cfg);

/* y[n,f,oh,ow] (+)= sum_{c,kh,kw} x[n,c,oh*sh-ph+kh,ow*sw-pw+kw] * w[f,c,kh,kw],
 * contiguous NCHW / FCHW / NFHW fp32, zero padding, HO = (H+2ph-KH)/sh+1. */
int mlkh_conv2d_f32(int64_t N, int64_t C, int64_t H, int64_t W, int64_t F, int64_t KH, int64_t KW, int32_t sh,
                    int32_t sw, int32_t ph, int32_t pw, const float* x, const float* w, float* y, int accumulate,
                    const mlkh_config* cfg);

/*
 * Search the host tiling of one problem (op 0: matmul M, N, K; op 1: conv with
 * dims[] = {N, C, H, W, F, KH, KW, sh, sw, ph, pw}) on seeded scratch inputs
 * of that shape: strategy 0 measures every configuration of the space, 1 a
 * (1+1) evolution strategy over the fields that stops after
 * ceil(budget_frac * S) measurements.  Each measurement is the median of
 * `reps` timed calls (wall clock).  *best receives the fastest, *best_us its
 * time; times_us (may be NULL, length mlkh_config_count) receives every
 * measured time in enumeration order, -1 where not measured.
 */
int32_t mlkh_config_count(int32_t op, const int64_t* dims);
int mlkh_config_get(int32_t op, const int64_t* dims, int32_t i, mlkh_config* cfg);
int mlkh_tune(int32_t op, const int64_t* dims, int32_t strategy, double budget_frac, int32_t reps, uint64_t seed,
              mlkh_config* best, double* best_us, double* times_us);

/* Threads OpenMP offers this process. */
int32_t mlkh_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif /* MLK_HOST_H */
