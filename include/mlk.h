/*
 * mlk.h -- C ABI of the MI355X (gfx950) dense-kernel library for the
 * computations of "nelli: A lightweight frontend for MLIR" (arXiv 2307.16080).
 *
 * The paper defines its kernels as destination-passing functions over typed,
 * shaped, row-major buffers: matmul(A, B, C) with C updated in place
 * (Sec. 1, listing "nelli_for_to_affine_for"; Sec. 2.1, listing
 * "linalg-matmul") and conv2d_nchw_fchw(input, kernel, output) accumulating
 * into output (Sec. 4.1, listing "2dnchwconv"), and chooses tile sizes and
 * unroll factors by black-box search over measured run times (Sec. 4.3).
 * This header exposes those operations for hand-written CDNA4 kernels.
 *
 * Conventions for every entry point:
 *  - Pointers named A, B, C, x, w, y, q, descs' A/B/C, scale pointers and
 *    statistic outputs are DEVICE pointers (HIP allocations, e.g. torch CUDA
 *    tensors) unless stated otherwise.  Structs passed by pointer
 *    (mlk_tile_config, mlk_problem, mlk_tune_opts, mlk_gemm_desc arrays,
 *    mlk_tune_report) are HOST memory.
 *  - The caller owns every buffer it passes; the library never frees or
 *    reallocates them.  The library owns its internal workspaces (reduction
 *    partials, device task lists, captured graphs) and frees them in
 *    mlk_release().
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Launch entry points enqueue work on it and return without synchronising;
 *    device faults therefore surface at the caller's next synchronisation.
 *  - Every argument is validated on the host before any HIP call, so all
 *    MLK_ERR_* codes except MLK_ERR_HIP can be produced without a GPU.  On
 *    error nothing is enqueued and mlk_last_error() returns a thread-local
 *    message.
 *  - Scratch memory: the routes that need a workspace (a direct-to-LDS
 *    matmul tile whose operands need zero-padded copies, the channels-last
 *    conv layout, e4m3 quantisation, the error statistics and the MLP
 *    kernels' activations) use one library-owned buffer per device,
 *    grown on demand up to 512 MiB and held until mlk_release(); larger
 *    requests take a stream-ordered allocation of their own for the call.
 *    Uses of the buffer are ordered on the device with an event, whatever
 *    streams they run on.
 *  - Stream capture: those workspace routes are not recorded into a captured
 *    graph: on a stream that is capturing they return MLK_ERR_CONFIG and
 *    enqueue nothing.  Configurations without a workspace (register-loaded
 *    tiles, aligned direct-to-LDS operands, conv layout 0) may be captured;
 *    so may every run of a bound convolution (mlk_conv2d_plan_run, whose
 *    buffers are allocated when the plan is created) and mlk_matmul_noalloc.
 *  - Thread safety: calls from several host threads are safe; calls that
 *    overlap on one device share its workspaces and are serialised inside
 *    the library.
 */
#ifndef MLK_H
#define MLK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLK_OK = 0,
    MLK_ERR_NULL = 1,        /* a required pointer is NULL */
    MLK_ERR_SHAPE = 2,       /* a dimension is negative / zero where not allowed, or too large */
    MLK_ERR_LAYOUT = 3,      /* leading dimension too small, or output aliases an input */
    MLK_ERR_DTYPE = 4,       /* unsupported (input, output) dtype pair for the operation */
    MLK_ERR_CONFIG = 5,      /* tile configuration not legal for the problem */
    MLK_ERR_DB = 6,          /* tuning database unreadable / unwritable */
    MLK_ERR_HIP = 7,         /* a HIP runtime call failed; message has the HIP error */
    MLK_ERR_NOMEM = 8,       /* host or device allocation failed */
    MLK_ERR_ARG = 9          /* any other invalid argument (flag, option, strategy) */
} mlk_status;

typedef enum {
    MLK_F32 = 0,     /* IEEE binary32 */
    MLK_BF16 = 1,    /* bfloat16 (binary32 with 16 fraction bits dropped) */
    MLK_F8E4M3 = 2,  /* OCP 8-bit float E4M3 (bias 7, max 448, no inf) */
    MLK_I8 = 3,      /* two's complement int8 */
    MLK_I32 = 4      /* two's complement int32 */
} mlk_dtype;

/*
 * Tile configuration: the search space of the paper's tiling + unrolling
 * experiment (Sec. 4.3: parallel-loop tile sizes and an unroll factor),
 * re-expressed for a workgroup-tiled MFMA kernel.
 *   bm, bn     output tile per workgroup (rows of C x columns of C)
 *   bk         contraction depth staged in LDS per main-loop step (elements);
 *              the K-loop is unrolled over bk in steps of one MFMA.
 *   wm, wn     waves (64 lanes) per workgroup along M and N
 *   split_k    number of workgroups sharing one output tile along K (>= 1);
 *              > 1 adds partial results with atomics (floating-point
 *              results then depend on arrival order within rounding).
 *   group_m    workgroup raster: tiles are visited in column bands of group_m
 *              tile-rows (1 = row-major order)
 *   xcd_remap  1: map consecutive tiles to the same XCD (shared L2)
 *   stages     0: register-staged kernel (operands pass through registers
 *              on their way to a double-buffered LDS tile; any shape and
 *              alignment).  2..5: direct-to-LDS kernel (bf16, e4m3) whose
 *              loads go from memory straight into a ring of `stages` LDS
 *              buffers; matmul operands without 16-byte rows, with K not
 *              a multiple of bk, or (B) with N not a multiple of 16 bytes, are
 *              first copied into zero-padded buffers (library scratch memory); the bf16 conv tiles of this form
 *              (channels-last layout) need C*KH*KW a multiple of bk.  1: the
 *              same kernel with its operands loaded through registers into
 *              two LDS buffers (bf16, e4m3; bf16 channels-last conv): any
 *              shape and alignment, and usable by the persistent batched
 *              launch.  For fp32 conv (layout 0), 1 is the chunk-gather
 *              tile: bk-deep chunks of filter and im2col input requested
 *              whole, up to six chunks in flight in registers, one LDS
 *              buffer; any shape with N*C*H*W below 2^31 and
 *              C*KH*KW*KH*KW below 2^32; its split_k may leave one chunk
 *              per part.
 *   layout     conv2d only.  0: the kernel gathers its operands straight from
 *              the NCHW input (any C).  1: the input is first transposed to
 *              channels-last (NHWC) and the filter to F x KH x KW x C in the
 *              library's scratch memory (one launch for both), so every
 *              operand load is one aligned 16-byte read; needs C a multiple
 *              of 8 (bf16) or 4 (fp32) and 16-byte aligned x and w.  3: the
 *              channel gather (bf16, register-loaded conv tiles, stages 1):
 *              the kernel reads the NCHW input itself, each 16-byte LDS chunk
 *              being 8 channels of one input pixel (8 two-byte loads H*W
 *              elements apart), so no input copy is made; the filter is used
 *              as F x KH x KW x C (a 1 x 1 filter as it is; otherwise a
 *              transposed copy in scratch memory per call, or once per bound
 *              convolution); needs C a multiple of 8 and F <= 65535.  2: the
 *              direct (stencil) conv, no GEMM tiling: a workgroup computes a
 *              bm x bn block of output pixels (bn = 64) for all F filters
 *              from the input window staged in LDS; its configurations have
 *              bk = 1, wm = wn = 0, split_k = 1, and it needs F <= 16,
 *              strides <= 2 and filters up to 7 x 7.  Must be 0 for matmul.
 *   mfma       output tile of one MFMA instruction: 0 or 16 (16 x 16, every
 *              kernel), 32 (32 x 32 x 16 bf16: twice the flops per MFMA
 *              instruction, half the instructions; direct-layout bf16 matmul
 *              tiles, fp32 or bias outputs).
 * A zeroed struct or a NULL pointer means "choose": the tuning database
 * entry for this problem if one was loaded, else a built-in heuristic.
 */
typedef struct {
    int32_t bm, bn, bk;
    int32_t wm, wn;
    int32_t split_k;
    int32_t group_m;
    int32_t xcd_remap;
    int32_t stages;
    int32_t layout;
    int32_t mfma;
} mlk_tile_config;

/*
 * C[M,N] (+)= A[M,K] * B[K,N]   -- linalg.matmul (Sec. 2.1, listing
 * "linalg-matmul"; Sec. 1, listing "nelli_for_to_affine_for").
 *
 * Row-major operands: A[i,k] at A[i*lda + k], B[k,j] at B[k*ldb + j],
 * C[i,j] at C[i*ldc + j]; lda >= K, ldb >= N, ldc >= N.
 * Supported (in, out) pairs:
 *   (MLK_F32,    MLK_F32)  fp32 products on MFMA, fp32 accumulation
 *   (MLK_BF16,   MLK_F32)  bf16 products, fp32 accumulation
 *   (MLK_F8E4M3, MLK_F32)  e4m3 products, fp32 accumulation, then the result
 *                          is multiplied by (*scale_a) * (*scale_b)
 *   (MLK_I8,     MLK_I32)  sign-extended int8 products, int32 sums that
 *                          wrap modulo 2^32; bit-exact
 *   (MLK_BF16,   MLK_BF16) bf16 output: the fp32 result (with accumulate, the
 *   (MLK_F8E4M3, MLK_BF16) bf16 C read back and added in fp32) is rounded
 *                          once to bf16, to nearest even, in the kernel's
 *                          output stage; C is M x N bf16 with row stride ldc
 *                          (elements).  A result rounded once from the whole
 *                          sum cannot be split over K: split_k must be 1; the
 *                          register-loaded fast tiles (stages 1) are refused.
 * accumulate = 1: C += product (the linalg "outs" semantics);
 * accumulate = 0: C = product (C is not read).
 * scale_a / scale_b: device pointers to one float each (MLK_F8E4M3 only; NULL
 * means 1.0), e.g. as written by mlk_quantize.
 * M, N, K >= 0; M == 0 or N == 0 is a no-op; K == 0 leaves C (accumulate) or
 * zeroes it (overwrite).  C must not overlap A or B.
 * cfg: NULL or zeroed = choose (see mlk_tile_config); otherwise must satisfy
 * mlk_config_legal or MLK_ERR_CONFIG is returned.
 */
mlk_status mlk_matmul(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                      const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                      int64_t ldc, const float* scale_a, const float* scale_b, int accumulate,
                      const mlk_tile_config* cfg, void* stream);

/*
 * mlk_matmul for callers that cannot allocate device memory: code recorded
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, dtypes, results and errors as mlk_matmul, and
 * the same kernels; the only difference is where a direct-to-LDS tile's
 * zero-padded operand copies go (needed when A or B lacks 16-byte rows, K
 * is not a multiple of the tile depth, or B's N is not a multiple of 16
 * bytes): into a fixed device array of
 * MLK_NOALLOC_WORKSPACE_BYTES (64 MiB), one per device, held by the library
 * until the process ends, instead of the library's growable scratch buffer.
 * The call allocates nothing, takes no scratch lock, and may be captured.
 * A shape and tile whose packed copies exceed the array return
 * MLK_ERR_SHAPE before anything is enqueued.
 * Every call on one device shares that device's array: calls that overlap
 * in time on one device (different streams, or several host threads) race on
 * it; order them on one stream.  The packing kernel writes every byte the
 * GEMM reads, so nothing carries over from an earlier call.
 */
#define MLK_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
mlk_status mlk_matmul_noalloc(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                              const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                              int64_t ldc, const float* scale_a, const float* scale_b, int accumulate,
                              const mlk_tile_config* cfg, void* stream);

/*
 * The Linear layer: C[i,j] (+)= sum_k A[i,k] * B[k,j] + bias[j]  -- the
 * product nest followed by the bias nest that adds bias[j] to every row
 * (Sec. 2.1, listing "listing1"), with the bias add fused into the product's
 * output stage instead of a second pass over C.
 * Same arguments, dtypes and conventions as mlk_matmul, plus
 * bias: device pointer to N floats (must not overlap C).  Float outputs only:
 * (MLK_I8, MLK_I32) returns MLK_ERR_DTYPE.  For MLK_F8E4M3 the bias is added
 * after the scale: C (+)= scale_a * scale_b * (A B) + bias.  With a bf16
 * output the bias is added in fp32 before the one rounding.
 * accumulate = 1: C += A B + bias; accumulate = 0: C = A B + bias.
 * K == 0 gives C (+)= bias.  bias == NULL with M, N > 0 is MLK_ERR_NULL.
 * The tile configuration is chosen (and tuned) as for mlk_matmul of the same
 * shape.
 */
mlk_status mlk_matmul_bias(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                           const void* A, int64_t lda, const void* B, int64_t ldb,
                           const float* bias, void* C, int64_t ldc, const float* scale_a,
                           const float* scale_b, int accumulate, const mlk_tile_config* cfg,
                           void* stream);

/*
 * y[n,f,oh,ow] (+)= sum_{c,kh,kw} x[n,c,oh*sh-ph+kh, ow*sw-pw+kw] * w[f,c,kh,kw]
 * -- linalg.conv_2d_nchw_fchw (Sec. 4.1, listing "2dnchwconv"), generalised
 * to stride (sh, sw) and symmetric zero padding (ph, pw): taps that fall
 * outside the image read zero; no filter flip (cross-correlation).
 * Contiguous layouts: x (N,C,H,W), w (F,C,KH,KW), y (N,F,HO,WO) with
 * HO = floor((H + 2ph - KH)/sh) + 1, WO likewise.
 * Supported (in, out): (MLK_F32, MLK_F32) and (MLK_BF16, MLK_F32).
 * Computed as an implicit GEMM: rows = F, columns = N*HO*WO,
 * depth = C*KH*KW, with the im2col gather done inside the kernel's loads.
 * All dims >= 1, strides >= 1, pads >= 0, HO, WO >= 1.
 */
mlk_status mlk_conv2d_nchw_fchw(mlk_dtype in, mlk_dtype out, int64_t N, int64_t C, int64_t H,
                                int64_t W, int64_t F, int64_t KH, int64_t KW, int32_t sh,
                                int32_t sw, int32_t ph, int32_t pw, const void* x, const void* w,
                                void* y, int accumulate, const mlk_tile_config* cfg, void* stream);

/*
 * A convolution bound once to its shape, tile configuration and filter, for
 * callers that run the same layer many times (a network's layers in a
 * serving loop), including under HIP graph capture.  Same operation, dtypes
 * and results as mlk_conv2d_nchw_fchw (Sec. 4.1, listing "2dnchwconv").
 *
 * mlk_conv2d_plan_create validates the problem, resolves the configuration
 * (cfg NULL or zeroed: the tuned default or the heuristic, as for
 * mlk_conv2d_nchw_fchw), and, for the channels-last layout (layout 1),
 * allocates the plan's own buffers (an NHWC copy of the input and, for
 * filters larger than 1 x 1, the filter as F x KH x KW x C) and enqueues the
 * filter's transpose on `stream`; for the channel-gather layout (layout 3)
 * only the transposed filter (none for a 1 x 1 filter), so that each run is
 * a single kernel launch.  It must not be called on a capturing
 * stream (MLK_ERR_CONFIG).  `w` (device, FCHW) is bound to the plan: runs use
 * its values as of creation (or of the last mlk_conv2d_plan_update_filter,
 * which re-reads it, stream-ordered); it must stay allocated while the plan
 * exists.  `accumulate` is fixed per plan.  On success *plan owns the
 * buffers; free with mlk_conv2d_plan_destroy (which waits for the device).
 *
 * mlk_conv2d_plan_run computes y (+)= conv(x, w) on `stream`: x (N,C,H,W) and
 * y (N,F,HO,WO) contiguous device buffers (x 16-byte aligned for layout 1);
 * it allocates nothing, takes no library lock and may be recorded into a
 * captured graph.  Runs of one plan that overlap in time (several streams)
 * race on its input copy; different plans are independent.  The plan must be
 * run on the device it was created on.
 * mlk_conv2d_plan_config returns the configuration the plan resolved.
 */
typedef struct mlk_conv_plan mlk_conv_plan;
mlk_status mlk_conv2d_plan_create(mlk_dtype in, mlk_dtype out, int64_t N, int64_t C, int64_t H, int64_t W,
                                  int64_t F, int64_t KH, int64_t KW, int32_t sh, int32_t sw, int32_t ph,
                                  int32_t pw, const void* w, int accumulate, const mlk_tile_config* cfg,
                                  void* stream, mlk_conv_plan** plan);
mlk_status mlk_conv2d_plan_run(const mlk_conv_plan* plan, const void* x, void* y, void* stream);
mlk_status mlk_conv2d_plan_update_filter(mlk_conv_plan* plan, void* stream);
mlk_status mlk_conv2d_plan_config(const mlk_conv_plan* plan, mlk_tile_config* cfg);
void mlk_conv2d_plan_destroy(mlk_conv_plan* plan);

/*
 * Many independent convolutions in one persistent launch (Sec. 4.1's
 * linalg.conv_2d_nchw_fchw, once per descriptor; the batching of uneven
 * problems into one launch is this library's, as for mlk_batched_matmul).
 *
 * Each descriptor is one convolution y (+)= conv(x, w) with the layouts of
 * mlk_conv2d_nchw_fchw: x (N,C,H,W) bf16, w (F,C,KH,KW) bf16, y (N,F,HO,WO)
 * fp32, contiguous device buffers bound at creation (their contents are read
 * at each run; x and w must stay allocated while the batch exists).  Every
 * convolution needs C a multiple of 8 and F <= 65535; no y may overlap any
 * descriptor's x, w or y.
 *
 * mlk_conv2d_batch_create validates the descriptors, allocates the batch's
 * device buffers (each filter transposed to F x KH x KW x C, except 1 x 1
 * filters, which are used in place; the convolutions' arguments and the
 * schedule), enqueues the filter transposes on `stream`, and plans the launch:
 * every convolution is cut into tasks -- an output tile of the register-loaded
 * channel-gather conv kernel (conv layout 3) and one part of a K split --
 * that are dealt longest first into one range per resident workgroup.  A
 * convolution of S 64-deep stages is split into min(cap, ceil(S / 4)) parts
 * (cap: cfg->split_k, 1 .. 32), so each task keeps its loads in flight at
 * once; split parts add into y with fp32 atomics.  cfg NULL or zeroed: the
 * 64 x 64 tile, cap 16; otherwise cfg selects bm, bn, wm, wn of a
 * register-loaded conv tile (stages 1, layout 3) and the cap; other fields
 * must be zero or their defaults (group_m 0/1).  Not on a capturing stream.
 *
 * mlk_conv2d_batch_run enqueues the batch on `stream`: with accumulate = 0,
 * first a zero fill of each split convolution's y, then the one persistent
 * launch.  It allocates nothing and may be recorded into a captured graph.
 * Runs of one batch must not overlap in time; the batch must run on the
 * device it was created on.  mlk_conv2d_batch_update_filters re-reads every
 * w (stream-ordered).  mlk_conv2d_batch_info reports the tile configuration
 * (split_k = the cap), the task count and the workgroups of the launch.
 * mlk_conv2d_batch_destroy waits for the device and frees the batch.
 */
typedef struct {
    int64_t N, C, H, W, F, KH, KW;
    int32_t sh, sw, ph, pw;
    const void* x;
    const void* w;
    void* y;
} mlk_conv_desc;
typedef struct mlk_conv_batch mlk_conv_batch;
mlk_status mlk_conv2d_batch_create(mlk_dtype in, mlk_dtype out, int64_t count, const mlk_conv_desc* descs,
                                   int accumulate, const mlk_tile_config* cfg, void* stream,
                                   mlk_conv_batch** batch);
mlk_status mlk_conv2d_batch_run(const mlk_conv_batch* batch, void* stream);
mlk_status mlk_conv2d_batch_update_filters(mlk_conv_batch* batch, void* stream);
mlk_status mlk_conv2d_batch_info(const mlk_conv_batch* batch, mlk_tile_config* cfg, int64_t* tasks,
                                 int32_t* workgroups);
void mlk_conv2d_batch_destroy(mlk_conv_batch* batch);

/*
 * The matrix cores' sustained rate, to set beside the datasheet peak (the
 * measured ceiling that a GEMM's roofline fraction can be read against): one
 * launch of 2 x CUs workgroups of four waves, each wave running `iters` steps
 * of eight independent 16x16x32 bf16 (in = MLK_BF16) or 16x16x128 e4m3
 * (MLK_F8E4M3) MFMAs on register operands, with no memory traffic in the
 * loop.  *flops receives the launch's flop count (the caller times the
 * launch, e.g. with events on `stream`).  Every operand is 1.0 and chain c
 * starts at c, so wave w writes out[w] = 28 + 8 * iters * k exactly (k = 32
 * bf16, 128 e4m3).  out: device
 * buffer of out_len >= 8 * CUs floats; iters in [1, 16384].
 */
mlk_status mlk_mfma_rate(mlk_dtype in, int64_t iters, float* out, int64_t out_len, int64_t* flops, void* stream);

/*
 * Quantise n fp32 values for the low-precision paths.
 *   out = MLK_BF16:   q[i] = bf16 round-to-nearest-even of x[i]; scale unused
 *                     (may be NULL).  NaN becomes a quiet NaN, overflow inf.
 *   out = MLK_F8E4M3: amax = max |x[i]| (NaNs ignored); s = amax / 448
 *                     rounded to fp32 (s = 1 when amax is 0 or not finite);
 *                     q[i] = e4m3(RNE(x[i] / s)) with the quotient rounded to
 *                     fp32 first and magnitudes beyond 448 saturated to 448;
 *                     *scale = s (device float).
 * x, q, scale device pointers; q has n elements of the output type.
 * e4m3 runs in one launch when x is 16-byte aligned and fits the registers of
 * a grid that is all resident at once (up to 16.8 M values on an MI355X): the
 * workgroups exchange their maxima through device words and then encode.  Its
 * waits are bounded (if work on other streams keeps some workgroups from
 * starting, the resident ones wait up to that bound); a workgroup that stops
 * waiting scans x for the maximum itself, so the codes are the same.  The
 * environment variable MLK_QUANT_WAIT_POLLS sets the bound in polls (tests).
 * Larger or unaligned inputs take two launches (maximum, then codes).
 * e4m3 takes the library's scratch memory (not under stream capture), which
 * also orders concurrent e4m3 calls on any streams.
 * Per-tensor scaling as in the fp8 extension; the paper itself is fp32-only.
 */
mlk_status mlk_quantize(mlk_dtype out, int64_t n, const float* x, void* q, float* scale,
                        void* stream);

/* One GEMM of a batch: C = A * B (+ C) with the conventions of mlk_matmul. */
typedef struct {
    int64_t M, N, K;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    void* C;
    int64_t ldc;
} mlk_gemm_desc;

#define MLK_BATCH_PERSISTENT 0x1u /* one persistent launch over all tiles of all GEMMs */
#define MLK_BATCH_GRAPH 0x2u      /* capture the launch(es) in a hipGraph, cached per batch */

/*
 * Many independent matmuls of different shapes (the extension that batches
 * uneven GEMMs into one launch).  descs: HOST array of `count` descriptors
 * (device A/B/C pointers inside).  Supported (in, out): (MLK_BF16, MLK_F32),
 * (MLK_F32, MLK_F32).
 * cfgs / ncfgs: the tile configurations (HOST array).
 *   ncfgs = 0 (cfgs ignored): one configuration for the whole batch, its
 *     tuned choice (mlk_tune on the MLK_OP_BATCHED problem) else a heuristic;
 *   ncfgs = 1: cfgs[0] for every GEMM;
 *   ncfgs = count: cfgs[i] for GEMM i; a zeroed entry leaves GEMM i to choose:
 *     per-GEMM launches take its own tuned matmul configuration (else the
 *     heuristic for its shape), persistent launches the batch's choice.
 * Other ncfgs values return MLK_ERR_ARG.
 * flags: 0 = one launch per GEMM, each with its configuration (split_k
 * honoured); MLK_BATCH_PERSISTENT = one persistent launch per kernel used by
 * the batch (GEMMs whose configurations share a kernel form one group; the
 * groups run one after another), whose workgroups walk a precomputed,
 * load-balanced list of (GEMM, tile) tasks, split_k ignored;
 * MLK_BATCH_GRAPH = replay a hipGraph captured on the first call with the
 * same descriptors, configurations and flags (the graph bakes in the device
 * pointers, so a changed pointer is a new batch; a graph of per-GEMM launches
 * takes its packed operand copies from a workspace the cached batch owns,
 * not from scratch memory).  Persistent task lists, workspaces and graphs are
 * cached per batch, at most 16 (the least recently used is freed first, after
 * a device synchronisation), and freed by mlk_release().
 * Results equal per-GEMM mlk_matmul calls with the same configurations
 * (split_k 1).
 */
mlk_status mlk_batched_matmul(mlk_dtype in, mlk_dtype out, int64_t count,
                              const mlk_gemm_desc* descs, const mlk_tile_config* cfgs, int64_t ncfgs,
                              int accumulate, uint32_t flags, void* stream);

/*
 * Error statistics of a computed result against a double-precision
 * reference, reduced on the GPU in FP64:
 *   out[0] = sum (c_i - r_i)^2     out[1] = sum r_i^2
 *   out[2] = max |c_i - r_i|       out[3] = max |c_i - r_i| / bound_i over
 *                                           bound_i > 0 (0 if bound is NULL)
 * c: n values of c_dtype (MLK_F32 or MLK_I32); r, bound: n doubles; out: 4
 * doubles.  All device pointers.  The summation order is fixed (two-level
 * tree), so results are reproducible run to run.
 */
mlk_status mlk_err_stats(mlk_dtype c_dtype, int64_t n, const void* c, const double* r,
                         const double* bound, double* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Tuning (Sec. 4.3: search over tile sizes and unroll factors)              */

typedef enum {
    MLK_OP_MATMUL = 0,
    MLK_OP_CONV2D = 1,
    MLK_OP_BATCHED = 2
} mlk_op;

typedef struct {
    int32_t op;             /* mlk_op */
    int32_t in, out;        /* mlk_dtype pair */
    int32_t accumulate;
    int64_t M, N, K;        /* MLK_OP_MATMUL */
    int64_t n, c, h, w, f, kh, kw; /* MLK_OP_CONV2D */
    int32_t sh, sw, ph, pw;
    int64_t count;          /* MLK_OP_BATCHED: count host descriptors */
    const mlk_gemm_desc* descs;
} mlk_problem;

typedef enum {
    MLK_TUNE_EXHAUSTIVE = 0, /* measure every legal configuration */
    MLK_TUNE_RANDOM = 1,     /* measure a uniform random sample of the budget */
    MLK_TUNE_MODEL = 2,      /* rank all by the cost model, measure the top budget */
    MLK_TUNE_ES = 3          /* (1+1) evolution strategy over the configuration's
                                fields: mutate the best so far, keep the child if it
                                is faster, adapt the mutation strength by the 1/5
                                success rule; stops at the budget */
} mlk_tune_strategy;

typedef struct mlk_cost_model mlk_cost_model; /* opaque, see mlk_model_* */

typedef struct {
    int32_t strategy;       /* mlk_tune_strategy */
    double budget_frac;     /* RANDOM / MODEL / ES: measure ceil(budget_frac * n_legal) configs */
    int32_t reps;           /* timed runs per configuration (median taken); 0 = 20 */
    int32_t warmup;         /* untimed runs first; 0 = 3 */
    uint64_t seed;          /* RANDOM / ES seed; also seeds the scratch inputs */
    const char* db_path;    /* NULL = no database; else JSON-lines file, appended */
    int32_t use_db;         /* 1: if the database holds this problem, return it unmeasured */
    mlk_cost_model* model;  /* MLK_TUNE_MODEL: the trained model (else ignored) */
    double* times_us;       /* optional HOST array [mlk_config_count]: median time per
                               legal config in enumeration order, -1 if not measured */
    int32_t fake_timer;     /* 1: replace GPU timing by a deterministic analytic cost
                               (host-only; for testing the search logic) */
    const double* table_us; /* optional HOST array [mlk_config_count]: times to use
                               instead of measuring (<= 0: the configuration fails),
                               for replaying a strategy offline on a measured table;
                               host-only, like fake_timer (which it overrides) */
} mlk_tune_opts;

typedef struct {
    int32_t n_legal;        /* size of the legal configuration space */
    int32_t n_measured;     /* configurations timed in this call */
    int32_t best_index;     /* enumeration index of the returned config */
    int32_t from_db;        /* 1 if answered from the database */
    double best_us;         /* median time of the returned config */
} mlk_tune_report;

/*
 * Search the legal tile configurations of problem p and return the fastest
 * found in *best.  Scratch inputs are allocated by the library (seeded, the
 * caller's buffers are never touched; for MLK_OP_BATCHED the descriptors'
 * shapes are used, not their pointers).  Synchronises the device.
 * A configuration within 1% of the fastest counts as tied; ties go to the
 * smaller LDS footprint, then the lower enumeration index.
 */
mlk_status mlk_tune(const mlk_problem* p, const mlk_tune_opts* o, mlk_tile_config* best,
                    mlk_tune_report* rep);

/* MLK_OK if cfg is legal for p (pure host check, no GPU), else MLK_ERR_CONFIG
 * with the reason in mlk_last_error(). */
mlk_status mlk_config_legal(const mlk_problem* p, const mlk_tile_config* cfg);

/* Number of legal configurations for p (>= 1 for a valid problem; < 0 on
 * an invalid problem), and the i-th in enumeration order. */
int32_t mlk_config_count(const mlk_problem* p);
mlk_status mlk_config_get(const mlk_problem* p, int32_t i, mlk_tile_config* cfg);

/* Record cfg as the tuned choice for p in the in-memory table consulted when
 * a launch gets cfg == NULL (mlk_tune does this for a measured result; its
 * table_us and fake_timer replays leave the table alone). */
mlk_status mlk_config_set_default(const mlk_problem* p, const mlk_tile_config* cfg);

/* ------------------------------------------------------------------------ */
/* Learned cost model: MLPs  features(problem, config) -> log(time in us),
 * trained on the GPU by the library's own forward / backward / Adam kernels.
 * A model holds three networks of the same shape, initialised and trained
 * from different seeds on the same samples; its prediction is the mean of
 * their log-time predictions. */

/* Feature vector length and the features of (p, cfg) (host computation). */
int32_t mlk_model_feature_count(void);
mlk_status mlk_model_features(const mlk_problem* p, const mlk_tile_config* cfg, float* out);

/* hidden: width of both hidden layers of each network (1..256).  Weights
 * are initialised on the host from `seed` and uploaded; the model owns
 * device buffers. */
mlk_status mlk_model_create(int32_t hidden, uint64_t seed, mlk_cost_model** out);
void mlk_model_destroy(mlk_cost_model* m);
/* Add one training sample (a measured median time, microseconds > 0). */
mlk_status mlk_model_add_sample(mlk_cost_model* m, const mlk_problem* p,
                                const mlk_tile_config* cfg, double time_us);
int64_t mlk_model_sample_count(const mlk_cost_model* m);
/* Normalise features over the current samples, then run `epochs` passes of
 * minibatch Adam (batch rows, learning rate lr) on the GPU for each network.
 * *final_loss (may be NULL) receives the networks' mean full-batch squared
 * error in normalised log space. */
mlk_status mlk_model_train(mlk_cost_model* m, int32_t epochs, int32_t batch, float lr,
                           float* final_loss);
/* Predicted time (microseconds) of n configurations of p (host arrays). */
mlk_status mlk_model_predict(mlk_cost_model* m, const mlk_problem* p,
                             const mlk_tile_config* cfgs, int32_t n, float* pred_us);

/*
 * The cost model's network kernels, exposed so their arithmetic can be
 * checked: layers D0 -> H1 -> H2 -> 1, ReLU after both hidden layers, one
 * flat fp32 parameter vector laid out W1 (D0 x H1 row-major), b1 (H1),
 * W2 (H1 x H2), b2 (H2), W3 (H2), b3 (1).  All pointers device.
 *   mlk_mlp_forward:   y[B] = net(X[B x D0])
 *   mlk_mlp_loss_grad: loss[0] = mean_r (net(X_r) - t_r)^2, grad = d loss / d params
 *   mlk_adam_step:     Adam (Kingma & Ba) with bias correction at step t >= 1
 */
mlk_status mlk_mlp_forward(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* params,
                           const float* X, float* y, void* stream);
mlk_status mlk_mlp_loss_grad(int64_t B, int64_t D0, int64_t H1, int64_t H2,
                             const float* params, const float* X, const float* t, float* grad,
                             float* loss, void* stream);
mlk_status mlk_adam_step(int64_t n, float* params, const float* grad, float* m, float* v,
                         float lr, float beta1, float beta2, float eps, int64_t t, void* stream);

/* ------------------------------------------------------------------------ */

const char* mlk_status_str(mlk_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char* mlk_last_error(void);
/* Library version string. */
const char* mlk_version(void);
/* Free every library-owned workspace, cached graph and table. */
void mlk_release(void);

#ifdef __cplusplus
}
#endif
#endif /* MLK_H */
