/*
 * oracle.c -- plain, slow, CPU reference for the dense kernels of
 * "nelli: A lightweight frontend for MLIR" (arXiv 2307.16080).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Every routine here is the plain definition of what the paper's kernels
 * compute, written as the loop nest the paper prints, with no blocking, no
 * fusion and no reordering:
 *
 *   matmul   Sec. 1 (Introduction), listing "nelli_for_to_affine_for" (affine i/j/k nest,
 *            load a, load b, load c, mulf, addf, store) and Sec. 2.1 (MLIR), listing
 *            "linalg-matmul" (linalg.generic with maps (d0,d2),(d2,d1),
 *            (d0,d1), iterators parallel/parallel/reduction, body mulf then
 *            addf into the output).  Naming here: C[M,N] += A[M,K] * B[K,N].
 *   linear   Sec. 2.1 (MLIR), listing "listing1" (torch.nn.Linear lowered to
 *            scf loops): the matmul nest into a zeroed buffer, then a
 *            separate nest adding bias[j] to every row.
 *   conv2d   Sec. 4.1 (End-to-end GPU), listing "2dnchwconv": output[n,co,ho,wo] +=
 *            input[n,ci,ho+ki,wo+kj] * kernel[co,ci,ki,kj]; outer four loops
 *            parallel, ci/ki/kj sequential in that order.  Generalised to
 *            stride s and symmetric zero padding p (reading: ih = oh*s - p +
 *            kh, taps outside the image contribute zero, no filter flip).
 *
 * Precisions:
 *   *_f64    inputs converted exactly to double, accumulated in double.  This
 *            is the reference ("REF64") every error figure is measured
 *            against.
 *   *_f32    float accumulator, product rounded then sum rounded (mulf then
 *            addf, the literal IR body).  Built with -ffp-contract=off so the
 *            two roundings stay separate.  Informational only.
 *   *_i8     int8 operands sign-extended, products and sums in uint32, so the
 *            int32 result wraps exactly like two's complement hardware.
 *
 * Number formats (not in the paper; the extension to bf16 / fp8):
 *   bf16     IEEE-754 binary32 with 16 low mantissa bits dropped; encode is
 *            round-to-nearest-even, decode is exact.
 *   e4m3     OCP 8-bit floating point, E4M3 variant: bias 7, no infinities,
 *            S.1111.111 is NaN, largest finite 448.  Encode rounds to the
 *            nearest representable value (ties to even mantissa) and
 *            saturates to +-448.
 *
 * Small multi-layer perceptron (the learned cost model): forward, mean
 * squared error, back-propagation and the Adam update of Kingma & Ba (2015),
 * all in double.
 *
 * Threads: routines taking `threads` split their outermost parallel loop over
 * that many POSIX threads; each output element is still computed by one
 * thread in the plain order, so results do not depend on `threads`.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* a tiny row-range thread pool: run fn(lo, hi, ctx) over [0, n)              */

typedef void (*range_fn)(int64_t lo, int64_t hi, void* ctx);

struct range_job {
    range_fn fn;
    void* ctx;
    int64_t lo, hi;
};

static void* range_thread(void* p) {
    struct range_job* j = (struct range_job*)p;
    j->fn(j->lo, j->hi, j->ctx);
    return NULL;
}

static void parallel_range(int64_t n, int threads, range_fn fn, void* ctx) {
    if (threads <= 1 || n <= 1) {
        fn(0, n, ctx);
        return;
    }
    if (threads > 256) threads = 256;
    if (threads > n) threads = (int)n;
    pthread_t tid[256];
    struct range_job jobs[256];
    int started = 0;
    for (int t = 0; t < threads; ++t) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].lo = n * t / threads;
        jobs[t].hi = n * (t + 1) / threads;
        if (pthread_create(&tid[t], NULL, range_thread, &jobs[t]) == 0) {
            started = t + 1;
        } else {
            /* could not start: run the remaining ranges here */
            for (int u = t; u < threads; ++u) {
                jobs[u].fn = fn;
                jobs[u].ctx = ctx;
                jobs[u].lo = n * u / threads;
                jobs[u].hi = n * (u + 1) / threads;
                fn(jobs[u].lo, jobs[u].hi, ctx);
            }
            break;
        }
    }
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
}

/* ------------------------------------------------------------------------ */
/* matmul                                                                    */

struct mm_f64 {
    int64_t N, K, lda, ldb, ldc;
    const double *A, *B;
    double* C;
};

/* The loop order is the paper's affine nest: row i, then the contraction
 * index, then the output column.  For every output element the terms are
 * added in ascending contraction order, exactly as a reduction-innermost nest
 * would add them. */
static void mm_f64_rows(int64_t lo, int64_t hi, void* p) {
    struct mm_f64* a = (struct mm_f64*)p;
    for (int64_t i = lo; i < hi; ++i)
        for (int64_t k = 0; k < a->K; ++k) {
            const double aik = a->A[i * a->lda + k];
            for (int64_t j = 0; j < a->N; ++j)
                a->C[i * a->ldc + j] = a->C[i * a->ldc + j] + aik * a->B[k * a->ldb + j];
        }
}

/* C[i,j] += sum_k A[i,k] * B[k,j], everything in double (REF64). */
void orc_matmul_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double* C, int64_t ldc, int threads) {
    struct mm_f64 a = {N, K, lda, ldb, ldc, A, B, C};
    parallel_range(M, threads, mm_f64_rows, &a);
}

/* The bias nest of the Linear layer (Sec. 2.1, listing "listing1": after the
 * product nest into a zeroed buffer, a second i/j nest loads the product and
 * bias[j], adds them and stores): C[i,j] = C[i,j] + bias[j], in double. */
void orc_bias_rows_f64(int64_t M, int64_t N, const double* bias, double* C, int64_t ldc) {
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) C[i * ldc + j] = C[i * ldc + j] + bias[j];
}

/* C[i,j] = (C[i,j] + (A[i,k] * B[k,j])) in float, one rounding after the
 * product and one after the sum, k ascending (the literal mulf / addf body). */
void orc_matmul_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                    const float* B, int64_t ldb, float* C, int64_t ldc) {
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j)
            for (int64_t k = 0; k < K; ++k) {
                float a = A[i * lda + k];
                float b = B[k * ldb + j];
                float c = C[i * ldc + j];
                float d = a * b;
                float e = c + d;
                C[i * ldc + j] = e;
            }
}

struct mm_i8 {
    int64_t N, K, lda, ldb, ldc;
    const int8_t *A, *B;
    int32_t* C;
};

static void mm_i8_rows(int64_t lo, int64_t hi, void* p) {
    struct mm_i8* a = (struct mm_i8*)p;
    for (int64_t i = lo; i < hi; ++i)
        for (int64_t j = 0; j < a->N; ++j) {
            uint32_t c = (uint32_t)a->C[i * a->ldc + j];
            for (int64_t k = 0; k < a->K; ++k) {
                int32_t x = (int32_t)a->A[i * a->lda + k]; /* sign extension */
                int32_t y = (int32_t)a->B[k * a->ldb + j];
                c = c + (uint32_t)x * (uint32_t)y; /* wraps modulo 2^32 */
            }
            a->C[i * a->ldc + j] = (int32_t)c;
        }
}

/* C[i,j] += sext(A[i,k]) * sext(B[k,j]) with int32 wrap-around. */
void orc_matmul_i8(int64_t M, int64_t N, int64_t K, const int8_t* A, int64_t lda,
                   const int8_t* B, int64_t ldb, int32_t* C, int64_t ldc, int threads) {
    struct mm_i8 a = {N, K, lda, ldb, ldc, A, B, C};
    parallel_range(M, threads, mm_i8_rows, &a);
}

/* ------------------------------------------------------------------------ */
/* conv2d, NCHW input, FCHW filter, NFHW output                              */

int64_t orc_conv_out_size(int64_t in, int64_t k, int64_t stride, int64_t pad) {
    /* floor((in + 2 pad - k) / stride) + 1; zero when the window never fits */
    int64_t span = in + 2 * pad - k;
    if (span < 0 || stride <= 0) return 0;
    return span / stride + 1;
}

struct conv_f64 {
    int64_t N, C, H, W, F, KH, KW, sh, sw, ph, pw, HO, WO;
    const double *x, *w;
    double* y;
};

static void conv_f64_range(int64_t lo, int64_t hi, void* p) {
    struct conv_f64* a = (struct conv_f64*)p;
    /* the parallel index runs over (n, f) pairs */
    for (int64_t nf = lo; nf < hi; ++nf) {
        int64_t n = nf / a->F, f = nf % a->F;
        for (int64_t oh = 0; oh < a->HO; ++oh)
            for (int64_t ow = 0; ow < a->WO; ++ow) {
                double acc = a->y[((n * a->F + f) * a->HO + oh) * a->WO + ow];
                for (int64_t c = 0; c < a->C; ++c)
                    for (int64_t kh = 0; kh < a->KH; ++kh)
                        for (int64_t kw = 0; kw < a->KW; ++kw) {
                            int64_t ih = oh * a->sh - a->ph + kh;
                            int64_t iw = ow * a->sw - a->pw + kw;
                            if (ih < 0 || ih >= a->H || iw < 0 || iw >= a->W) continue;
                            double inp = a->x[((n * a->C + c) * a->H + ih) * a->W + iw];
                            double ker = a->w[((f * a->C + c) * a->KH + kh) * a->KW + kw];
                            acc = acc + inp * ker;
                        }
                a->y[((n * a->F + f) * a->HO + oh) * a->WO + ow] = acc;
            }
    }
}

/* y[n,f,oh,ow] += sum_{c,kh,kw} x_pad[n,c,oh*sh+kh,ow*sw+kw] * w[f,c,kh,kw]
 * in double; x_pad is x surrounded by ph rows / pw columns of zeros. */
void orc_conv2d_f64(int64_t N, int64_t C, int64_t H, int64_t W, int64_t F, int64_t KH,
                    int64_t KW, int64_t sh, int64_t sw, int64_t ph, int64_t pw,
                    const double* x, const double* w, double* y, int threads) {
    struct conv_f64 a;
    a.N = N; a.C = C; a.H = H; a.W = W; a.F = F; a.KH = KH; a.KW = KW;
    a.sh = sh; a.sw = sw; a.ph = ph; a.pw = pw;
    a.HO = orc_conv_out_size(H, KH, sh, ph);
    a.WO = orc_conv_out_size(W, KW, sw, pw);
    a.x = x; a.w = w; a.y = y;
    parallel_range(N * F, threads, conv_f64_range, &a);
}

/* The same nest in float: product rounded, then sum rounded. */
void orc_conv2d_f32(int64_t N, int64_t C, int64_t H, int64_t W, int64_t F, int64_t KH,
                    int64_t KW, int64_t sh, int64_t sw, int64_t ph, int64_t pw,
                    const float* x, const float* w, float* y) {
    int64_t HO = orc_conv_out_size(H, KH, sh, ph), WO = orc_conv_out_size(W, KW, sw, pw);
    for (int64_t n = 0; n < N; ++n)
        for (int64_t f = 0; f < F; ++f)
            for (int64_t oh = 0; oh < HO; ++oh)
                for (int64_t ow = 0; ow < WO; ++ow)
                    for (int64_t c = 0; c < C; ++c)
                        for (int64_t kh = 0; kh < KH; ++kh)
                            for (int64_t kw = 0; kw < KW; ++kw) {
                                int64_t ih = oh * sh - ph + kh, iw = ow * sw - pw + kw;
                                if (ih < 0 || ih >= H || iw < 0 || iw >= W) continue;
                                float inp = x[((n * C + c) * H + ih) * W + iw];
                                float ker = w[((f * C + c) * KH + kh) * KW + kw];
                                float d = inp * ker;
                                float* o = &y[((n * F + f) * HO + oh) * WO + ow];
                                *o = *o + d;
                            }
}

/* im2col: col[(c*KH + kh)*KW + kw][(n*HO + oh)*WO + ow] = x_pad[n, c, oh*sh+kh,
 * ow*sw+kw].  With it the convolution is the matmul W[F, C*KH*KW] * col,
 * scattered back as y[n, f, oh, ow]; the tests use this as a second,
 * independent route to the convolution. */
void orc_im2col_f64(int64_t N, int64_t C, int64_t H, int64_t W, int64_t KH, int64_t KW,
                    int64_t sh, int64_t sw, int64_t ph, int64_t pw, const double* x,
                    double* col) {
    int64_t HO = orc_conv_out_size(H, KH, sh, ph), WO = orc_conv_out_size(W, KW, sw, pw);
    int64_t P = N * HO * WO;
    for (int64_t c = 0; c < C; ++c)
        for (int64_t kh = 0; kh < KH; ++kh)
            for (int64_t kw = 0; kw < KW; ++kw) {
                int64_t r = (c * KH + kh) * KW + kw;
                for (int64_t n = 0; n < N; ++n)
                    for (int64_t oh = 0; oh < HO; ++oh)
                        for (int64_t ow = 0; ow < WO; ++ow) {
                            int64_t ih = oh * sh - ph + kh, iw = ow * sw - pw + kw;
                            double v = 0.0;
                            if (ih >= 0 && ih < H && iw >= 0 && iw < W)
                                v = x[((n * C + c) * H + ih) * W + iw];
                            col[r * P + (n * HO + oh) * WO + ow] = v;
                        }
            }
}

/* ------------------------------------------------------------------------ */
/* number formats                                                            */

static uint32_t f32_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* bf16 code -> exact value: sign, 8-bit exponent (bias 127), 7-bit fraction. */
double orc_bf16_value(uint16_t code) {
    int s = (code >> 15) & 1;
    int e = (code >> 7) & 0xFF;
    int m = code & 0x7F;
    double v;
    if (e == 0xFF) v = (m == 0) ? INFINITY : NAN;
    else if (e == 0) v = ldexp((double)m, -126 - 7);     /* subnormal */
    else v = ldexp(1.0 + (double)m / 128.0, e - 127);
    return s ? -v : v;
}

void orc_bf16_decode(int64_t n, const uint16_t* codes, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_bf16_value(codes[i]);
}

/* float -> bf16, round to nearest, ties to the code with an even last bit.
 * The two candidates are the bf16 values just below and just above |x| in
 * magnitude; the nearer one is chosen by comparing exact distances in double. */
uint16_t orc_bf16_from_float(float x) {
    uint32_t u = f32_bits(x);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000);
    if (isnan(x)) return (uint16_t)(sign | 0x7FC0);
    if (isinf(x)) return (uint16_t)(sign | 0x7F80);
    double ax = fabs((double)x);
    /* lower candidate: the largest bf16 magnitude <= ax, i.e. |x| with its
     * 16 low fraction bits cleared */
    uint16_t lo_code = (uint16_t)((u & 0x7FFFFFFFu) >> 16);
    double lo = orc_bf16_value(lo_code);
    if (lo == ax) return (uint16_t)(sign | lo_code);
    uint16_t hi_code = (uint16_t)(lo_code + 1); /* next magnitude up (may be inf) */
    /* Past the largest finite value the upper neighbour is infinity; IEEE
     * rounding measures the distance to it as if the exponent range went on,
     * i.e. to 2^128. */
    double hi = (hi_code == 0x7F80) ? ldexp(1.0, 128) : orc_bf16_value(hi_code);
    double dlo = ax - lo, dhi = hi - ax;
    uint16_t pick;
    if (dlo < dhi) pick = lo_code;
    else if (dhi < dlo) pick = hi_code;
    else pick = (lo_code & 1) ? hi_code : lo_code;
    return (uint16_t)(sign | pick);
}

void orc_bf16_encode(int64_t n, const float* x, uint16_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_bf16_from_float(x[i]);
}

/* OCP E4M3 code -> exact value. */
double orc_e4m3_value(uint8_t code) {
    int s = (code >> 7) & 1;
    int e = (code >> 3) & 0xF;
    int m = code & 0x7;
    double v;
    if (e == 0xF && m == 0x7) v = NAN;
    else if (e == 0) v = ldexp((double)m, -6 - 3);       /* subnormal: m/8 * 2^-6 */
    else v = ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

void orc_e4m3_decode(int64_t n, const uint8_t* codes, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = orc_e4m3_value(codes[i]);
}

/* value -> nearest E4M3 code by exhaustive search over the 127 finite
 * non-negative codes; ties go to the code whose mantissa is even; magnitudes
 * beyond 448 saturate to 448; NaN maps to 0x7F. */
uint8_t orc_e4m3_from_float(float v) {
    if (isnan(v)) return 0x7F;
    uint8_t sign = signbit(v) ? 0x80 : 0x00;
    double a = fabs((double)v);
    if (a >= 448.0) return (uint8_t)(sign | 0x7E);
    int best = 0;
    double bestd = INFINITY;
    for (int c = 0; c <= 0x7E; ++c) {
        double d = fabs(orc_e4m3_value((uint8_t)c) - a);
        if (d < bestd || (d == bestd && (c & 1) == 0 && (best & 1) == 1)) {
            best = c;
            bestd = d;
        }
    }
    return (uint8_t)(sign | best);
}

/* Per-tensor scaling: scale = amax / 448 rounded to float (1 when amax is 0);
 * code = e4m3(round_to_float(x / scale)); value = code * scale. */
float orc_e4m3_scale(float amax) {
    if (!(amax > 0.0f) || isinf(amax)) return 1.0f;
    return (float)((double)amax / 448.0);
}

void orc_e4m3_encode(int64_t n, const float* x, float scale, uint8_t* out) {
    for (int64_t i = 0; i < n; ++i) {
        /* one float division, rounded to nearest: computing the quotient in
         * double and rounding once to float gives that same float */
        float q = (float)((double)x[i] / (double)scale);
        out[i] = orc_e4m3_from_float(q);
    }
}

/* max |x_i| over the array (0 for an empty array); NaNs are ignored. */
float orc_amax(int64_t n, const float* x) {
    float m = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        float a = fabsf(x[i]);
        if (a > m) m = a;
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* error metrics against a REF64 result                                      */

/* out[0] = sum (c - r)^2, out[1] = sum r^2, out[2] = max |c - r|,
 * out[3] = max |c - r| / bound_i over elements whose bound is > 0
 * (bound may be NULL, then out[3] = 0). */
void orc_err_stats(int64_t n, const double* c, const double* r, const double* bound,
                   double* out) {
    double s2 = 0.0, r2 = 0.0, mx = 0.0, ratio = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = c[i] - r[i];
        s2 += d * d;
        r2 += r[i] * r[i];
        if (fabs(d) > mx) mx = fabs(d);
        if (bound && bound[i] > 0.0) {
            double q = fabs(d) / bound[i];
            if (q > ratio) ratio = q;
        }
    }
    out[0] = s2;
    out[1] = r2;
    out[2] = mx;
    out[3] = ratio;
}

/* ------------------------------------------------------------------------ */
/* multi-layer perceptron: x[D0] -> relu(x W1 + b1)[H1] -> relu(. W2 + b2)[H2]
 * -> (. W3 + b3)[1].  Parameters live in one flat vector in the order
 * W1 (D0 x H1, row-major), b1 (H1), W2 (H1 x H2), b2 (H2), W3 (H2 x 1), b3 (1). */

int64_t orc_mlp_param_count(int64_t D0, int64_t H1, int64_t H2) {
    return D0 * H1 + H1 + H1 * H2 + H2 + H2 + 1;
}

/* Forward pass for B rows of X (B x D0, row-major); writes y (B). */
void orc_mlp_forward(int64_t B, int64_t D0, int64_t H1, int64_t H2, const double* p,
                     const double* X, double* y) {
    const double* W1 = p;
    const double* b1 = W1 + D0 * H1;
    const double* W2 = b1 + H1;
    const double* b2 = W2 + H1 * H2;
    const double* W3 = b2 + H2;
    const double* b3 = W3 + H2;
    double* h1 = (double*)malloc(sizeof(double) * (size_t)(H1 + H2));
    double* h2 = h1 + H1;
    for (int64_t r = 0; r < B; ++r) {
        const double* x = X + r * D0;
        for (int64_t j = 0; j < H1; ++j) {
            double s = b1[j];
            for (int64_t i = 0; i < D0; ++i) s += x[i] * W1[i * H1 + j];
            h1[j] = s > 0.0 ? s : 0.0;
        }
        for (int64_t j = 0; j < H2; ++j) {
            double s = b2[j];
            for (int64_t i = 0; i < H1; ++i) s += h1[i] * W2[i * H2 + j];
            h2[j] = s > 0.0 ? s : 0.0;
        }
        double s = b3[0];
        for (int64_t i = 0; i < H2; ++i) s += h2[i] * W3[i];
        y[r] = s;
    }
    free(h1);
}

/* Loss L = (1/B) sum_r (y_r - t_r)^2 and its gradient dL/dp (same layout as
 * p) by back-propagation.  Returns L.  A ReLU's derivative at exactly 0 is
 * taken as 0. */
double orc_mlp_loss_grad(int64_t B, int64_t D0, int64_t H1, int64_t H2, const double* p,
                         const double* X, const double* t, double* g) {
    const double* W1 = p;
    const double* b1 = W1 + D0 * H1;
    const double* W2 = b1 + H1;
    const double* b2 = W2 + H1 * H2;
    const double* W3 = b2 + H2;
    const double* b3 = W3 + H2;
    int64_t P = orc_mlp_param_count(D0, H1, H2);
    for (int64_t i = 0; i < P; ++i) g[i] = 0.0;
    double* gW1 = g;
    double* gb1 = gW1 + D0 * H1;
    double* gW2 = gb1 + H1;
    double* gb2 = gW2 + H1 * H2;
    double* gW3 = gb2 + H2;
    double* gb3 = gW3 + H2;
    double* buf = (double*)malloc(sizeof(double) * (size_t)(2 * H1 + 2 * H2));
    double *z1 = buf, *z2 = buf + H1, *d1 = buf + H1 + H2, *d2 = buf + 2 * H1 + H2;
    double loss = 0.0;
    for (int64_t r = 0; r < B; ++r) {
        const double* x = X + r * D0;
        for (int64_t j = 0; j < H1; ++j) {
            double s = b1[j];
            for (int64_t i = 0; i < D0; ++i) s += x[i] * W1[i * H1 + j];
            z1[j] = s;
        }
        for (int64_t j = 0; j < H2; ++j) {
            double s = b2[j];
            for (int64_t i = 0; i < H1; ++i) s += (z1[i] > 0.0 ? z1[i] : 0.0) * W2[i * H2 + j];
            z2[j] = s;
        }
        double y = b3[0];
        for (int64_t i = 0; i < H2; ++i) y += (z2[i] > 0.0 ? z2[i] : 0.0) * W3[i];
        double e = y - t[r];
        loss += e * e;
        double dy = 2.0 * e / (double)B; /* dL/dy_r */
        /* output layer */
        gb3[0] += dy;
        for (int64_t i = 0; i < H2; ++i) {
            double a2 = z2[i] > 0.0 ? z2[i] : 0.0;
            gW3[i] += a2 * dy;
            d2[i] = (z2[i] > 0.0) ? W3[i] * dy : 0.0; /* dL/dz2 */
        }
        /* second hidden layer */
        for (int64_t i = 0; i < H1; ++i) {
            double a1 = z1[i] > 0.0 ? z1[i] : 0.0;
            double s = 0.0;
            for (int64_t j = 0; j < H2; ++j) {
                gW2[i * H2 + j] += a1 * d2[j];
                s += W2[i * H2 + j] * d2[j];
            }
            d1[i] = (z1[i] > 0.0) ? s : 0.0; /* dL/dz1 */
        }
        for (int64_t j = 0; j < H2; ++j) gb2[j] += d2[j];
        /* first layer */
        for (int64_t i = 0; i < D0; ++i)
            for (int64_t j = 0; j < H1; ++j) gW1[i * H1 + j] += x[i] * d1[j];
        for (int64_t j = 0; j < H1; ++j) gb1[j] += d1[j];
    }
    free(buf);
    return loss / (double)B;
}

/* One Adam step (Kingma & Ba 2015, Algorithm 1) at step number t >= 1:
 *   m = b1 m + (1 - b1) g;   v = b2 v + (1 - b2) g^2
 *   mhat = m / (1 - b1^t);   vhat = v / (1 - b2^t)
 *   p = p - lr * mhat / (sqrt(vhat) + eps)                                  */
void orc_adam_step(int64_t n, double* p, const double* g, double* m, double* v, double lr,
                   double b1, double b2, double eps, int64_t t) {
    double c1 = 1.0 - pow(b1, (double)t);
    double c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        p[i] = p[i] - lr * mh / (sqrt(vh) + eps);
    }
}
