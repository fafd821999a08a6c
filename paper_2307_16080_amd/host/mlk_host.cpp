// mlk_host.cpp -- the OpenMP host kernels (include/mlk_host.h): linalg.matmul
// and linalg.conv_2d_nchw_fchw in fp32 with the parallel output loops as
// OpenMP worksharing loops (the paper's CPU lowering, Sec. 4.2) and a tiling /
// unroll factor chosen by measured search (Sec. 4.3).
//
// Matmul: each work item is an mb x nb block of C; it walks K in kb-deep slabs
// and, per k, streams one row slice of B into `unroll` rows of C at once
// (register blocking over rows: each loaded B element feeds U fused
// multiply-adds).  The nb-wide inner loop is left to the compiler's vectoriser.
// Conv: each work item is (image, block of mb filters, output row); per input
// channel and filter tap the input row slice is loaded once and feeds
// `unroll` filters' output rows.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/mlk_host.h"

namespace {

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- matmul

template <int U>
void mm_block(int64_t i0, int64_t i1, int64_t j0, int64_t j1, int64_t K, int64_t kb, const float* A, int64_t lda,
              const float* B, int64_t ldb, float* C, int64_t ldc) {
    const int64_t nj = j1 - j0;
    for (int64_t k0 = 0; k0 < K; k0 += kb) {
        const int64_t k1 = std::min(K, k0 + kb);
        int64_t i = i0;
        for (; i + U <= i1; i += U) {
            float* c[U];
            const float* a[U];
            for (int u = 0; u < U; ++u) {
                c[u] = C + (i + u) * ldc + j0;
                a[u] = A + (i + u) * lda;
            }
            for (int64_t k = k0; k < k1; ++k) {
                const float* b = B + k * ldb + j0;
                float av[U];
                for (int u = 0; u < U; ++u) av[u] = a[u][k];
#pragma omp simd
                for (int64_t j = 0; j < nj; ++j) {
                    const float bj = b[j];
                    for (int u = 0; u < U; ++u) c[u][j] += av[u] * bj;
                }
            }
        }
        for (; i < i1; ++i) {  // rows left over by the unroll
            float* c = C + i * ldc + j0;
            for (int64_t k = k0; k < k1; ++k) {
                const float av = A[i * lda + k];
                const float* b = B + k * ldb + j0;
#pragma omp simd
                for (int64_t j = 0; j < nj; ++j) c[j] += av * b[j];
            }
        }
    }
}

typedef void (*mm_fn)(int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, const float*, int64_t, const float*,
                      int64_t, float*, int64_t);

mm_fn mm_kernel(int u) {
    switch (u) {
        case 1: return mm_block<1>;
        case 2: return mm_block<2>;
        case 4: return mm_block<4>;
        case 8: return mm_block<8>;
        default: return nullptr;
    }
}

// ---------------------------------------------------------------- conv

// output row oh of filters f0 .. f0+U-1 of image n
template <int U>
void conv_row(int64_t n, int64_t f0, int64_t oh, int64_t C, int64_t H, int64_t W, int64_t F, int64_t KH, int64_t KW,
              int sh, int sw, int ph, int pw, int64_t HO, int64_t WO, const float* x, const float* w, float* y) {
    float* yr[U];
    for (int u = 0; u < U; ++u) yr[u] = y + ((n * F + f0 + u) * HO + oh) * WO;
    // output columns whose whole window is inside the image in w (no bounds test)
    const int64_t lo = std::min<int64_t>(WO, std::max<int64_t>(0, cdiv(pw, sw)));
    const int64_t hi = std::max<int64_t>(lo, std::min<int64_t>(WO, (W - KW + pw) / sw + 1));
    for (int64_t c = 0; c < C; ++c) {
        const float* xc = x + (n * C + c) * H * W;
        for (int64_t kh = 0; kh < KH; ++kh) {
            const int64_t ih = oh * sh - ph + kh;
            if (ih < 0 || ih >= H) continue;
            const float* xr = xc + ih * W;
            for (int64_t kw = 0; kw < KW; ++kw) {
                float wv[U];
                for (int u = 0; u < U; ++u) wv[u] = w[(((f0 + u) * C + c) * KH + kh) * KW + kw];
                const int64_t off = kw - pw;
                for (int64_t ow = 0; ow < lo; ++ow) {
                    const int64_t iw = ow * sw + off;
                    if (iw < 0 || iw >= W) continue;
                    for (int u = 0; u < U; ++u) yr[u][ow] += wv[u] * xr[iw];
                }
                if (sw == 1) {
                    const float* xs = xr + off;
#pragma omp simd
                    for (int64_t ow = lo; ow < hi; ++ow)
                        for (int u = 0; u < U; ++u) yr[u][ow] += wv[u] * xs[ow];
                } else {
                    for (int64_t ow = lo; ow < hi; ++ow) {
                        const float xv = xr[ow * sw + off];
                        for (int u = 0; u < U; ++u) yr[u][ow] += wv[u] * xv;
                    }
                }
                for (int64_t ow = hi; ow < WO; ++ow) {
                    const int64_t iw = ow * sw + off;
                    if (iw < 0 || iw >= W) continue;
                    for (int u = 0; u < U; ++u) yr[u][ow] += wv[u] * xr[iw];
                }
            }
        }
    }
}

typedef void (*conv_fn)(int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int, int,
                        int, int, int64_t, int64_t, const float*, const float*, float*);

conv_fn conv_kernel(int u) {
    switch (u) {
        case 1: return conv_row<1>;
        case 2: return conv_row<2>;
        case 4: return conv_row<4>;
        case 8: return conv_row<8>;
        default: return nullptr;
    }
}

bool unroll_ok(int u) { return u == 1 || u == 2 || u == 4 || u == 8; }

int threads_of(const mlkh_config& c) { return c.threads > 0 ? c.threads : omp_get_max_threads(); }

mlkh_config default_mm(int64_t M, int64_t N) {
    (void)M;
    return mlkh_config{64, (int32_t)std::min<int64_t>(std::max<int64_t>(N, 1), 256), 256, 4, 0};
}
mlkh_config default_conv() { return mlkh_config{8, 0, 0, 4, 0}; }

int64_t conv_out(int64_t in, int64_t k, int64_t s, int64_t p) {
    const int64_t span = in + 2 * p - k;
    return span < 0 || s <= 0 ? 0 : span / s + 1;
}

// ---------------------------------------------------------------- search space

std::vector<mlkh_config> space(int32_t op, const int64_t* d) {
    std::vector<mlkh_config> v;
    const int32_t nt = omp_get_max_threads();
    std::vector<int32_t> thr{nt};
    if (nt >= 4) thr.push_back(nt / 2);
    if (op == 0) {
        const int64_t M = d[0], N = d[1], K = d[2];
        for (int32_t mb : {16, 32, 64, 128})
            for (int32_t nb : {64, 128, 256, 512}) {
                if (mb > 2 * std::max<int64_t>(M, 8) || nb > 2 * std::max<int64_t>(N, 32)) continue;
                for (int32_t kb : {64, 256, 1024}) {
                    if (kb > 2 * std::max<int64_t>(K, 32)) continue;
                    for (int32_t u : {1, 2, 4, 8})
                        if (u <= mb)
                            for (int32_t t : thr) v.push_back(mlkh_config{mb, nb, kb, u, t});
                }
            }
    } else {
        const int64_t F = d[4];
        for (int32_t fb : {1, 2, 4, 8, 16, 32})
            for (int32_t u : {1, 2, 4, 8}) {
                if (u > fb || fb > 2 * std::max<int64_t>(F, 1)) continue;
                for (int32_t t : thr) v.push_back(mlkh_config{fb, 0, 0, u, t});
            }
    }
    if (v.empty()) v.push_back(op == 0 ? default_mm(d[0], d[1]) : default_conv());
    return v;
}

int check_cfg(int32_t op, const mlkh_config& c) {
    if (!unroll_ok(c.unroll) || c.mb < 1 || c.threads < 0) return MLKH_ERR_CONFIG;
    if (op == 0 && (c.nb < 1 || c.kb < 1)) return MLKH_ERR_CONFIG;
    if (c.unroll > c.mb) return MLKH_ERR_CONFIG;
    return MLKH_OK;
}

bool zero_cfg(const mlkh_config* c) { return !c || (c->mb == 0 && c->nb == 0 && c->kb == 0 && c->unroll == 0); }

}  // namespace

extern "C" {

int32_t mlkh_max_threads(void) { return omp_get_max_threads(); }

int mlkh_matmul_f32(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B, int64_t ldb,
                    float* C, int64_t ldc, int accumulate, const mlkh_config* cfg) {
    if (M < 0 || N < 0 || K < 0) return MLKH_ERR_SHAPE;
    if (M == 0 || N == 0) return MLKH_OK;
    if (!C || (K > 0 && (!A || !B))) return MLKH_ERR_NULL;
    if (lda < std::max<int64_t>(K, 1) || ldb < std::max<int64_t>(N, 1) || ldc < std::max<int64_t>(N, 1))
        return MLKH_ERR_LAYOUT;
    const mlkh_config c = zero_cfg(cfg) ? default_mm(M, N) : *cfg;
    if (int st = check_cfg(0, c)) return st;
    const mm_fn fn = mm_kernel(c.unroll);
    const int64_t tm = cdiv(M, c.mb), tn = cdiv(N, c.nb);
#pragma omp parallel for collapse(2) schedule(dynamic, 1) num_threads(threads_of(c))
    for (int64_t bi = 0; bi < tm; ++bi)
        for (int64_t bj = 0; bj < tn; ++bj) {
            const int64_t i0 = bi * c.mb, i1 = std::min(M, i0 + c.mb);
            const int64_t j0 = bj * c.nb, j1 = std::min(N, j0 + c.nb);
            if (!accumulate)
                for (int64_t i = i0; i < i1; ++i) std::memset(C + i * ldc + j0, 0, sizeof(float) * (j1 - j0));
            if (K > 0) fn(i0, i1, j0, j1, K, c.kb, A, lda, B, ldb, C, ldc);
        }
    return MLKH_OK;
}

int mlkh_conv2d_f32(int64_t N, int64_t C, int64_t H, int64_t W, int64_t F, int64_t KH, int64_t KW, int32_t sh,
                    int32_t sw, int32_t ph, int32_t pw, const float* x, const float* w, float* y, int accumulate,
                    const mlkh_config* cfg) {
    if (N < 1 || C < 1 || H < 1 || W < 1 || F < 1 || KH < 1 || KW < 1 || sh < 1 || sw < 1 || ph < 0 || pw < 0)
        return MLKH_ERR_SHAPE;
    const int64_t HO = conv_out(H, KH, sh, ph), WO = conv_out(W, KW, sw, pw);
    if (HO < 1 || WO < 1) return MLKH_ERR_SHAPE;
    if (!x || !w || !y) return MLKH_ERR_NULL;
    const mlkh_config c = zero_cfg(cfg) ? default_conv() : *cfg;
    if (int st = check_cfg(1, c)) return st;
    const int64_t fb = std::min<int64_t>(c.mb, F);
    const int64_t nfb = cdiv(F, fb);
    const conv_fn fu = conv_kernel(c.unroll), f1 = conv_kernel(1);
#pragma omp parallel for collapse(3) schedule(dynamic, 1) num_threads(threads_of(c))
    for (int64_t n = 0; n < N; ++n)
        for (int64_t b = 0; b < nfb; ++b)
            for (int64_t oh = 0; oh < HO; ++oh) {
                const int64_t f0 = b * fb, f1e = std::min(F, f0 + fb);
                if (!accumulate)
                    for (int64_t f = f0; f < f1e; ++f) std::memset(y + ((n * F + f) * HO + oh) * WO, 0, sizeof(float) * WO);
                int64_t f = f0;
                for (; f + c.unroll <= f1e; f += c.unroll)
                    fu(n, f, oh, C, H, W, F, KH, KW, sh, sw, ph, pw, HO, WO, x, w, y);
                for (; f < f1e; ++f) f1(n, f, oh, C, H, W, F, KH, KW, sh, sw, ph, pw, HO, WO, x, w, y);
            }
    return MLKH_OK;
}

int32_t mlkh_config_count(int32_t op, const int64_t* d) {
    if ((op != 0 && op != 1) || !d) return -1;
    return (int32_t)space(op, d).size();
}

int mlkh_config_get(int32_t op, const int64_t* d, int32_t i, mlkh_config* cfg) {
    if ((op != 0 && op != 1) || !d || !cfg) return MLKH_ERR_NULL;
    const std::vector<mlkh_config> v = space(op, d);
    if (i < 0 || i >= (int32_t)v.size()) return MLKH_ERR_ARG;
    *cfg = v[(size_t)i];
    return MLKH_OK;
}

int mlkh_tune(int32_t op, const int64_t* d, int32_t strategy, double budget_frac, int32_t reps, uint64_t seed,
              mlkh_config* best, double* best_us, double* times_us) {
    if ((op != 0 && op != 1) || !d || !best) return MLKH_ERR_NULL;
    if (strategy != 0 && strategy != 1) return MLKH_ERR_ARG;
    if (strategy == 1 && !(budget_frac > 0.0 && budget_frac <= 1.0)) return MLKH_ERR_ARG;
    const int r = reps > 0 ? reps : 5;
    const std::vector<mlkh_config> cfgs = space(op, d);
    const int S = (int)cfgs.size();
    // seeded scratch inputs of the problem's shape
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<float> ud(-1.0f, 1.0f);
    std::vector<float> a, b, c;
    if (op == 0) {
        if (d[0] < 1 || d[1] < 1 || d[2] < 0) return MLKH_ERR_SHAPE;
        a.resize((size_t)(d[0] * d[2]));
        b.resize((size_t)(d[2] * d[1]));
        c.assign((size_t)(d[0] * d[1]), 0.0f);
    } else {
        const int64_t HO = conv_out(d[2], d[5], d[7], d[9]), WO = conv_out(d[3], d[6], d[8], d[10]);
        if (HO < 1 || WO < 1) return MLKH_ERR_SHAPE;
        a.resize((size_t)(d[0] * d[1] * d[2] * d[3]));
        b.resize((size_t)(d[4] * d[1] * d[5] * d[6]));
        c.assign((size_t)(d[0] * d[4] * HO * WO), 0.0f);
    }
    for (float& v : a) v = ud(rng);
    for (float& v : b) v = ud(rng);
    auto run = [&](const mlkh_config& cf) {
        return op == 0 ? mlkh_matmul_f32(d[0], d[1], d[2], a.data(), d[2], b.data(), d[1], c.data(), d[1], 0, &cf)
                       : mlkh_conv2d_f32(d[0], d[1], d[2], d[3], d[4], d[5], d[6], (int32_t)d[7], (int32_t)d[8],
                                         (int32_t)d[9], (int32_t)d[10], a.data(), b.data(), c.data(), 0, &cf);
    };
    std::vector<double> t((size_t)S, -1.0);
    auto eval = [&](int i) {
        if (t[(size_t)i] >= 0) return t[(size_t)i];
        if (run(cfgs[(size_t)i]) != MLKH_OK) return t[(size_t)i] = 1e30;
        std::vector<double> v;
        for (int k = 0; k < r; ++k) {
            const auto t0 = std::chrono::steady_clock::now();
            run(cfgs[(size_t)i]);
            v.push_back(std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count());
        }
        std::sort(v.begin(), v.end());
        return t[(size_t)i] = v[v.size() / 2];
    };
    if (strategy == 0) {
        for (int i = 0; i < S; ++i) eval(i);
    } else {
        // (1+1) evolution strategy: mutate one or two fields of the best so far
        // to a neighbouring value in the space; keep the child when faster
        const int budget = std::max(1, std::min(S, (int)std::ceil(budget_frac * S - 1e-9)));
        int parent = (int)(rng() % (uint64_t)S);
        double tp = eval(parent);
        int used = 1;
        auto dist = [&](const mlkh_config& x, const mlkh_config& y) {
            return (x.mb != y.mb) + (x.nb != y.nb) + (x.kb != y.kb) + (x.unroll != y.unroll) + (x.threads != y.threads);
        };
        int fails = 0;
        while (used < budget) {
            std::vector<int> cand;
            for (int dd = 1; dd <= 5 && cand.empty(); ++dd)
                for (int i = 0; i < S; ++i)
                    if (t[(size_t)i] < 0 && dist(cfgs[(size_t)i], cfgs[(size_t)parent]) == dd) cand.push_back(i);
            if (cand.empty()) break;
            const int child = cand[(size_t)(rng() % cand.size())];
            const double tc = eval(child);
            ++used;
            if (tc < tp) {
                parent = child;
                tp = tc;
                fails = 0;
            } else if (++fails >= 8 && used < budget) {  // restart from an unmeasured configuration
                std::vector<int> fresh;
                for (int i = 0; i < S; ++i)
                    if (t[(size_t)i] < 0) fresh.push_back(i);
                if (fresh.empty()) break;
                const int s2 = fresh[(size_t)(rng() % fresh.size())];
                const double ts = eval(s2);
                ++used;
                if (ts < tp) {
                    parent = s2;
                    tp = ts;
                }
                fails = 0;
            }
        }
    }
    int pick = -1;
    for (int i = 0; i < S; ++i)
        if (t[(size_t)i] >= 0 && t[(size_t)i] < 1e29 && (pick < 0 || t[(size_t)i] < t[(size_t)pick])) pick = i;
    if (pick < 0) return MLKH_ERR_CONFIG;
    *best = cfgs[(size_t)pick];
    if (best_us) *best_us = t[(size_t)pick];
    if (times_us)
        for (int i = 0; i < S; ++i) times_us[i] = t[(size_t)i] >= 1e29 ? -1.0 : t[(size_t)i];
    return MLKH_OK;
}

}  // extern "C"
