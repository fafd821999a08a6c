// api.cpp -- the C ABI (include/mlk.h): validation, configuration space,
// dispatch to the compiled tile kernels, batched / persistent / graph
// launches, and the elementwise entry points.
//
// Every argument check runs on the host before the first HIP call, so each
// MLK_ERR_* except MLK_ERR_HIP can be produced without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace mlk {

// ------------------------------------------------------------------ errors

static thread_local std::string t_err;

mlk_status fail(mlk_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return s;
}

void clear_error() { t_err.clear(); }

mlk_status hip_fail(hipError_t e, const char* what) {
    return fail(MLK_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ------------------------------------------------------------------ device facts

int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        v = 256;
    cache[dev] = v;
    return v;
}

// ------------------------------------------------------------------ registry

const std::vector<const KernelEntry*>& registry() {
    static std::vector<const KernelEntry*> all = [] {
        std::vector<const KernelEntry*> v;
        const KernelEntry* (*tables[])(int*) = {kernels_f32, kernels_bf16, kernels_i8, kernels_f8,
                                                kernels_conv, kernels_fast, kernels_direct, kernels_conv_chunk};
        for (auto t : tables) {
            int n = 0;
            const KernelEntry* e = t(&n);
            for (int i = 0; i < n; ++i) v.push_back(e + i);
        }
        return v;
    }();
    return all;
}

// the MFMA tile of an entry or configuration: 32, or 16 (also written 0)
static int mfma_of(int v) { return v == 32 ? 32 : 16; }

const KernelEntry* find_kernel(int dt, int conv, const mlk_tile_config& c) {
    if (c.mfma != 0 && c.mfma != 16 && c.mfma != 32) return nullptr;
    for (const KernelEntry* e : registry())
        if (e->dt == dt && e->conv == conv && e->bm == c.bm && e->bn == c.bn && e->bk == c.bk &&
            e->wm == c.wm && e->wn == c.wn && e->stages == c.stages && mfma_of(e->mfma) == mfma_of(c.mfma))
            return e;
    return nullptr;
}

int dt_of(mlk_dtype in, mlk_dtype out, int conv, bool* ok) {
    *ok = true;
    if (in == MLK_F32 && out == MLK_F32) return DT_F32;
    if (in == MLK_BF16 && out == MLK_F32) return DT_BF16;
    if (!conv && in == MLK_F8E4M3 && out == MLK_F32) return DT_F8;
    // bf16 results (matmul only): the input type picks the kernel
    if (!conv && in == MLK_BF16 && out == MLK_BF16) return DT_BF16;
    if (!conv && in == MLK_F8E4M3 && out == MLK_BF16) return DT_F8;
    if (!conv && in == MLK_I8 && out == MLK_I32) return DT_I8;
    *ok = false;
    return -1;
}

static int esize_in(int dt) { return dt == DT_F32 ? 4 : dt == DT_BF16 ? 2 : 1; }

int64_t conv_out(int64_t in, int64_t k, int64_t stride, int64_t pad) {
    const int64_t span = in + 2 * pad - k;
    if (span < 0 || stride <= 0) return 0;
    return span / stride + 1;
}

// largest extent any one launch accepts (tile coordinates are int32)
static const int64_t kMaxDim = (int64_t)1 << 31;

static mlk_status check_conv_dims(int64_t n, int64_t c, int64_t h, int64_t w, int64_t f,
                                  int64_t kh, int64_t kw, int sh, int sw, int ph, int pw,
                                  int64_t* ho, int64_t* wo) {
    if (n < 1 || c < 1 || h < 1 || w < 1 || f < 1 || kh < 1 || kw < 1)
        return fail(MLK_ERR_SHAPE, "conv2d: every dimension must be >= 1");
    if (sh < 1 || sw < 1) return fail(MLK_ERR_SHAPE, "conv2d: strides must be >= 1");
    if (ph < 0 || pw < 0) return fail(MLK_ERR_SHAPE, "conv2d: padding must be >= 0");
    if (n > kMaxDim || c > kMaxDim || h > kMaxDim || w > kMaxDim || f > kMaxDim)
        return fail(MLK_ERR_SHAPE, "conv2d: dimension too large");
    *ho = conv_out(h, kh, sh, ph);
    *wo = conv_out(w, kw, sw, pw);
    if (*ho < 1 || *wo < 1)
        return fail(MLK_ERR_SHAPE, "conv2d: the filter does not fit the padded image");
    if (n * (*ho) * (*wo) > kMaxDim || c * kh * kw > kMaxDim || n * c * h * w >= kMaxDim)
        return fail(MLK_ERR_SHAPE, "conv2d: problem too large for one launch");
    return MLK_OK;
}

mlk_status shape_of_problem(const mlk_problem* p, Shape* s) {
    if (!p) return fail(MLK_ERR_NULL, "problem is NULL");
    bool ok = false;
    s->conv = p->op == MLK_OP_CONV2D;
    s->accumulate = p->accumulate ? 1 : 0;
    if (p->op != MLK_OP_MATMUL && p->op != MLK_OP_CONV2D && p->op != MLK_OP_BATCHED)
        return fail(MLK_ERR_ARG, "unknown op %d", p->op);
    s->dt = dt_of((mlk_dtype)p->in, (mlk_dtype)p->out, s->conv, &ok);
    if (!ok) return fail(MLK_ERR_DTYPE, "unsupported dtype pair (%d, %d) for op %d", p->in, p->out, p->op);
    s->out16 = p->out == MLK_BF16 ? 1 : 0;
    if (p->op == MLK_OP_MATMUL) {
        if (p->M < 0 || p->N < 0 || p->K < 0) return fail(MLK_ERR_SHAPE, "negative matmul dimension");
        if (p->M > kMaxDim || p->N > kMaxDim || p->K > kMaxDim)
            return fail(MLK_ERR_SHAPE, "matmul dimension too large");
        s->M = p->M;
        s->N = p->N;
        s->K = p->K;
    } else if (p->op == MLK_OP_CONV2D) {
        int64_t ho, wo;
        mlk_status st = check_conv_dims(p->n, p->c, p->h, p->w, p->f, p->kh, p->kw, p->sh, p->sw,
                                        p->ph, p->pw, &ho, &wo);
        if (st != MLK_OK) return st;
        s->M = p->f;
        s->N = p->n * ho * wo;
        s->K = p->c * p->kh * p->kw;
        s->conv_c = p->c;
        s->conv_in = p->n * p->c * p->h * p->w;
        s->conv_kh = (int)p->kh;
        s->conv_kw = (int)p->kw;
        s->conv_sh = p->sh;
        s->conv_sw = p->sw;
    } else {
        if (p->count < 1) return fail(MLK_ERR_SHAPE, "batched: count must be >= 1");
        if (!p->descs) return fail(MLK_ERR_NULL, "batched: descs is NULL");
        if ((s->dt != DT_BF16 && s->dt != DT_F32) || s->out16)
            return fail(MLK_ERR_DTYPE, "batched: only bf16 and f32 inputs with fp32 outputs are supported");
        int64_t mm = 0, nn = 0, kk = 0;
        for (int64_t i = 0; i < p->count; ++i) {
            const mlk_gemm_desc& d = p->descs[i];
            if (d.M < 0 || d.N < 0 || d.K < 0) return fail(MLK_ERR_SHAPE, "batched: negative dimension in desc %lld", (long long)i);
            if (d.M > kMaxDim || d.N > kMaxDim || d.K > kMaxDim)
                return fail(MLK_ERR_SHAPE, "batched: dimension too large in desc %lld", (long long)i);
            mm = std::max(mm, d.M);
            nn = std::max(nn, d.N);
            kk = std::max(kk, d.K);
        }
        s->M = mm;
        s->N = nn;
        s->K = kk;
    }
    return MLK_OK;
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Shapes the direct-to-LDS kernels take: after packing (K rounded up to the
// stage depth, rows to 16 bytes) each operand stays below 2 GiB (32-bit buffer
// offsets).
static bool fast_shape_ok(const Shape& s, int bk) {
    const int64_t es = esize_in(s.dt);
    // conv: the filter (F x C*KH*KW) and the NHWC input are read in place, the
    // depth in whole stages
    if (s.conv) return s.K % bk == 0 && s.M * s.K * es < ((int64_t)1 << 31) && s.conv_in * es < ((int64_t)1 << 31);
    const int64_t Kp = cdiv(std::max<int64_t>(s.K, 1), bk) * bk, Np = cdiv(s.N, 16 / es) * (16 / es);
    return s.M * Kp * es < ((int64_t)1 << 31) && Kp * Np * es < ((int64_t)1 << 31);
}

static bool is_direct(const KernelEntry* e) { return e->conv && e->wm == 0; }

bool is_chunk_conv(const KernelEntry* e) { return e->conv && e->dt == DT_F32 && e->stages == 1; }

bool chunk_conv_ok(const Shape& s) {
    const int64_t taps = (int64_t)s.conv_kh * s.conv_kw;
    return s.conv && s.conv_in < ((int64_t)1 << 31) && s.K * std::max<int64_t>(taps, 1) < ((int64_t)1 << 32);
}

// The direct-layout matmul tiles address their output tile with 32-bit
// offsets from its corner; with ldc >= N the rows of a tile span at least
// (bm - 1) * N + bn elements.
static bool fast_ldc_ok(const Shape& s, const KernelEntry* e) {
    return s.conv || e->stages < 1 || (int64_t)(e->bm - 1) * std::max<int64_t>(s.N, 1) + e->bn < ((int64_t)1 << 31);
}

// the direct (stencil) conv covers few filters, small strides and taps
static bool direct_ok(const Shape& s) {
    return s.conv && s.M <= kDirectMaxF && s.conv_sh <= kDirectMaxStride && s.conv_sw <= kDirectMaxStride &&
           s.conv_kh <= kDirectMaxTap && s.conv_kw <= kDirectMaxTap;
}

mlk_status check_config(const Shape& s, int op, const mlk_tile_config& c) {
    const KernelEntry* e = find_kernel(s.dt, s.conv, c);
    if (!e)
        return fail(MLK_ERR_CONFIG, "no compiled kernel for tile %dx%dx%d waves %dx%d stages %d mfma %d (dtype %d%s)",
                    c.bm, c.bn, c.bk, c.wm, c.wn, c.stages, c.mfma, s.dt, s.conv ? ", conv" : "");
    if (!fast_ldc_ok(s, e))
        return fail(MLK_ERR_CONFIG, "direct-layout tile: N too large for its %d-row tile (32-bit output offsets)",
                    e->bm);
    // (matmul operands that do not fit these tiles are packed, so any shape is fine)
    if (e->stages >= 2 && op != MLK_OP_BATCHED && !fast_shape_ok(s, e->bk)) {
        if (s.conv)
            return fail(MLK_ERR_CONFIG, "direct-to-LDS conv tile: needs C*KH*KW a multiple of %d and operands "
                        "below 2 GiB", e->bk);
        return fail(MLK_ERR_CONFIG, "direct-to-LDS tile: an operand exceeds 2 GiB");
    }
    if (c.split_k < 1 || c.split_k > 64) return fail(MLK_ERR_CONFIG, "split_k must be in [1, 64]");
    const int64_t stages = cdiv(std::max<int64_t>(s.K, 1), c.bk);
    if (c.split_k > 1 && c.split_k > stages)
        return fail(MLK_ERR_CONFIG, "split_k %d exceeds the %lld K stages", c.split_k, (long long)stages);
    if (c.split_k > 1 && s.out16)
        return fail(MLK_ERR_CONFIG, "a bf16 output is rounded once from the whole sum: split_k must be 1");
    if (s.out16 && !e->launch_epi16)
        return fail(MLK_ERR_CONFIG, "a bf16 output is written by the direct-to-LDS (stages >= 2, 16x16 MFMA) and "
                    "plain (stages 0) tiles, not the register-loaded fast tiles or the 32x32 MFMA tiles");
    if (c.group_m < 0 || c.group_m > 64) return fail(MLK_ERR_CONFIG, "group_m must be in [0, 64]");
    if (c.xcd_remap != 0 && c.xcd_remap != 1) return fail(MLK_ERR_CONFIG, "xcd_remap must be 0 or 1");
    if (is_direct(e)) {
        if (c.layout != 2 || c.split_k != 1)
            return fail(MLK_ERR_CONFIG, "the direct conv tile runs as layout 2 with split_k 1");
        if (!direct_ok(s))
            return fail(MLK_ERR_CONFIG, "direct conv: needs F <= %d, strides <= %d and filters up to %dx%d",
                        kDirectMaxF, kDirectMaxStride, kDirectMaxTap, kDirectMaxTap);
        return MLK_OK;
    }
    if (is_chunk_conv(e) && (c.layout != 0 || !chunk_conv_ok(s)))
        return fail(MLK_ERR_CONFIG, "the fp32 chunk-gather conv tile runs as layout 0 and needs C*H*W*N below 2^31 "
                    "and C*KH*KW*KH*KW below 2^32");
    if (c.layout != 0 && !(s.conv && (c.layout == 1 || c.layout == 3)))
        return fail(MLK_ERR_CONFIG, "layout must be 0, or 1 or 3 for conv2d (2 only for the direct conv tiles)");
    if (s.conv && !e->launch && c.layout == 0)
        return fail(MLK_ERR_CONFIG, "this conv tile runs only the channels-last layouts (layout 1 or 3)");
    if (c.layout == 1 && (!e->launch_nhwc || s.conv_c % (16 / esize_in(s.dt)) != 0))
        return fail(MLK_ERR_CONFIG, "channels-last layout needs C a multiple of %d", 16 / esize_in(s.dt));
    if (c.layout == 3 && (!e->launch_gather || s.conv_c % (16 / esize_in(s.dt)) != 0 || s.M > 65535))
        return fail(MLK_ERR_CONFIG, "the channel-gather layout (3) needs a register-loaded bf16 conv tile, C a "
                    "multiple of %d and F <= 65535", 16 / esize_in(s.dt));
    const int64_t tiles = cdiv(s.M, c.bm) * cdiv(s.N, c.bn) * c.split_k;
    if (tiles > ((int64_t)1 << 31) - 1) return fail(MLK_ERR_CONFIG, "too many workgroups");
    return MLK_OK;
}

std::vector<mlk_tile_config> enumerate_configs(const mlk_problem* p, const Shape& s) {
    std::vector<mlk_tile_config> out;
    const bool batched = p->op == MLK_OP_BATCHED;
    for (const KernelEntry* e : registry()) {
        if (e->dt != s.dt || e->conv != s.conv) continue;
        if (batched && !e->persist) continue;
        if (is_direct(e)) {
            if (direct_ok(s)) out.push_back(mlk_tile_config{e->bm, e->bn, e->bk, 0, 0, 1, 1, 0, 0, 2, 0});
            continue;
        }
        if (e->stages >= 2 && !batched && !fast_shape_ok(s, e->bk)) continue;
        if (is_chunk_conv(e) && !chunk_conv_ok(s)) continue;
        if (!fast_ldc_ok(s, e)) continue;
        if (s.out16 && !e->launch_epi16) continue;
        // a tile at least twice the problem in a dimension only adds padding
        if (e->bm > 32 && e->bm >= 2 * s.M) continue;
        if (e->bn > 32 && e->bn >= 2 * s.N) continue;
        const int64_t stages = cdiv(std::max<int64_t>(s.K, 1), e->bk);
        const int64_t tiles = cdiv(std::max<int64_t>(s.M, 1), e->bm) * cdiv(std::max<int64_t>(s.N, 1), e->bn);
        const int64_t tm = cdiv(std::max<int64_t>(s.M, 1), e->bm);
        // deep, narrow problems (batch-1 convolutions) fill the device only by splitting K far
        for (int sk : {1, 2, 4, 8, 16, 32}) {
            if ((batched || s.out16) && sk > 1) break;
            // (the chunk-gather conv tiles are built for one or two chunks per split)
            if (sk > 1 && stages < (is_chunk_conv(e) ? 1 : 2) * sk) break;
            // past 8, split only problems with too few tiles for four rounds of the device
            if (sk > 8 && tiles * sk > 4 * device_cus()) break;
            for (int gm : {1, 8}) {
                if (gm == 8 && (batched || tm < 16)) continue;
                for (int xcd : {0, 1}) {
                    const int64_t nblk = tiles * sk;
                    if (xcd == 1 && (batched || nblk < 64 || nblk % 8 != 0)) continue;
                    for (int lay : {0, 1, 3}) {
                        const bool cl = s.conv && s.conv_c % (16 / esize_in(s.dt)) == 0;
                        if (lay == 1 && !(cl && e->launch_nhwc)) continue;
                        if (lay == 3 && !(cl && e->launch_gather && s.M <= 65535)) continue;
                        if (lay == 0 && !e->launch) continue;
                        mlk_tile_config c{e->bm, e->bn, e->bk, e->wm, e->wn, sk, gm, xcd, e->stages, lay,
                                          e->mfma == 32 ? 32 : 0};
                        out.push_back(c);
                    }
                }
            }
        }
    }
    return out;
}

mlk_tile_config heuristic_config(const Shape& s, int op, bool conv_gather) {
    const int cus = device_cus();
    // biggest tile (by area, then by fewer waves) that still gives >= one tile per CU
    const KernelEntry* best = nullptr;
    const KernelEntry* smallest = nullptr;
    for (const KernelEntry* e : registry()) {
        if (e->dt != s.dt || e->conv != s.conv || e->stages || is_direct(e)) continue;
        if (op == MLK_OP_BATCHED && !e->persist) continue;
        if (!smallest || e->bm * e->bn < smallest->bm * smallest->bn ||
            (e->bm * e->bn == smallest->bm * smallest->bn && e->bk > smallest->bk))
            smallest = e;
        const int64_t tiles = cdiv(std::max<int64_t>(s.M, 1), e->bm) * cdiv(std::max<int64_t>(s.N, 1), e->bn);
        if (tiles < cus) continue;
        if (e->bm * e->bn > 128 * 256) continue;  // the largest tiles only win when tuned
        if (!best || e->bm * e->bn > best->bm * best->bn ||
            (e->bm * e->bn == best->bm * best->bn && e->bk > best->bk))
            best = e;
    }
    const KernelEntry* e = best ? best : smallest;
    mlk_tile_config c{e->bm, e->bn, e->bk, e->wm, e->wn, 1, 1, 0, 0, 0, 0};
    // large bf16 / e4m3 matmuls: the 8-wave direct-to-LDS tile, grouped raster
    if (op == MLK_OP_MATMUL && (s.dt == DT_BF16 || s.dt == DT_F8) &&
        cdiv(s.M, 256) * cdiv(s.N, 256) >= cus && s.K >= 256) {
        for (const KernelEntry* f : registry())
            if (f->dt == s.dt && !f->conv && f->stages == 2 && f->bm == 256 && f->bn == 256 &&
                f->wm == 2 && f->wn == 4 && mfma_of(f->mfma) == 16 && fast_shape_ok(s, f->bk) && fast_ldc_ok(s, f)) {
                const int64_t tiles = cdiv(s.M, 256) * cdiv(s.N, 256);
                return mlk_tile_config{256, 256, f->bk, 2, 4, 1, 8, tiles % 8 == 0 ? 1 : 0, 2, 0, 0};
            }
    }
    // few filters over a shallow depth: the direct (stencil) conv, whose MFMA
    // tile would be mostly padding rows
    if (s.conv && direct_ok(s) && (s.dt == DT_F32 || s.K <= 64)) {
        for (const KernelEntry* d : registry())
            if (is_direct(d) && d->dt == s.dt && d->bm == 16)
                return mlk_tile_config{d->bm, d->bn, d->bk, 0, 0, 1, 1, 0, 0, 2, 0};
    }
    // bf16 convolutions with C a multiple of 8: the 64 x 64 channel-gather
    // tile (one launch, no input copy, any depth), K split while the device
    // has fewer than two tiles per CU and each split keeps two stages
    if (conv_gather && s.conv && s.dt == DT_BF16 && s.conv_c % 8 == 0 && s.M <= 65535 && op == MLK_OP_CONV2D) {
        for (const KernelEntry* f : registry())
            if (f->dt == DT_BF16 && f->conv && f->stages == 1 && f->bm == 64 && f->bn == 64 && f->launch_gather) {
                mlk_tile_config h{64, 64, f->bk, f->wm, f->wn, 1, 1, 0, 1, 3, 0};
                const int64_t tiles = cdiv(s.M, 64) * cdiv(s.N, 64);
                const int64_t stages = cdiv(s.K, f->bk);
                while (h.split_k < 16 && tiles * h.split_k * 2 <= cus && stages >= 2 * 2 * h.split_k) h.split_k *= 2;
                return h;
            }
    }
    // fp32 convolutions with fewer 64 x 64 tiles than CUs: the chunk-gather
    // tile (one launch, no input copy), K split into at most 16 parts while the
    // parts keep two 16-deep chunks each and the grid stays within two
    // workgroups per CU
    if (s.conv && s.dt == DT_F32 && op == MLK_OP_CONV2D && chunk_conv_ok(s) &&
        cdiv(s.M, 64) * cdiv(s.N, 64) < cus) {
        for (const KernelEntry* f : registry())
            if (is_chunk_conv(f) && f->bm == 64 && f->bn == 64 && f->bk == 16) {
                mlk_tile_config h{64, 64, 16, f->wm, f->wn, 1, 1, 0, 1, 0, 0};
                const int64_t tiles = cdiv(s.M, 64) * cdiv(s.N, 64);
                const int64_t stages = cdiv(s.K, 16);
                while (h.split_k < 16 && tiles * h.split_k * 2 <= 2 * cus && stages >= 2 * 2 * h.split_k)
                    h.split_k *= 2;
                return h;
            }
    }
    // channels-last pays a transpose of the input: worth it for large images
    if (s.conv && e->launch_nhwc && s.conv_c % (16 / esize_in(s.dt)) == 0 && s.N >= 16384) c.layout = 1;
    if (!best && op != MLK_OP_BATCHED && !s.out16) {
        // too few tiles: split K while each split keeps >= 4 stages
        const int64_t tiles = cdiv(std::max<int64_t>(s.M, 1), e->bm) * cdiv(std::max<int64_t>(s.N, 1), e->bn);
        const int64_t stages = cdiv(std::max<int64_t>(s.K, 1), e->bk);
        while (c.split_k < 8 && tiles * c.split_k * 2 <= cus && stages >= 4 * 2 * c.split_k) c.split_k *= 2;
    }
    return c;
}

std::string problem_key(const mlk_problem* p) {
    char buf[256];
    if (p->op == MLK_OP_MATMUL) {
        snprintf(buf, sizeof buf, "matmul;in=%d;out=%d;acc=%d;M=%lld;N=%lld;K=%lld", p->in, p->out,
                 p->accumulate ? 1 : 0, (long long)p->M, (long long)p->N, (long long)p->K);
        return buf;
    }
    if (p->op == MLK_OP_CONV2D) {
        snprintf(buf, sizeof buf,
                 "conv2d;in=%d;out=%d;acc=%d;n=%lld;c=%lld;h=%lld;w=%lld;f=%lld;kh=%lld;kw=%lld;s=%d,%d;p=%d,%d",
                 p->in, p->out, p->accumulate ? 1 : 0, (long long)p->n, (long long)p->c,
                 (long long)p->h, (long long)p->w, (long long)p->f, (long long)p->kh,
                 (long long)p->kw, p->sh, p->sw, p->ph, p->pw);
        return buf;
    }
    // batched: FNV-1a over the shape list
    uint64_t h = 1469598103934665603ull;
    for (int64_t i = 0; i < p->count; ++i) {
        const int64_t v[3] = {p->descs[i].M, p->descs[i].N, p->descs[i].K};
        const unsigned char* b = (const unsigned char*)v;
        for (size_t j = 0; j < sizeof v; ++j) h = (h ^ b[j]) * 1099511628211ull;
    }
    snprintf(buf, sizeof buf, "batched;in=%d;out=%d;acc=%d;count=%lld;shapes=%016llx", p->in, p->out,
             p->accumulate ? 1 : 0, (long long)p->count, (unsigned long long)h);
    return buf;
}

static std::mutex g_def_mu;
static std::unordered_map<std::string, mlk_tile_config> g_defaults;

bool lookup_default(const std::string& key, mlk_tile_config* c) {
    std::lock_guard<std::mutex> g(g_def_mu);
    auto it = g_defaults.find(key);
    if (it == g_defaults.end()) return false;
    *c = it->second;
    return true;
}

void store_default(const std::string& key, const mlk_tile_config& c) {
    std::lock_guard<std::mutex> g(g_def_mu);
    g_defaults[key] = c;
}

static bool cfg_is_zero(const mlk_tile_config* c) {
    return !c || (c->bm == 0 && c->bn == 0 && c->bk == 0 && c->wm == 0 && c->wn == 0);
}

// resolve the configuration of a launch (explicit / tuned default / heuristic)
static mlk_status resolve(const mlk_problem& p, const Shape& s, const mlk_tile_config* cfg,
                          mlk_tile_config* out) {
    if (!cfg_is_zero(cfg)) {
        *out = *cfg;
        if (out->group_m == 0) out->group_m = 1;
        if (out->split_k == 0) out->split_k = 1;
        return check_config(s, p.op, *out);
    }
    if (lookup_default(problem_key(&p), out)) return MLK_OK;
    *out = heuristic_config(s, p.op);
    return MLK_OK;
}

// ------------------------------------------------------------------ launches

static GemmArgs base_args(const Shape& s, const mlk_tile_config& cfg) {
    GemmArgs g;
    memset(&g, 0, sizeof g);
    g.M = s.M;
    g.N = s.N;
    g.K = s.K;
    g.accumulate = s.accumulate;
    g.split_k = cfg.split_k;
    g.atomic = cfg.split_k > 1 ? 1 : 0;
    g.tiles_m = (int32_t)cdiv(s.M, cfg.bm);
    g.tiles_n = (int32_t)cdiv(s.N, cfg.bn);
    g.group_m = cfg.group_m < 1 ? 1 : cfg.group_m;
    g.xcd_remap = cfg.xcd_remap;
    g.out_bf16 = s.out16;
    return g;
}

static mlk_status run_gemm(const KernelEntry* e, GemmArgs& g, const Shape& s, void* C, int64_t M,
                           int64_t N, int64_t ldc, hipStream_t st) {
    const int esz = 4;  // split K (the only zeroing route) has 32-bit outputs
    if (!e->launch) return fail(MLK_ERR_CONFIG, "this conv tile runs only the channels-last layout (layout 1)");
    if (g.atomic && !s.accumulate) {
        hipError_t z = launch_zero_matrix(C, M, N, ldc, esz, st);
        if (z != hipSuccess) return hip_fail(z, "zero output");
    }
    // a bf16 C, or a bias, takes the entry's variant with that output stage
    const launch_fn fn = g.out_bf16 ? e->launch_epi16 : g.bias ? e->launch_epi : e->launch;
    if (!fn) return fail(MLK_ERR_CONFIG, "this tile has no bias / bf16-output variant");
    const int64_t nblk = (int64_t)g.tiles_m * g.tiles_n * g.split_k;
    hipError_t err = fn(g, (int)nblk, st);
    if (err != hipSuccess) return hip_fail(err, "kernel launch");
    return MLK_OK;
}

// Routes that use the library's scratch memory are refused on a capturing
// stream (checked before anything is enqueued).
static mlk_status refuse_under_capture(hipStream_t st, const char* what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(MLK_ERR_CONFIG, "%s needs library scratch memory, which is not used under stream capture; "
                    "choose a configuration without it", what);
    return MLK_OK;
}

// How a direct-to-LDS launch takes its operands: an operand without 16-byte
// rows, or with K not a multiple of the stage depth, is first copied into a
// zero-padded buffer (A as M x Kp, B as Kp x Np; Kp = K rounded up to the
// stage depth, Np = N rounded up to 16 bytes).
struct PackPlan {
    bool pa = false, pb = false;
    int64_t Kp = 0, Np = 0, lda2 = 0, ldb2 = 0;
    int64_t abytes = 0, bbytes = 0;  // workspace bytes of each packed copy
};

static PackPlan pack_plan(const Shape& s, const KernelEntry* e, const void* A, int64_t lda, const void* B,
                          int64_t ldb) {
    PackPlan pp;
    const int es = esize_in(s.dt);
    pp.lda2 = lda;
    pp.ldb2 = ldb;
    if (e->stages < 2 || s.K == 0 || s.M == 0 || s.N == 0) return pp;
    const bool vec_a = ((uintptr_t)A % 16 == 0) && ((lda * es) % 16 == 0);
    const bool vec_b = ((uintptr_t)B % 16 == 0) && ((ldb * es) % 16 == 0);
    const bool kfit = s.K % e->bk == 0;
    pp.pa = !(vec_a && kfit);
    // B is read in whole 16-byte chunks up to its last row's padded end
    pp.pb = !(vec_b && kfit && s.N % (16 / es) == 0);
    pp.Kp = cdiv(s.K, e->bk) * e->bk;
    pp.Np = cdiv(s.N, 16 / es) * (16 / es);
    pp.lda2 = pp.pa ? pp.Kp : lda;
    pp.ldb2 = pp.pb ? pp.Np : ldb;
    pp.abytes = pp.pa ? cdiv(s.M * pp.Kp * es, 256) * 256 : 0;
    pp.bbytes = pp.pb ? pp.Kp * pp.Np * es : 0;
    return pp;
}

int64_t dense_workspace_bytes(const Shape& s, const void* A, int64_t lda, const void* B, int64_t ldb,
                              const mlk_tile_config& cfg) {
    const KernelEntry* e = find_kernel(s.dt, 0, cfg);
    if (!e) return 0;
    const PackPlan pp = pack_plan(s, e, A, lda, B, ldb);
    return pp.abytes + pp.bbytes;
}

mlk_status launch_dense(const Shape& s, const void* A, int64_t lda, const void* B, int64_t ldb,
                        void* C, int64_t ldc, const float* sa, const float* sb,
                        const mlk_tile_config& cfg, hipStream_t st, const float* bias, void* ext_ws,
                        size_t ext_bytes) {
    const KernelEntry* e = find_kernel(s.dt, 0, cfg);
    if (!e) return fail(MLK_ERR_CONFIG, "no kernel for configuration");
    if (s.M == 0 || s.N == 0) return MLK_OK;
    // the direct-layout kernel addresses its output tile with 32-bit offsets
    // from the tile corner: rows up to bm - 1 apart at pitch ldc
    if (e->stages >= 1 && (int64_t)(e->bm - 1) * ldc + e->bn >= ((int64_t)1 << 31))
        return fail(MLK_ERR_CONFIG, "direct-layout tile: ldc %lld too large for its %d-row tile (32-bit offsets)",
                    (long long)ldc, e->bm);
    GemmArgs g = base_args(s, cfg);
    const int es = esize_in(s.dt);
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.C = C;
    g.ldc = ldc;
    g.scale_a = sa;
    g.scale_b = sb;
    g.bias = bias;
    g.vec_a = ((uintptr_t)A % 16 == 0) && ((lda * es) % 16 == 0);
    g.vec_b = ((uintptr_t)B % 16 == 0) && ((ldb * es) % 16 == 0);
    if (e->stages < 2 || s.K == 0) return run_gemm(e, g, s, C, s.M, s.N, ldc, st);
    const PackPlan pp = pack_plan(s, e, A, lda, B, ldb);
    if (((s.M - 1) * pp.lda2 + pp.Kp) * es >= ((int64_t)1 << 31) ||
        ((pp.Kp - 1) * pp.ldb2 + s.N) * es >= ((int64_t)1 << 31))
        return fail(MLK_ERR_CONFIG, "direct-to-LDS tile: an operand exceeds 2 GiB");
    if (!pp.pa && !pp.pb) return run_gemm(e, g, s, C, s.M, s.N, ldc, st);
    // the packed copies go to the caller's workspace when one is given (no
    // allocation, no scratch lock, capturable), else to the library's scratch
    ScratchUse scratch;
    void* ws = ext_ws;
    if (ext_ws) {
        if ((size_t)(pp.abytes + pp.bbytes) > ext_bytes)
            return fail(MLK_ERR_SHAPE, "operand packing needs %lld bytes of workspace, %zu available",
                        (long long)(pp.abytes + pp.bbytes), ext_bytes);
    } else {
        if (mlk_status rc = scratch.begin((size_t)(pp.abytes + pp.bbytes), st,
                                          "a direct-to-LDS tile with operand packing");
            rc != MLK_OK)
            return rc;
        ws = scratch.ptr();
    }
    PackJob jobs[2];
    int nj = 0;
    if (pp.pa) {
        jobs[nj++] = PackJob{A, ws, lda, pp.Kp, (int32_t)s.M, (int32_t)s.K, (int32_t)s.M, 0};
        g.A = ws;
    }
    if (pp.pb) {
        void* wb = (char*)ws + pp.abytes;
        jobs[nj++] = PackJob{B, wb, ldb, pp.Np, (int32_t)s.K, (int32_t)s.N, (int32_t)pp.Kp, 0};
        g.B = wb;
    }
    g.lda = pp.lda2;
    g.ldb = pp.ldb2;
    g.K = pp.Kp;
    g.vec_a = g.vec_b = 1;
    const hipError_t err = launch_pack_pair(jobs, nj, es, st);
    mlk_status r = err == hipSuccess ? run_gemm(e, g, s, C, s.M, s.N, ldc, st) : hip_fail(err, "operand packing");
    const mlk_status rel = scratch.end();
    return r != MLK_OK ? r : rel;
}

mlk_status launch_conv(const Shape& s, int64_t n, int64_t c, int64_t h, int64_t w, int64_t f,
                       int64_t kh, int64_t kw, int sh, int sw, int ph, int pw, int64_t ho,
                       int64_t wo, const void* x, const void* wt, void* y,
                       const mlk_tile_config& cfg, hipStream_t st, const ConvPrep* prep) {
    const KernelEntry* e = find_kernel(s.dt, 1, cfg);
    if (!e) return fail(MLK_ERR_CONFIG, "no kernel for configuration");
    GemmArgs g = base_args(s, cfg);
    const int es = esize_in(s.dt);
    g.A = wt;
    g.lda = c * kh * kw;
    g.B = x;
    g.ldb = 0;
    g.C = y;
    g.ldc = 0;
    g.vec_a = ((uintptr_t)wt % 16 == 0) && ((g.lda * es) % 16 == 0);
    g.vec_b = 0;
    g.cn = (int32_t)n;
    g.cc = (int32_t)c;
    g.ch = (int32_t)h;
    g.cw = (int32_t)w;
    g.ckh = (int32_t)kh;
    g.ckw = (int32_t)kw;
    g.csh = sh;
    g.csw = sw;
    g.cph = ph;
    g.cpw = pw;
    g.cho = (int32_t)ho;
    g.cwo = (int32_t)wo;
    if (is_direct(e)) {
        if (cfg.layout != 2) return fail(MLK_ERR_CONFIG, "the direct conv tile runs as layout 2");
        const hipError_t err = e->launch(g, 0, st);
        return err == hipSuccess ? MLK_OK : hip_fail(err, "direct conv launch");
    }
    const int epv = 16 / es;
    if (cfg.layout == 3) {
        if (!(e->launch_gather && c % epv == 0 && f <= 65535))
            return fail(MLK_ERR_CONFIG, "the channel-gather layout needs a register-loaded bf16 conv tile, C %% %d == 0 "
                        "and F <= 65535", epv);
        if (!prep && kh * kw != 1)
            if (mlk_status rc = refuse_under_capture(st, "the channel-gather conv layout without a plan"); rc != MLK_OK)
                return rc;
    } else if (cfg.layout == 1) {
        if (!(e->launch_nhwc && c % epv == 0 && (uintptr_t)x % 16 == 0 && (uintptr_t)wt % 16 == 0 &&
              n <= 65535 && f <= 65535))
            return fail(MLK_ERR_CONFIG, "channels-last layout needs C %% %d == 0, aligned x and w, N, F <= 65535", epv);
        if (!prep)
            if (mlk_status rc = refuse_under_capture(st, "the channels-last conv layout"); rc != MLK_OK) return rc;
    } else if (!e->launch) {
        return fail(MLK_ERR_CONFIG, "this conv tile runs only the channels-last layout (layout 1)");
    }
    if (g.atomic && !s.accumulate) {
        hipError_t z = launch_zero_matrix(y, n * f, ho * wo, ho * wo, 4, st);
        if (z != hipSuccess) return hip_fail(z, "zero output");
    }
    const int64_t nblk = (int64_t)g.tiles_m * g.tiles_n * g.split_k;
    // Channel-gather route: the kernel reads the NCHW input itself (8 channels
    // of one pixel per 16-byte LDS chunk); only the filter is needed as
    // F x KH x KW x C -- the plan's copy, the filter itself when 1 x 1, else
    // a transposed copy in the library's scratch buffer.
    if (cfg.layout == 3) {
        g.B = x;
        const void* a = prep ? prep->w_cl : kh * kw == 1 ? wt : nullptr;
        if (a) {
            g.A = a;
            g.vec_a = (uintptr_t)a % 16 == 0 && (g.lda * es) % 16 == 0;
            const hipError_t err = e->launch_gather(g, (int)nblk, st);
            return err == hipSuccess ? MLK_OK : hip_fail(err, "conv launch");
        }
        ScratchUse scratch;
        if (mlk_status rc = scratch.begin((size_t)(f * c * kh * kw) * es, st, "the channel-gather conv layout");
            rc != MLK_OK)
            return rc;
        hipError_t err = launch_transpose_pair(nullptr, nullptr, 0, 0, 0, wt, scratch.ptr(), f, c, kh * kw, es, st);
        if (err == hipSuccess) {
            g.A = scratch.ptr();
            g.vec_a = 1;
            err = e->launch_gather(g, (int)nblk, st);
        }
        const mlk_status rel = scratch.end();
        if (err != hipSuccess) return hip_fail(err, "conv launch");
        return rel;
    }
    // Channels-last route: with C a multiple of the 16-byte vector, transpose
    // x to NHWC and the filter to F x KH x KW x C in the library's scratch
    // buffer, so every operand load of the tile kernel is one aligned 16-byte
    // read.
    if (cfg.layout == 1 && prep) {
        // a bound convolution: its own NHWC buffer, its filter already transposed
        hipError_t err = launch_transpose_pair(x, prep->xn, n, c, h * w, nullptr, nullptr, 0, 0, 0, es, st);
        if (err == hipSuccess) {
            g.A = prep->w_cl;
            g.B = prep->xn;
            g.vec_a = 1;
            err = e->launch_nhwc(g, (int)nblk, st);
        }
        return err == hipSuccess ? MLK_OK : hip_fail(err, "conv launch");
    }
    if (cfg.layout == 1) {
        const size_t xb = ((size_t)(n * c * h * w) * es + 255) & ~(size_t)255;
        const size_t wb = (size_t)(f * c * kh * kw) * es;
        ScratchUse scratch;
        if (mlk_status rc = scratch.begin(xb + wb, st, "the channels-last conv layout"); rc != MLK_OK) return rc;
        hipError_t err = hipSuccess;
        uint8_t* xn = (uint8_t*)scratch.ptr();
        uint8_t* wn = xn + xb;
        // a 1 x 1 filter is already F x C; otherwise FCHW -> F x KH x KW x C
        // in the same launch as the input
        const bool w_as_is = kh * kw == 1;
        if ((err = launch_transpose_pair(x, xn, n, c, h * w, wt, wn, w_as_is ? 0 : f, c, kh * kw, es, st)) ==
            hipSuccess) {
            if (!w_as_is) wt = wn;
            g.A = wt;
            g.B = xn;
            g.vec_a = 1;
            err = e->launch_nhwc(g, (int)nblk, st);
        }
        const mlk_status rel = scratch.end();
        if (err != hipSuccess) return hip_fail(err, "conv launch");
        return rel;
    }
    hipError_t err = e->launch(g, (int)nblk, st);
    if (err != hipSuccess) return hip_fail(err, "kernel launch");
    return MLK_OK;
}

// ------------------------------------------------------------------ no-alloc workspace

// The workspace of mlk_matmul_noalloc: a fixed device array, one copy per
// device that loads the library, held until the process ends.  Host code
// never passes the array's name as an address: each device's copy is looked
// up once (hipGetSymbolAddress with that device current) and its address kept.
constexpr size_t kNoallocBytes = MLK_NOALLOC_WORKSPACE_BYTES;
static __device__ __align__(256) uint8_t noalloc_scratch[kNoallocBytes];

static std::mutex g_noalloc_mu;
static std::map<int, void*> g_noalloc_ptr;

static mlk_status noalloc_workspace(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(dev);
    if (it == g_noalloc_ptr.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(no-alloc workspace)");
        if (!p) return fail(MLK_ERR_HIP, "hipGetSymbolAddress(no-alloc workspace) returned NULL");
        it = g_noalloc_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return MLK_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace mlk

using namespace mlk;

extern "C" {

const char* mlk_status_str(mlk_status s) {
    switch (s) {
        case MLK_OK: return "MLK_OK";
        case MLK_ERR_NULL: return "MLK_ERR_NULL";
        case MLK_ERR_SHAPE: return "MLK_ERR_SHAPE";
        case MLK_ERR_LAYOUT: return "MLK_ERR_LAYOUT";
        case MLK_ERR_DTYPE: return "MLK_ERR_DTYPE";
        case MLK_ERR_CONFIG: return "MLK_ERR_CONFIG";
        case MLK_ERR_DB: return "MLK_ERR_DB";
        case MLK_ERR_HIP: return "MLK_ERR_HIP";
        case MLK_ERR_NOMEM: return "MLK_ERR_NOMEM";
        case MLK_ERR_ARG: return "MLK_ERR_ARG";
    }
    return "MLK_ERR_UNKNOWN";
}

const char* mlk_last_error(void) { return t_err.c_str(); }

const char* mlk_version(void) { return "mlk 0.1 (gfx950)"; }

static mlk_status matmul_impl(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                              const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                              int64_t ldc, const float* scale_a, const float* scale_b,
                              const float* bias, int accumulate, const mlk_tile_config* cfg,
                              void* stream, bool noalloc = false) {
    mlk_problem p;
    memset(&p, 0, sizeof p);
    p.op = MLK_OP_MATMUL;
    p.in = in;
    p.out = out;
    p.accumulate = accumulate ? 1 : 0;
    p.M = M;
    p.N = N;
    p.K = K;
    Shape s;
    mlk_status st = shape_of_problem(&p, &s);
    if (st != MLK_OK) return st;
    if (M > 0 && N > 0) {
        if (!C) return fail(MLK_ERR_NULL, "matmul: C is NULL");
        if (K > 0 && (!A || !B)) return fail(MLK_ERR_NULL, "matmul: A or B is NULL");
    }
    if (lda < std::max<int64_t>(K, 1) || ldb < std::max<int64_t>(N, 1) || ldc < std::max<int64_t>(N, 1))
        return fail(MLK_ERR_LAYOUT, "matmul: leading dimension too small (lda %lld >= K %lld, ldb %lld >= N, ldc %lld >= N %lld)",
                    (long long)lda, (long long)K, (long long)ldb, (long long)ldc, (long long)N);
    const int cs = s.out16 ? 2 : 4;  // bytes per element of C
    if (M > 0 && N > 0 && K > 0) {
        const int es = esize_in(s.dt);
        const size_t cb = (size_t)((M - 1) * ldc + N) * cs;
        const size_t ab = (size_t)((M - 1) * lda + K) * es;
        const size_t bb = (size_t)((K - 1) * ldb + N) * es;
        if (overlaps(C, cb, A, ab) || overlaps(C, cb, B, bb))
            return fail(MLK_ERR_LAYOUT, "matmul: C overlaps A or B");
    }
    if ((scale_a || scale_b) && s.dt != DT_F8)
        return fail(MLK_ERR_ARG, "matmul: scales apply to MLK_F8E4M3 inputs only");
    if (bias && M > 0 && N > 0) {
        if (s.dt == DT_I8) return fail(MLK_ERR_DTYPE, "matmul_bias: the bias applies to float outputs only");
        if (overlaps(C, (size_t)((M - 1) * ldc + N) * cs, bias, (size_t)N * 4))
            return fail(MLK_ERR_LAYOUT, "matmul_bias: C overlaps bias");
    }
    mlk_tile_config c;
    st = resolve(p, s, cfg, &c);
    if (st != MLK_OK) return st;
    if (M == 0 || N == 0) return MLK_OK;
    if (noalloc) {
        // packed operand copies go to the fixed device array: refuse what it cannot hold
        const int64_t need = dense_workspace_bytes(s, A, lda, B, ldb, c);
        if (need > (int64_t)kNoallocBytes)
            return fail(MLK_ERR_SHAPE,
                        "matmul_noalloc: operand packing for this shape and tile needs %lld bytes, more than "
                        "the %zu-byte no-alloc workspace; use operands with 16-byte rows and K a multiple of "
                        "the tile depth, or a tile without packing (stages 0 or 1)",
                        (long long)need, kNoallocBytes);
        void* ws = nullptr;
        if (need > 0)
            if (mlk_status r = noalloc_workspace(&ws); r != MLK_OK) return r;
        return launch_dense(s, A, lda, B, ldb, C, ldc, scale_a, scale_b, c, (hipStream_t)stream, bias, ws,
                            kNoallocBytes);
    }
    return launch_dense(s, A, lda, B, ldb, C, ldc, scale_a, scale_b, c, (hipStream_t)stream, bias);
}

mlk_status mlk_matmul(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                      const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                      int64_t ldc, const float* scale_a, const float* scale_b, int accumulate,
                      const mlk_tile_config* cfg, void* stream) {
    clear_error();
    return matmul_impl(in, out, M, N, K, A, lda, B, ldb, C, ldc, scale_a, scale_b, nullptr,
                       accumulate, cfg, stream);
}

mlk_status mlk_matmul_noalloc(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                              const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                              int64_t ldc, const float* scale_a, const float* scale_b, int accumulate,
                              const mlk_tile_config* cfg, void* stream) {
    clear_error();
    return matmul_impl(in, out, M, N, K, A, lda, B, ldb, C, ldc, scale_a, scale_b, nullptr,
                       accumulate, cfg, stream, true);
}

mlk_status mlk_matmul_bias(mlk_dtype in, mlk_dtype out, int64_t M, int64_t N, int64_t K,
                           const void* A, int64_t lda, const void* B, int64_t ldb,
                           const float* bias, void* C, int64_t ldc, const float* scale_a,
                           const float* scale_b, int accumulate, const mlk_tile_config* cfg,
                           void* stream) {
    clear_error();
    if (!bias && M > 0 && N > 0) return fail(MLK_ERR_NULL, "matmul_bias: bias is NULL");
    return matmul_impl(in, out, M, N, K, A, lda, B, ldb, C, ldc, scale_a, scale_b, bias,
                       accumulate, cfg, stream);
}

mlk_status mlk_conv2d_nchw_fchw(mlk_dtype in, mlk_dtype out, int64_t N, int64_t C, int64_t H,
                                int64_t W, int64_t F, int64_t KH, int64_t KW, int32_t sh,
                                int32_t sw, int32_t ph, int32_t pw, const void* x, const void* w,
                                void* y, int accumulate, const mlk_tile_config* cfg, void* stream) {
    clear_error();
    mlk_problem p;
    memset(&p, 0, sizeof p);
    p.op = MLK_OP_CONV2D;
    p.in = in;
    p.out = out;
    p.accumulate = accumulate ? 1 : 0;
    p.n = N;
    p.c = C;
    p.h = H;
    p.w = W;
    p.f = F;
    p.kh = KH;
    p.kw = KW;
    p.sh = sh;
    p.sw = sw;
    p.ph = ph;
    p.pw = pw;
    Shape s;
    mlk_status st = shape_of_problem(&p, &s);
    if (st != MLK_OK) return st;
    if (!x || !w || !y) return fail(MLK_ERR_NULL, "conv2d: x, w or y is NULL");
    const int64_t ho = conv_out(H, KH, sh, ph), wo = conv_out(W, KW, sw, pw);
    const int es = esize_in(s.dt);
    const size_t yb = (size_t)(N * F * ho * wo) * 4;
    if (overlaps(y, yb, x, (size_t)(N * C * H * W) * es) || overlaps(y, yb, w, (size_t)(F * C * KH * KW) * es))
        return fail(MLK_ERR_LAYOUT, "conv2d: y overlaps x or w");
    mlk_tile_config c;
    st = resolve(p, s, cfg, &c);
    if (st != MLK_OK) return st;
    if (cfg_is_zero(cfg) && c.layout == 3 && KH * KW != 1) {
        // the chosen channel gather would transpose the filter into scratch
        // memory, which a capturing stream cannot take: the plain tile instead
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const hipError_t e = hipStreamIsCapturing((hipStream_t)stream, &cs);
        if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
        if (cs != hipStreamCaptureStatusNone) c = heuristic_config(s, p.op, false);
    }
    if (c.layout == 1 && cfg_is_zero(cfg) &&
        ((uintptr_t)x % 16 != 0 || (uintptr_t)w % 16 != 0 || N > 65535 || F > 65535))
        c.layout = 0;
    return launch_conv(s, N, C, H, W, F, KH, KW, sh, sw, ph, pw, ho, wo, x, w, y, c,
                       (hipStream_t)stream);
}

}  // extern "C"

// A convolution bound to its shape, configuration and filter.
struct mlk_conv_plan {
    mlk::Shape s;
    int64_t n = 0, c = 0, h = 0, w = 0, f = 0, kh = 0, kw = 0, ho = 0, wo = 0;
    int32_t sh = 1, sw = 1, ph = 0, pw = 0;
    mlk_tile_config cfg{};
    const void* filter = nullptr;  // the caller's FCHW filter
    void* buf = nullptr;           // channels-last layout: NHWC input copy, then the transposed filter
                                   // (channel-gather layout: the transposed filter only)
    size_t xb = 0;                 // bytes of the input copy (256-byte multiple; 0 for channel gather)
    int device = 0;
};

namespace {

// the filter in F x KH x KW x C for a channels-last or channel-gather plan
// (a 1 x 1 filter is used as it is)
mlk_status plan_transpose_filter(const mlk_conv_plan* pl, hipStream_t st) {
    if ((pl->cfg.layout != 1 && pl->cfg.layout != 3) || pl->kh * pl->kw == 1) return MLK_OK;
    const int es = esize_in(pl->s.dt);
    const hipError_t e = launch_transpose_pair(nullptr, nullptr, 0, 0, 0, pl->filter, (char*)pl->buf + pl->xb,
                                               pl->f, pl->c, pl->kh * pl->kw, es, st);
    return e == hipSuccess ? MLK_OK : hip_fail(e, "conv plan filter transpose");
}

}  // namespace

extern "C" {

mlk_status mlk_conv2d_plan_create(mlk_dtype in, mlk_dtype out, int64_t N, int64_t C, int64_t H, int64_t W,
                                  int64_t F, int64_t KH, int64_t KW, int32_t sh, int32_t sw, int32_t ph,
                                  int32_t pw, const void* w, int accumulate, const mlk_tile_config* cfg,
                                  void* stream, mlk_conv_plan** plan) {
    clear_error();
    if (!plan) return fail(MLK_ERR_NULL, "conv plan: plan is NULL");
    *plan = nullptr;
    mlk_problem p;
    memset(&p, 0, sizeof p);
    p.op = MLK_OP_CONV2D;
    p.in = in;
    p.out = out;
    p.accumulate = accumulate ? 1 : 0;
    p.n = N;
    p.c = C;
    p.h = H;
    p.w = W;
    p.f = F;
    p.kh = KH;
    p.kw = KW;
    p.sh = sh;
    p.sw = sw;
    p.ph = ph;
    p.pw = pw;
    Shape s;
    mlk_status st = shape_of_problem(&p, &s);
    if (st != MLK_OK) return st;
    if (!w) return fail(MLK_ERR_NULL, "conv plan: w is NULL");
    mlk_tile_config c;
    st = resolve(p, s, cfg, &c);
    if (st != MLK_OK) return st;
    if (c.layout == 1 && (uintptr_t)w % 16 != 0) {
        if (!cfg_is_zero(cfg)) return fail(MLK_ERR_CONFIG, "conv plan: the channels-last layout needs an aligned w");
        c.layout = 0;
    }
    if (c.layout == 1 && (N > 65535 || F > 65535)) {
        if (!cfg_is_zero(cfg)) return fail(MLK_ERR_CONFIG, "conv plan: the channels-last layout needs N, F <= 65535");
        c.layout = 0;
    }
    const hipStream_t hs = (hipStream_t)stream;
    // the plan's buffers are allocated here, so creation cannot be captured
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(hs, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(MLK_ERR_CONFIG, "conv plan: create plans outside stream capture (runs may be captured)");
    mlk_conv_plan* pl = new mlk_conv_plan();
    pl->s = s;
    pl->n = N;
    pl->c = C;
    pl->h = H;
    pl->w = W;
    pl->f = F;
    pl->kh = KH;
    pl->kw = KW;
    pl->ho = conv_out(H, KH, sh, ph);
    pl->wo = conv_out(W, KW, sw, pw);
    pl->sh = sh;
    pl->sw = sw;
    pl->ph = ph;
    pl->pw = pw;
    pl->cfg = c;
    pl->filter = w;
    if ((e = hipGetDevice(&pl->device)) != hipSuccess) {
        delete pl;
        return hip_fail(e, "hipGetDevice");
    }
    const size_t wb = KH * KW == 1 ? 0 : (size_t)(F * C * KH * KW) * esize_in(s.dt);
    if (c.layout == 1 || (c.layout == 3 && wb > 0)) {
        pl->xb = c.layout == 1 ? ((size_t)(N * C * H * W) * esize_in(s.dt) + 255) & ~(size_t)255 : 0;
        if ((e = hipMalloc(&pl->buf, pl->xb + wb)) != hipSuccess) {
            delete pl;
            return hip_fail(e, "conv plan buffers");
        }
        if ((st = plan_transpose_filter(pl, hs)) != MLK_OK) {
            mlk_conv2d_plan_destroy(pl);
            return st;
        }
    }
    *plan = pl;
    return MLK_OK;
}

mlk_status mlk_conv2d_plan_update_filter(mlk_conv_plan* plan, void* stream) {
    clear_error();
    if (!plan) return fail(MLK_ERR_NULL, "conv plan is NULL");
    return plan_transpose_filter(plan, (hipStream_t)stream);
}

mlk_status mlk_conv2d_plan_run(const mlk_conv_plan* plan, const void* x, void* y, void* stream) {
    clear_error();
    if (!plan) return fail(MLK_ERR_NULL, "conv plan is NULL");
    if (!x || !y) return fail(MLK_ERR_NULL, "conv plan: x or y is NULL");
    const mlk_conv_plan& pl = *plan;
    const int es = esize_in(pl.s.dt);
    const size_t yb = (size_t)(pl.n * pl.f * pl.ho * pl.wo) * 4;
    if (overlaps(y, yb, x, (size_t)(pl.n * pl.c * pl.h * pl.w) * es) ||
        overlaps(y, yb, pl.filter, (size_t)(pl.f * pl.c * pl.kh * pl.kw) * es))
        return fail(MLK_ERR_LAYOUT, "conv plan: y overlaps x or w");
    if (pl.cfg.layout == 1 && (uintptr_t)x % 16 != 0)
        return fail(MLK_ERR_LAYOUT, "conv plan: its channels-last layout needs a 16-byte aligned x");
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != pl.device) return fail(MLK_ERR_ARG, "conv plan: created on device %d, run on device %d", pl.device, dev);
    ConvPrep prep{pl.buf, pl.kh * pl.kw == 1 ? pl.filter : (const void*)((const char*)pl.buf + pl.xb)};
    return launch_conv(pl.s, pl.n, pl.c, pl.h, pl.w, pl.f, pl.kh, pl.kw, pl.sh, pl.sw, pl.ph, pl.pw, pl.ho, pl.wo, x,
                       pl.filter, y, pl.cfg, (hipStream_t)stream,
                       pl.cfg.layout == 1 || pl.cfg.layout == 3 ? &prep : nullptr);
}

mlk_status mlk_conv2d_plan_config(const mlk_conv_plan* plan, mlk_tile_config* cfg) {
    clear_error();
    if (!plan || !cfg) return fail(MLK_ERR_NULL, "conv plan: NULL pointer");
    *cfg = plan->cfg;
    return MLK_OK;
}

void mlk_conv2d_plan_destroy(mlk_conv_plan* plan) {
    if (!plan) return;
    if (plan->buf) (void)hipFree(plan->buf);
    delete plan;
}

mlk_status mlk_mfma_rate(mlk_dtype in, int64_t iters, float* out, int64_t out_len, int64_t* flops, void* stream) {
    clear_error();
    if (in != MLK_BF16 && in != MLK_F8E4M3) return fail(MLK_ERR_DTYPE, "mfma_rate: MLK_BF16 or MLK_F8E4M3");
    if (iters < 1 || iters > 16384) return fail(MLK_ERR_ARG, "mfma_rate: iters must be in [1, 16384]");
    if (!out || !flops) return fail(MLK_ERR_NULL, "mfma_rate: out or flops is NULL");
    if (out_len < 1) return fail(MLK_ERR_SHAPE, "mfma_rate: out_len must be >= 1");
    const int blocks = 2 * device_cus();
    const int64_t waves = (int64_t)blocks * 4;
    if (out_len < waves)
        return fail(MLK_ERR_SHAPE, "mfma_rate: out holds %lld floats, the launch writes %lld", (long long)out_len,
                    (long long)waves);
    *flops = waves * iters * 8 * (in == MLK_BF16 ? 2LL * 16 * 16 * 32 : 2LL * 16 * 16 * 128);
    const hipError_t e = launch_mfma_rate(in == MLK_BF16 ? DT_BF16 : DT_F8, iters, blocks, out, (hipStream_t)stream);
    return e == hipSuccess ? MLK_OK : hip_fail(e, "mfma_rate launch");
}

mlk_status mlk_quantize(mlk_dtype out, int64_t n, const float* x, void* q, float* scale,
                        void* stream) {
    clear_error();
    if (out != MLK_BF16 && out != MLK_F8E4M3)
        return fail(MLK_ERR_DTYPE, "quantize: output must be MLK_BF16 or MLK_F8E4M3");
    if (n < 0) return fail(MLK_ERR_SHAPE, "quantize: n < 0");
    if (out == MLK_F8E4M3 && !scale) return fail(MLK_ERR_NULL, "quantize: e4m3 needs a scale output");
    if (n > 0 && (!x || !q)) return fail(MLK_ERR_NULL, "quantize: x or q is NULL");
    if (n > 0 && overlaps(x, (size_t)n * 4, q, (size_t)n * (out == MLK_BF16 ? 2 : 1)))
        return fail(MLK_ERR_LAYOUT, "quantize: q overlaps x");
    const hipStream_t st = (hipStream_t)stream;
    if (out == MLK_BF16) {
        const hipError_t e = launch_quant_bf16(x, n, (uint16_t*)q, st);
        return e == hipSuccess ? MLK_OK : hip_fail(e, "quantize launch");
    }
    ScratchUse scratch;
    if (n > 0) {
        if (mlk_status rc = scratch.begin(sizeof(float) * quant_e4m3_parts(), st, "e4m3 quantisation");
            rc != MLK_OK)
            return rc;
    }
    hipError_t e = launch_quant_e4m3_fused(x, n, (uint8_t*)q, scale, st);
    if (e == hipErrorNotSupported) e = launch_quant_e4m3(x, n, (uint8_t*)q, scale, (float*)scratch.ptr(), st);
    const mlk_status rel = scratch.end();
    if (e != hipSuccess) return hip_fail(e, "quantize launch");
    return rel;
}

mlk_status mlk_err_stats(mlk_dtype c_dtype, int64_t n, const void* c, const double* r,
                         const double* bound, double* out, void* stream) {
    clear_error();
    if (c_dtype != MLK_F32 && c_dtype != MLK_I32)
        return fail(MLK_ERR_DTYPE, "err_stats: c must be MLK_F32 or MLK_I32");
    if (n < 0) return fail(MLK_ERR_SHAPE, "err_stats: n < 0");
    if (!out || (n > 0 && (!c || !r))) return fail(MLK_ERR_NULL, "err_stats: NULL pointer");
    const hipStream_t st = (hipStream_t)stream;
    ScratchUse scratch;
    if (mlk_status rc = scratch.begin(sizeof(double) * 4 * err_stats_parts(), st, "err_stats"); rc != MLK_OK)
        return rc;
    const hipError_t e = launch_err_stats(c_dtype == MLK_I32, n, c, r, bound, out, (double*)scratch.ptr(), st);
    const mlk_status rel = scratch.end();
    if (e != hipSuccess) return hip_fail(e, "err_stats launch");
    return rel;
}

mlk_status mlk_mlp_forward(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* params,
                           const float* X, float* y, void* stream) {
    clear_error();
    if (B < 0 || D0 < 1 || H1 < 1 || H2 < 1 || D0 > 4096 || H1 > 4096 || H2 > 4096)
        return fail(MLK_ERR_SHAPE, "mlp: bad sizes");
    if (B > 0 && (!params || !X || !y)) return fail(MLK_ERR_NULL, "mlp: NULL pointer");
    if (B == 0) return MLK_OK;
    const hipStream_t st = (hipStream_t)stream;
    ScratchUse scratch;
    if (mlk_status rc = scratch.begin(sizeof(float) * mlp_forward_words(B, H1, H2), st, "mlp forward"); rc != MLK_OK)
        return rc;
    const hipError_t e = launch_mlp_forward(B, D0, H1, H2, params, X, y, (float*)scratch.ptr(), st);
    const mlk_status rel = scratch.end();
    if (e != hipSuccess) return hip_fail(e, "mlp forward");
    return rel;
}

mlk_status mlk_mlp_loss_grad(int64_t B, int64_t D0, int64_t H1, int64_t H2,
                             const float* params, const float* X, const float* t, float* grad,
                             float* loss, void* stream) {
    clear_error();
    if (B < 1 || D0 < 1 || H1 < 1 || H2 < 1 || D0 > 4096 || H1 > 4096 || H2 > 4096)
        return fail(MLK_ERR_SHAPE, "mlp: bad sizes");
    if (!params || !X || !t || !grad || !loss) return fail(MLK_ERR_NULL, "mlp: NULL pointer");
    const hipStream_t st = (hipStream_t)stream;
    ScratchUse scratch;
    if (mlk_status rc = scratch.begin(sizeof(float) * mlp_loss_grad_words(B, H1, H2), st, "mlp loss/grad");
        rc != MLK_OK)
        return rc;
    const hipError_t e = launch_mlp_loss_grad(B, D0, H1, H2, params, X, t, grad, loss, (float*)scratch.ptr(), st);
    const mlk_status rel = scratch.end();
    if (e != hipSuccess) return hip_fail(e, "mlp loss/grad");
    return rel;
}

mlk_status mlk_adam_step(int64_t n, float* params, const float* grad, float* m, float* v,
                         float lr, float beta1, float beta2, float eps, int64_t t, void* stream) {
    clear_error();
    if (n < 0) return fail(MLK_ERR_SHAPE, "adam: n < 0");
    if (t < 1) return fail(MLK_ERR_ARG, "adam: step t must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(MLK_ERR_ARG, "adam: bad hyper-parameters");
    if (n > 0 && (!params || !grad || !m || !v)) return fail(MLK_ERR_NULL, "adam: NULL pointer");
    hipError_t e = launch_adam(n, params, grad, m, v, lr, beta1, beta2, eps, t, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adam");
    return MLK_OK;
}

mlk_status mlk_config_legal(const mlk_problem* p, const mlk_tile_config* cfg) {
    clear_error();
    if (!cfg) return fail(MLK_ERR_NULL, "cfg is NULL");
    Shape s;
    mlk_status st = shape_of_problem(p, &s);
    if (st != MLK_OK) return st;
    mlk_tile_config c = *cfg;
    if (c.group_m == 0) c.group_m = 1;
    return check_config(s, p->op, c);
}

int32_t mlk_config_count(const mlk_problem* p) {
    clear_error();
    Shape s;
    if (shape_of_problem(p, &s) != MLK_OK) return -1;
    return (int32_t)enumerate_configs(p, s).size();
}

mlk_status mlk_config_get(const mlk_problem* p, int32_t i, mlk_tile_config* cfg) {
    clear_error();
    if (!cfg) return fail(MLK_ERR_NULL, "cfg is NULL");
    Shape s;
    mlk_status st = shape_of_problem(p, &s);
    if (st != MLK_OK) return st;
    std::vector<mlk_tile_config> v = enumerate_configs(p, s);
    if (i < 0 || i >= (int32_t)v.size()) return fail(MLK_ERR_ARG, "config index %d out of range [0, %zu)", i, v.size());
    *cfg = v[i];
    return MLK_OK;
}

mlk_status mlk_config_set_default(const mlk_problem* p, const mlk_tile_config* cfg) {
    clear_error();
    mlk_status st = mlk_config_legal(p, cfg);
    if (st != MLK_OK) return st;
    mlk_tile_config c = *cfg;
    if (c.group_m == 0) c.group_m = 1;
    store_default(problem_key(p), c);
    return MLK_OK;
}

}  // extern "C"
