// k_direct.hip -- direct (stencil) convolution for layers with few filters.
//
// When F (the GEMM view's M) is tiny -- the paper's own workload is one input
// channel, three 3x3 filters over a 1280 x 1280 image -- an MFMA tile is
// mostly padding rows and the layer is a stream over the image: each input
// element is read about once and each output element read and written once.
// This form keeps it that way.  A workgroup owns a TH x TW block of output
// pixels of one image and all F filters (F <= kDirectMaxF): per input
// channel it stages the block's input window (with its halo, zero outside the
// image) and the channel's F x KH x KW filter taps in LDS with contiguous
// loads, then every thread accumulates its pixels' F sums over the KH x KW
// taps (the taps are LDS broadcasts: every lane reads the same word).  Sums
// run over c, then kh, then kw, in the order of the definition, in fp32,
// starting from y (C += conv).  Output rows are written by consecutive lanes
// along ow.  Each pixel's sums are held for a bucket of 4, 8 or 16 filters,
// the smallest that holds F, picked at launch.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mlk {

namespace {

__device__ inline float load_val(const float* p, int64_t i) { return p[i]; }
__device__ inline float load_val(const uint16_t* p, int64_t i) { return __uint_as_float((uint32_t)p[i] << 16); }

// FB: filters held per pixel (a bucket of 4, 8 or 16 at least F): the sums and
// the taps of filters past F are not formed at all.
template <typename T, int TH, int TW, int FB>
__global__ __launch_bounds__(256) void k_conv_direct(GemmArgs g) {
    static_assert(TW == 64 && TH % 4 == 0, "one wave per output row segment of 64 pixels");
    static_assert(FB <= kDirectMaxF, "filter bucket");
    constexpr int P = TH * TW / 256;  // output pixels per thread (rows tid/64 + 4q)
    __shared__ float patch[direct_patch(TH, TW)];
    __shared__ float taps[FB * kDirectMaxTap * kDirectMaxTap];
    const T* __restrict__ x = (const T*)g.B;
    const T* __restrict__ w = (const T*)g.A;
    float* __restrict__ y = (float*)g.C;
    const int F = (int)g.M, C = g.cc, H = g.ch, W = g.cw, KH = g.ckh, KW = g.ckw;
    const int SH = g.csh, SW = g.csw, HO = g.cho, WO = g.cwo;
    const int img = blockIdx.z;
    const int oh0 = blockIdx.y * TH, ow0 = blockIdx.x * TW;
    const int PH = (TH - 1) * SH + KH, PW = (TW - 1) * SW + KW;
    const int ih0 = oh0 * SH - g.cph, iw0 = ow0 * SW - g.cpw;
    const int tid = threadIdx.x, col = tid & 63, row = tid >> 6;

    float acc[P][FB];
    const int64_t hw_out = (int64_t)HO * WO;
    float* ybase = y + (int64_t)img * F * hw_out;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int oh = oh0 + row + 4 * q, ow = ow0 + col;
        const bool in = oh < HO && ow < WO;
#pragma unroll
        for (int f = 0; f < FB; ++f)
            acc[q][f] = (in && f < F && g.accumulate) ? ybase[f * hw_out + (int64_t)oh * WO + ow] : 0.0f;
    }

    const T* xbase = x + (int64_t)img * C * H * W;
    for (int c = 0; c < C; ++c) {
        __syncthreads();  // the previous channel's window is no longer read
        const T* xc = xbase + (int64_t)c * H * W;
        for (int i = tid; i < PH * PW; i += 256) {
            const int pr = i / PW, pc = i - pr * PW;
            const int ih = ih0 + pr, iw = iw0 + pc;
            patch[i] = ((unsigned)ih < (unsigned)H && (unsigned)iw < (unsigned)W) ? load_val(xc, (int64_t)ih * W + iw)
                                                                                  : 0.0f;
        }
        // taps[(kh * KW + kw) * FB + f] = w[f][c][kh][kw] (0 past F)
        const int KK = KH * KW;
        for (int i = tid; i < KK * FB; i += 256) {
            const int f = i % FB, t = i / FB;
            taps[i] = f < F ? load_val(w, ((int64_t)f * C + c) * KK + t) : 0.0f;
        }
        __syncthreads();
        for (int kh = 0; kh < KH; ++kh)
            for (int kw = 0; kw < KW; ++kw) {
                float wt[FB];
                const float* tk = taps + (kh * KW + kw) * FB;
#pragma unroll
                for (int f = 0; f < FB; ++f) wt[f] = tk[f];
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const float xv = patch[((row + 4 * q) * SH + kh) * PW + col * SW + kw];
#pragma unroll
                    for (int f = 0; f < FB; ++f) acc[q][f] = __builtin_fmaf(xv, wt[f], acc[q][f]);
                }
            }
    }

#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int oh = oh0 + row + 4 * q, ow = ow0 + col;
        if (oh >= HO || ow >= WO) continue;
#pragma unroll
        for (int f = 0; f < FB; ++f)
            if (f < F) ybase[f * hw_out + (int64_t)oh * WO + ow] = acc[q][f];
    }
}

template <typename T, int TH, int TW>
hipError_t launch_conv_direct(const GemmArgs& g, int, hipStream_t s) {
    const dim3 grid((unsigned)((g.cwo + TW - 1) / TW), (unsigned)((g.cho + TH - 1) / TH), (unsigned)g.cn);
    // F <= kDirectMaxF is checked by the host before any launch
    if (g.M <= 4)
        hipLaunchKernelGGL((k_conv_direct<T, TH, TW, 4>), grid, dim3(256), 0, s, g);
    else if (g.M <= 8)
        hipLaunchKernelGGL((k_conv_direct<T, TH, TW, 8>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_conv_direct<T, TH, TW, 16>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace

#define MLK_ENTRY_DIRECT(DT, T, TH, TW)                                                                  \
    KernelEntry {                                                                                        \
        DT, 1, 0, TH, TW, 1, 0, 0, (int)(sizeof(float) * (direct_patch(TH, TW) + kDirectMaxF * kDirectMaxTap * kDirectMaxTap)), \
            256, &launch_conv_direct<T, TH, TW>,                                                         \
            nullptr, nullptr, nullptr                                                                    \
    }

const KernelEntry* kernels_direct(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY_DIRECT(DT_F32, float, 4, 64),
        MLK_ENTRY_DIRECT(DT_F32, float, 8, 64),
        MLK_ENTRY_DIRECT(DT_F32, float, 16, 64),
        MLK_ENTRY_DIRECT(DT_F32, float, 32, 64),
        MLK_ENTRY_DIRECT(DT_BF16, uint16_t, 4, 64),
        MLK_ENTRY_DIRECT(DT_BF16, uint16_t, 8, 64),
        MLK_ENTRY_DIRECT(DT_BF16, uint16_t, 16, 64),
        MLK_ENTRY_DIRECT(DT_BF16, uint16_t, 32, 64),
    };
    *n = (int)(sizeof t / sizeof t[0]);
    return t;
}

}  // namespace mlk
