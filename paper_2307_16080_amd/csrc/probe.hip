// probe.hip -- the matrix cores' sustained rate: every wave of a grid that
// fills the device issues back-to-back MFMAs on register operands (no memory
// traffic inside the loop), eight independent accumulator chains per wave so
// that no MFMA waits for the previous one's result.  The rate this reaches is
// the practical ceiling a GEMM kernel is measured against, beside the
// datasheet peak (which assumes the 2.4 GHz peak engine clock throughout).
//
// Every operand element is 1.0 and chain c starts at c, so each element of
// chain c after `iters` steps is exactly c + iters * k (k = 32 for bf16, 128
// for e4m3), and each wave stores the sum of its eight chains' first
// element: 28 + 8 * iters * k, exact in fp32 while below 2^24.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace mlk {

namespace {

constexpr int kChains = 8;

template <int DT>
__global__ __launch_bounds__(256) void k_mfma_rate(int64_t iters, uint32_t one, float* __restrict__ out) {
    // distinct starting values (per chain and per element) keep the chains
    // distinct computations in disjoint registers
    f4_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f4_t{(float)c, c + 0.25f, c + 0.5f, c + 0.75f};
    if constexpr (DT == DT_BF16) {
        // Written as one asm statement per step: built from the builtin, this
        // loop gets its accumulators rotated through extra registers every
        // step (~50 register moves per eight MFMAs), which would measure the
        // moves.  The eight MFMAs accumulate in place, each chain's next step
        // seven MFMAs later; the wait states before the first step (after the
        // accumulators are set) and after the last (before they are read)
        // are the asm's own, tied to the accumulators so nothing moves past them.
        const __bf16 x = __builtin_bit_cast(__bf16, (uint16_t)one);
        bf8_t a = bf8_t{x, x, x, x, x, x, x, x};
        asm volatile("s_nop 4"
                     : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
                       "+v"(acc[6]), "+v"(acc[7]), "+v"(a));
        for (int64_t it = 0; it < iters; ++it) {
            asm volatile(
                "v_mfma_f32_16x16x32_bf16 %0, %8, %8, %0\n\t"
                "v_mfma_f32_16x16x32_bf16 %1, %8, %8, %1\n\t"
                "v_mfma_f32_16x16x32_bf16 %2, %8, %8, %2\n\t"
                "v_mfma_f32_16x16x32_bf16 %3, %8, %8, %3\n\t"
                "v_mfma_f32_16x16x32_bf16 %4, %8, %8, %4\n\t"
                "v_mfma_f32_16x16x32_bf16 %5, %8, %8, %5\n\t"
                "v_mfma_f32_16x16x32_bf16 %6, %8, %8, %6\n\t"
                "v_mfma_f32_16x16x32_bf16 %7, %8, %8, %7"
                : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
                  "+v"(acc[6]), "+v"(acc[7])
                : "v"(a));
        }
        asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7"
                     : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
                       "+v"(acc[6]), "+v"(acc[7]));
    } else {
        const int w = (int)(one * 0x01010101u);  // four e4m3 codes per register
        const i8_t a = i8_t{w, w, w, w, w, w, w, w};
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, a, acc[c], 0, 0, 0, 127, 0, 127);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0];
    if ((threadIdx.x & 63) == 0) out[blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64] = s;
}

}  // namespace

// `blocks` workgroups of four waves; out receives one value per wave
hipError_t launch_mfma_rate(int dt, int64_t iters, int blocks, float* out, hipStream_t s) {
    if (dt == DT_BF16)
        hipLaunchKernelGGL(k_mfma_rate<DT_BF16>, dim3(blocks), dim3(256), 0, s, iters, 0x3F80u, out);
    else
        hipLaunchKernelGGL(k_mfma_rate<DT_F8>, dim3(blocks), dim3(256), 0, s, iters, 0x38u, out);
    return hipGetLastError();
}

}  // namespace mlk
