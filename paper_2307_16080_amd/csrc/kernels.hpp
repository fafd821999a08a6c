// kernels.hpp -- kernel-instance registry shared by the host code and the
// per-dtype instantiation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_fast.hpp"
#include "gemm_tile.hpp"

namespace mlk {

// One (GEMM, tile) work item of a persistent launch.
struct Task {
    int32_t gemm, tm, tn, kz;
};

typedef hipError_t (*launch_fn)(const GemmArgs& g, int nblk, hipStream_t s);
typedef hipError_t (*persist_fn)(const GemmArgs* gemms, const Task* tasks,
                                 const int32_t* bounds, int nblk, hipStream_t s);

// A compiled tile configuration.
struct KernelEntry {
    int dt;        // DT_*
    int conv;      // 1: implicit-GEMM convolution operand policy
    int stages;    // 0: register-staged; >= 2: direct-to-LDS ring of that many stages
    int bm, bn, bk;
    int wm, wn;
    int lds_bytes;
    int threads;
    launch_fn launch;
    persist_fn persist;  // null where no persistent variant is built
    launch_fn launch_nhwc;  // conv entries: the channels-last variant (CONV = 2)
};

template <int DT, int BM, int BN, int KB, int WM, int WN, int CONV>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(GemmArgs g) {
    typedef Tile<DT, BM, BN, KB, WM, WN, CONV> TL;
    __shared__ __attribute__((aligned(16))) uint8_t lds[TL::LDS_BYTES];
    int tm, tn, kz;
    tile_coords(g, blockIdx.x, gridDim.x, tm, tn, kz);
    TL::run(g, tm, tn, kz, lds);
}

// Persistent variant: workgroup b runs tasks [bounds[b], bounds[b+1]) in order.
template <int DT, int BM, int BN, int KB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_persist(const GemmArgs* gemms,
                                                               const Task* tasks,
                                                               const int32_t* bounds) {
    typedef Tile<DT, BM, BN, KB, WM, WN, 0> TL;
    __shared__ __attribute__((aligned(16))) uint8_t lds[TL::LDS_BYTES];
    const int b = blockIdx.x;
    const int t0 = bounds[b], t1 = bounds[b + 1];
    for (int t = t0; t < t1; ++t) {
        const Task tk = tasks[t];
        const GemmArgs g = gemms[tk.gemm];
        TL::run(g, tk.tm, tk.tn, tk.kz, lds);
        __syncthreads();
    }
}

template <int DT, int BM, int BN, int WM, int WN, int STAGES>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_fast(GemmArgs g) {
    typedef FastGemm<DT, BM, BN, WM, WN, STAGES> TL;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TL::LDS_BYTES];
    int tm, tn, kz;
    tile_coords(g, blockIdx.x, gridDim.x, tm, tn, kz);
    TL::run(g, tm, tn, kz, lds);
}

template <int DT, int BM, int BN, int WM, int WN, int STAGES>
hipError_t launch_fast(const GemmArgs& g, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm_fast<DT, BM, BN, WM, WN, STAGES>), dim3(nblk), dim3(64 * WM * WN), 0,
                       s, g);
    return hipGetLastError();
}

template <int DT, int BM, int BN, int KB, int WM, int WN, int CONV>
hipError_t launch_gemm(const GemmArgs& g, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm<DT, BM, BN, KB, WM, WN, CONV>), dim3(nblk), dim3(64 * WM * WN), 0,
                       s, g);
    return hipGetLastError();
}

template <int DT, int BM, int BN, int KB, int WM, int WN>
hipError_t launch_persist(const GemmArgs* gemms, const Task* tasks, const int32_t* bounds,
                          int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm_persist<DT, BM, BN, KB, WM, WN>), dim3(nblk), dim3(64 * WM * WN),
                       0, s, gemms, tasks, bounds);
    return hipGetLastError();
}

#define MLK_ENTRY(DT, BM, BN, KB, WM, WN, CONV)                                              \
    KernelEntry {                                                                            \
        DT, (CONV) ? 1 : 0, 0, BM, BN, (KB) / Traits<DT>::ES, WM, WN,                          \
            Tile<DT, BM, BN, KB, WM, WN, (CONV) ? 1 : 0>::LDS_BYTES, 64 * (WM) * (WN),         \
            &launch_gemm<DT, BM, BN, KB, WM, WN, (CONV) ? 1 : 0>, nullptr,                     \
            (CONV) ? &launch_gemm<DT, BM, BN, KB, WM, WN, 2> : nullptr                        \
    }

#define MLK_ENTRY_P(DT, BM, BN, KB, WM, WN)                                                  \
    KernelEntry {                                                                            \
        DT, 0, 0, BM, BN, (KB) / Traits<DT>::ES, WM, WN,                                     \
            Tile<DT, BM, BN, KB, WM, WN, 0>::LDS_BYTES, 64 * (WM) * (WN),                    \
            &launch_gemm<DT, BM, BN, KB, WM, WN, 0>, &launch_persist<DT, BM, BN, KB, WM, WN>,  \
            nullptr                                                                          \
    }

#define MLK_ENTRY_FAST(DT, BM, BN, WM, WN, STAGES)                                           \
    KernelEntry {                                                                            \
        DT, 0, STAGES, BM, BN, FastGemm<DT, BM, BN, WM, WN, STAGES>::BK, WM, WN,              \
            FastGemm<DT, BM, BN, WM, WN, STAGES>::LDS_BYTES, 64 * (WM) * (WN),               \
            &launch_fast<DT, BM, BN, WM, WN, STAGES>, nullptr, nullptr                       \
    }

// Tables defined by the instantiation units (host functions: the tables hold
// host launch functions, so they must not exist in the device pass).
const KernelEntry* kernels_f32(int* n);
const KernelEntry* kernels_bf16(int* n);
const KernelEntry* kernels_i8(int* n);
const KernelEntry* kernels_f8(int* n);
const KernelEntry* kernels_conv(int* n);
const KernelEntry* kernels_fast(int* n);

// Elementwise / reduction launchers (quant.hip, reduce.hip, mlp.hip).
hipError_t launch_zero_matrix(void* C, int64_t M, int64_t N, int64_t ldc, int esize,
                              hipStream_t s);
hipError_t launch_quant_bf16(const float* x, int64_t n, uint16_t* q, hipStream_t s);
hipError_t launch_quant_e4m3(const float* x, int64_t n, uint8_t* q, float* scale,
                             hipStream_t s);
hipError_t launch_err_stats(int c_is_int, int64_t n, const void* c, const double* r,
                            const double* bound, double* out, hipStream_t s);
hipError_t launch_fill_random(void* p, int64_t n, int dt, uint64_t seed, hipStream_t s);
// batch of [rows x cols] matrices -> [cols x rows] (NCHW -> NHWC, FCHW -> FHWC)
hipError_t launch_transpose_batched(const void* in, void* out, int64_t batch, int64_t rows,
                                    int64_t cols, int esize, hipStream_t s);
hipError_t launch_mlp_forward(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* p,
                              const float* X, float* y, hipStream_t s);
hipError_t launch_mlp_loss_grad(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* p,
                                const float* X, const float* t, float* grad, float* loss,
                                hipStream_t s);
hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, int64_t t, hipStream_t s);

}  // namespace mlk
