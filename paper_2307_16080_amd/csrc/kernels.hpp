// kernels.hpp -- kernel-instance registry shared by the host code and the
// per-dtype instantiation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gemm_fast.hpp"
#include "gemm_tile.hpp"

namespace mlk {

// One (GEMM, tile) work item of a persistent launch.  kind 0: a tile of the
// configured shape; kind 1: a 64 x 64 tile of the same kernel (used for GEMMs
// too small to fill the configured tile).
struct Task {
    int32_t gemm, tm, tn, kind;
};

// One operand copied into a zero-padded, 16-byte-pitched buffer: rows x cols
// elements from src (pitch ld_src) to dst (pitch ld_dst elements, rows_dst
// rows); every other element of the dst block is written as zero.
struct PackJob {
    const void* src;
    void* dst;
    int64_t ld_src, ld_dst;
    int32_t rows, cols, rows_dst, pad_;
};

typedef hipError_t (*launch_fn)(const GemmArgs& g, int nblk, hipStream_t s);
typedef hipError_t (*persist_fn)(const GemmArgs* gemms, const Task* tasks,
                                 const int32_t* bounds, int nblk, hipStream_t s);
typedef int (*occupancy_fn)();  // workgroups of the persistent kernel resident per CU

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
    occupancy_fn occupancy; // with persist: resident workgroups per CU
    launch_fn launch_epi;   // GEMM entries: the Linear variant, bias added to an fp32 C (EPI = 1)
    launch_fn launch_epi16; // GEMM entries that write a bf16 C (EPI = 2); null where not built
    int mfma;               // MFMA output tile: 16 (16 x 16) or 32 (32 x 32, bf16 direct-layout tiles)
    launch_fn launch_gather;  // conv entries: the NCHW channel-gather variant (CONV = 3); null where not built
    persist_fn persist_gather;      // conv entries: a persistent channel-gather launch over many convolutions
    occupancy_fn occupancy_gather;  // with persist_gather: resident workgroups per CU
};

template <int DT, int BM, int BN, int KB, int WM, int WN, int CONV, int EPI = 0>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(GemmArgs g) {
    typedef Tile<DT, BM, BN, KB, WM, WN, CONV, EPI> TL;
    __shared__ __attribute__((aligned(16))) uint8_t lds[TL::LDS_BYTES];
    int tm, tn, kz;
    tile_coords(g, blockIdx.x, gridDim.x, tm, tn, kz);
    TL::run(g, tm, tn, kz, lds);
}

// The small tile paired with a configured tile in one persistent kernel: a
// 64 x 64 tile with the same number of waves when the configured tile has 4
// waves, otherwise the configured tile itself (no second shape).
template <int DT, int BM, int BN, int KB, int WM, int WN>
struct SmallTile {
    static constexpr bool pair = WM * WN == 4 && !(BM == 64 && BN == 64);
    typedef typename std::conditional<pair, Tile<DT, 64, 64, 128, 2, 2, 0>,
                                      Tile<DT, BM, BN, KB, WM, WN, 0>>::type type;
};

// Persistent variant: workgroup b runs tasks [bounds[b], bounds[b+1]) in order.
template <int DT, int BM, int BN, int KB, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_persist(const GemmArgs* __restrict__ gemms,
                                                               const Task* __restrict__ tasks,
                                                               const int32_t* __restrict__ bounds) {
    typedef Tile<DT, BM, BN, KB, WM, WN, 0> TL;
    typedef typename SmallTile<DT, BM, BN, KB, WM, WN>::type TS;
    constexpr int LDS = TL::LDS_BYTES > TS::LDS_BYTES ? TL::LDS_BYTES : TS::LDS_BYTES;
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS];
    const int b = blockIdx.x;
    const int t0 = bounds[b], t1 = bounds[b + 1];
    for (int t = t0; t < t1; ++t) {
        const Task tk = tasks[t];
        const GemmArgs g = gemms[tk.gemm];
        if (SmallTile<DT, BM, BN, KB, WM, WN>::pair && tk.kind == 1) TS::run(g, tk.tm, tk.tn, 0, lds);
        else TL::run(g, tk.tm, tk.tn, 0, lds);
        __syncthreads();
    }
}

template <int DT, int BM, int BN, int WM, int WN, int STAGES, int EPI = 0, int MF = 16>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_fast(GemmArgs g) {
    typedef FastGemm<DT, BM, BN, WM, WN, STAGES, 0, EPI, MF> TL;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TL::LDS_BYTES];
    int tm, tn, kz;
    tile_coords(g, blockIdx.x, gridDim.x, tm, tn, kz);
    TL::run(g, tm, tn, kz, lds);
}

// The implicit-GEMM convolution forms of the direct-layout kernel: CONV 2
// gathers from a channels-last copy of the input, CONV 3 from NCHW itself.
template <int DT, int BM, int BN, int WM, int WN, int STAGES, int CONV = 2>
__global__ __launch_bounds__(64 * WM * WN) void k_fast_conv(GemmArgs g) {
    typedef FastGemm<DT, BM, BN, WM, WN, STAGES, CONV> TL;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TL::LDS_BYTES];
    int tm, tn, kz;
    tile_coords(g, blockIdx.x, gridDim.x, tm, tn, kz);
    TL::run(g, tm, tn, kz, lds);
}

template <int DT, int BM, int BN, int WM, int WN, int STAGES, int CONV = 2>
hipError_t launch_fast_conv(const GemmArgs& g, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_fast_conv<DT, BM, BN, WM, WN, STAGES, CONV>), dim3(nblk), dim3(64 * WM * WN), 0, s, g);
    return hipGetLastError();
}

// Persistent channel-gather convolution over a batch of convolutions: the
// host deals every convolution's tasks -- (output tile, K split) pairs, the
// split index in Task::kind -- into one range per workgroup; workgroup b runs
// its range in order.  Each task is exactly a plain launch's workgroup of the
// same tile, split and convolution.
template <int DT, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_conv_persist(const GemmArgs* __restrict__ convs,
                                                               const Task* __restrict__ tasks,
                                                               const int32_t* __restrict__ bounds) {
    typedef FastGemm<DT, BM, BN, WM, WN, 1, 3> TL;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TL::LDS_BYTES];
    const int b = blockIdx.x;
    const int t0 = bounds[b], t1 = bounds[b + 1];
    for (int t = t0; t < t1; ++t) {
        const Task tk = tasks[t];
        const GemmArgs g = convs[tk.gemm];
        TL::run(g, tk.tm, tk.tn, tk.kind, lds);
        __syncthreads();
    }
}

template <int DT, int BM, int BN, int WM, int WN>
hipError_t launch_conv_persist(const GemmArgs* convs, const Task* tasks, const int32_t* bounds, int nblk,
                               hipStream_t s) {
    hipLaunchKernelGGL((k_conv_persist<DT, BM, BN, WM, WN>), dim3(nblk), dim3(64 * WM * WN), 0, s, convs, tasks,
                       bounds);
    return hipGetLastError();
}

// the channel-gather variants exist for the register-loaded conv tiles only
template <int DT, int BM, int BN, int WM, int WN, int STAGES>
constexpr launch_fn gather_fn() {
    if constexpr (STAGES == 1) return &launch_fast_conv<DT, BM, BN, WM, WN, 1, 3>;
    else return nullptr;
}
template <int DT, int BM, int BN, int WM, int WN, int STAGES>
constexpr persist_fn gather_persist_fn() {
    if constexpr (STAGES == 1) return &launch_conv_persist<DT, BM, BN, WM, WN>;
    else return nullptr;
}

template <int DT, int BM, int BN, int WM, int WN, int STAGES, int EPI = 0, int MF = 16>
hipError_t launch_fast(const GemmArgs& g, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm_fast<DT, BM, BN, WM, WN, STAGES, EPI, MF>), dim3(nblk), dim3(64 * WM * WN), 0,
                       s, g);
    return hipGetLastError();
}

// Persistent form of the direct-layout kernel (one tile shape).  The
// direct-to-LDS form (STAGES >= 2) runs batches whose operands were packed
// into aligned, zero-padded buffers first.
template <int DT, int BM, int BN, int WM, int WN, int STAGES, int MF = 16>
__global__ __launch_bounds__(64 * WM * WN) void k_fast_persist(const GemmArgs* __restrict__ gemms,
                                                               const Task* __restrict__ tasks,
                                                               const int32_t* __restrict__ bounds) {
    typedef FastGemm<DT, BM, BN, WM, WN, STAGES, 0, 0, MF> TL;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[TL::LDS_BYTES];
    const int b = blockIdx.x;
    const int t0 = bounds[b], t1 = bounds[b + 1];
    for (int t = t0; t < t1; ++t) {
        const Task tk = tasks[t];
        const GemmArgs g = gemms[tk.gemm];
        TL::run(g, tk.tm, tk.tn, 0, lds);
        __syncthreads();
    }
}

template <int DT, int BM, int BN, int WM, int WN, int STAGES, int MF = 16>
hipError_t launch_fast_persist(const GemmArgs* gemms, const Task* tasks, const int32_t* bounds,
                               int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_fast_persist<DT, BM, BN, WM, WN, STAGES, MF>), dim3(nblk), dim3(64 * WM * WN), 0,
                       s, gemms, tasks, bounds);
    return hipGetLastError();
}

// Resident workgroups per CU of a persistent kernel (registers, LDS and waves
// all counted by the runtime), at least 1.
template <class K>
int occupancy_of(K kernel, int threads) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess) n = 1;
    return n > 0 ? n : 1;
}
template <int DT, int BM, int BN, int KB, int WM, int WN>
int occupancy_persist() {
    return occupancy_of(k_gemm_persist<DT, BM, BN, KB, WM, WN>, 64 * WM * WN);
}
template <int DT, int BM, int BN, int WM, int WN, int STAGES, int MF = 16>
int occupancy_fast_persist() {
    return occupancy_of(k_fast_persist<DT, BM, BN, WM, WN, STAGES, MF>, 64 * WM * WN);
}
template <int DT, int BM, int BN, int WM, int WN>
int occupancy_conv_persist() {
    return occupancy_of(k_conv_persist<DT, BM, BN, WM, WN>, 64 * WM * WN);
}
template <int DT, int BM, int BN, int WM, int WN, int STAGES>
constexpr occupancy_fn gather_occupancy_fn() {
    if constexpr (STAGES == 1) return &occupancy_conv_persist<DT, BM, BN, WM, WN>;
    else return nullptr;
}

template <int DT, int BM, int BN, int KB, int WM, int WN, int CONV, int EPI = 0>
hipError_t launch_gemm(const GemmArgs& g, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm<DT, BM, BN, KB, WM, WN, CONV, EPI>), dim3(nblk), dim3(64 * WM * WN), 0,
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

// Output-stage variants of a GEMM entry: the Linear variant (EPI = 1) for the
// float outputs, the bf16-output variant (EPI = 2) for bf16 and e4m3 inputs
// and, in the fast kernel, only its direct-to-LDS forms (the register-loaded
// form has no registers to spare for it).  Conv entries have neither.
template <int DT, int BM, int BN, int KB, int WM, int WN, int CONV, int EPI>
launch_fn tile_epi() {
    if constexpr (CONV != 0 || DT == DT_I8 || (EPI == 2 && DT == DT_F32)) return nullptr;
    else return &launch_gemm<DT, BM, BN, KB, WM, WN, 0, EPI>;
}
template <int DT, int BM, int BN, int WM, int WN, int STAGES>
launch_fn fast_epi16() {
    if constexpr (STAGES >= 2) return &launch_fast<DT, BM, BN, WM, WN, STAGES, 2>;
    else return nullptr;
}

#define MLK_ENTRY(DT, BM, BN, KB, WM, WN, CONV)                                              \
    KernelEntry {                                                                            \
        DT, (CONV) ? 1 : 0, 0, BM, BN, (KB) / Traits<DT>::ES, WM, WN,                          \
            Tile<DT, BM, BN, KB, WM, WN, (CONV) ? 1 : 0>::LDS_BYTES, 64 * (WM) * (WN),         \
            &launch_gemm<DT, BM, BN, KB, WM, WN, (CONV) ? 1 : 0>, nullptr,                     \
            (CONV) ? &launch_gemm<DT, BM, BN, KB, WM, WN, 2> : nullptr, nullptr,              \
            tile_epi<DT, BM, BN, KB, WM, WN, (CONV) ? 1 : 0, 1>(),                             \
            tile_epi<DT, BM, BN, KB, WM, WN, (CONV) ? 1 : 0, 2>(), 16                          \
    }

#define MLK_ENTRY_P(DT, BM, BN, KB, WM, WN)                                                  \
    KernelEntry {                                                                            \
        DT, 0, 0, BM, BN, (KB) / Traits<DT>::ES, WM, WN,                                     \
            Tile<DT, BM, BN, KB, WM, WN, 0>::LDS_BYTES, 64 * (WM) * (WN),                    \
            &launch_gemm<DT, BM, BN, KB, WM, WN, 0>, &launch_persist<DT, BM, BN, KB, WM, WN>,  \
            nullptr, &occupancy_persist<DT, BM, BN, KB, WM, WN>,                             \
            tile_epi<DT, BM, BN, KB, WM, WN, 0, 1>(), tile_epi<DT, BM, BN, KB, WM, WN, 0, 2>(), 16 \
    }

#define MLK_ENTRY_FAST(DT, BM, BN, WM, WN, STAGES)                                           \
    KernelEntry {                                                                            \
        DT, 0, STAGES, BM, BN, FastGemm<DT, BM, BN, WM, WN, STAGES>::BK, WM, WN,              \
            FastGemm<DT, BM, BN, WM, WN, STAGES>::LDS_BYTES, 64 * (WM) * (WN),               \
            &launch_fast<DT, BM, BN, WM, WN, STAGES>,                                        \
            &launch_fast_persist<DT, BM, BN, WM, WN, STAGES>, nullptr,                       \
            &occupancy_fast_persist<DT, BM, BN, WM, WN, STAGES>,                             \
            &launch_fast<DT, BM, BN, WM, WN, STAGES, 1>, fast_epi16<DT, BM, BN, WM, WN, STAGES>(), 16 \
    }

// the same direct-layout GEMM with 32 x 32 MFMA tiles (bf16): no bf16-output variant
#define MLK_ENTRY_FAST32(BM, BN, WM, WN, STAGES)                                             \
    KernelEntry {                                                                            \
        DT_BF16, 0, STAGES, BM, BN, FastGemm<DT_BF16, BM, BN, WM, WN, STAGES, 0, 0, 32>::BK, WM, WN, \
            FastGemm<DT_BF16, BM, BN, WM, WN, STAGES, 0, 0, 32>::LDS_BYTES, 64 * (WM) * (WN),   \
            &launch_fast<DT_BF16, BM, BN, WM, WN, STAGES, 0, 32>,                            \
            &launch_fast_persist<DT_BF16, BM, BN, WM, WN, STAGES, 32>, nullptr,              \
            &occupancy_fast_persist<DT_BF16, BM, BN, WM, WN, STAGES, 32>,                    \
            &launch_fast<DT_BF16, BM, BN, WM, WN, STAGES, 1, 32>, nullptr, 32                \
    }

// int8 direct-layout entry: the plain int32 output stage only (no Linear or
// bf16-output variant, no persistent form: batches are bf16 / fp32)
#define MLK_ENTRY_FAST_I8(BM, BN, WM, WN, STAGES)                                            \
    KernelEntry {                                                                            \
        DT_I8, 0, STAGES, BM, BN, FastGemm<DT_I8, BM, BN, WM, WN, STAGES>::BK, WM, WN,        \
            FastGemm<DT_I8, BM, BN, WM, WN, STAGES>::LDS_BYTES, 64 * (WM) * (WN),            \
            &launch_fast<DT_I8, BM, BN, WM, WN, STAGES>, nullptr, nullptr, nullptr, nullptr, nullptr, 16 \
    }

// conv entry: the channels-last layout (launch_nhwc) and, for the
// register-loaded tiles, the NCHW channel gather (launch_gather); no plain
// NCHW form (launch), no persistent form
#define MLK_ENTRY_FASTCONV(DT, BM, BN, WM, WN, STAGES)                                       \
    KernelEntry {                                                                            \
        DT, 1, STAGES, BM, BN, FastGemm<DT, BM, BN, WM, WN, STAGES, 2>::BK, WM, WN,          \
            FastGemm<DT, BM, BN, WM, WN, STAGES, 2>::LDS_BYTES, 64 * (WM) * (WN), nullptr,   \
            nullptr, &launch_fast_conv<DT, BM, BN, WM, WN, STAGES>, nullptr, nullptr, nullptr, 16, \
            gather_fn<DT, BM, BN, WM, WN, STAGES>(), gather_persist_fn<DT, BM, BN, WM, WN, STAGES>(), \
            gather_occupancy_fn<DT, BM, BN, WM, WN, STAGES>()                                   \
    }

// Tables defined by the instantiation units (host functions: the tables hold
// host launch functions, so they must not exist in the device pass).
const KernelEntry* kernels_f32(int* n);
const KernelEntry* kernels_bf16(int* n);
const KernelEntry* kernels_i8(int* n);
const KernelEntry* kernels_f8(int* n);
const KernelEntry* kernels_conv(int* n);
const KernelEntry* kernels_fast(int* n);

// Direct (stencil) convolution (k_direct.hip): a few filters (F <=
// kDirectMaxF), strides up to kDirectMaxStride, filter taps up to
// kDirectMaxTap per side.  Its entries have bk = 1 and wm = wn = 0 and run as
// conv layout 2; a TH x TW tile stages an input window of
// direct_patch(TH, TW) floats in LDS.
constexpr int kDirectMaxF = 16, kDirectMaxStride = 2, kDirectMaxTap = 7;
constexpr int direct_patch(int th, int tw) {
    return ((th - 1) * kDirectMaxStride + kDirectMaxTap) * ((tw - 1) * kDirectMaxStride + kDirectMaxTap);
}
const KernelEntry* kernels_direct(int* n);

// Elementwise / reduction launchers (quant.hip, reduce.hip, mlp.hip).
hipError_t launch_zero_matrix(void* C, int64_t M, int64_t N, int64_t ldc, int esize,
                              hipStream_t s);
hipError_t launch_quant_bf16(const float* x, int64_t n, uint16_t* q, hipStream_t s);
// `part`: device workspace of quant_e4m3_parts() floats (per-workgroup maxima)
constexpr int quant_e4m3_parts() { return 512; }
hipError_t launch_quant_e4m3(const float* x, int64_t n, uint8_t* q, float* scale, float* part,
                             hipStream_t s);
// `part`: device workspace of err_stats_parts() x 4 doubles (per-workgroup partials)
constexpr int err_stats_parts() { return 1024; }
hipError_t launch_err_stats(int c_is_int, int64_t n, const void* c, const double* r,
                            const double* bound, double* out, double* part, hipStream_t s);
hipError_t launch_fill_random(void* p, int64_t n, int dt, uint64_t seed, hipStream_t s);
// copy operands into zero-padded buffers, one wave per segment of kPackSeg
// consecutive destination elements; seg_start[j] = first segment of job j in
// a running count over all jobs (njobs + 1 entries, device memory)
constexpr int kPackSeg = 2048;
inline int64_t pack_segments(const PackJob& j) {
    return ((int64_t)j.rows_dst * j.ld_dst + kPackSeg - 1) / kPackSeg;
}
hipError_t launch_pack(const PackJob* jobs, const int64_t* seg_start, int njobs, int64_t total_segs,
                       int esize, hipStream_t s);
// the same for one or two jobs given in host memory (passed by value)
hipError_t launch_pack_pair(const PackJob* jobs, int njobs, int esize, hipStream_t s);
// two batches of [rows x cols] matrices -> [cols x rows] in one launch
// (NCHW -> NHWC and FCHW -> FHWC); a job with batch 0 is skipped
hipError_t launch_transpose_pair(const void* in0, void* out0, int64_t batch0, int64_t rows0, int64_t cols0,
                                 const void* in1, void* out1, int64_t batch1, int64_t rows1, int64_t cols1,
                                 int esize, hipStream_t s);
// `ws`: device workspace of mlp_forward_words() / mlp_loss_grad_words() floats
// (the hidden activations, pre-activations and deltas of the batch)
inline int64_t mlp_forward_words(int64_t B, int64_t H1, int64_t H2) { return B * (H1 + H2); }
inline int64_t mlp_loss_grad_words(int64_t B, int64_t H1, int64_t H2) { return B * (3 * H1 + 3 * H2 + 2); }
hipError_t launch_mlp_forward(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* p,
                              const float* X, float* y, float* ws, hipStream_t s);
hipError_t launch_mlp_loss_grad(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* p,
                                const float* X, const float* t, float* grad, float* loss, float* ws,
                                hipStream_t s);
hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, int64_t t, hipStream_t s);

}  // namespace mlk
