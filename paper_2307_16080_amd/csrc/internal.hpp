// internal.hpp -- host-side declarations shared by the C-ABI units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mlk.h"
#include "kernels.hpp"

namespace mlk {

// ---- errors (thread-local message)
mlk_status fail(mlk_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
mlk_status hip_fail(hipError_t e, const char* what);

// ---- device facts
int device_cus();  // compute units of the current device (256 on MI355X)

// ---- the normalised shape of one contraction (a matmul, or a conv viewed as
// rows = F, columns = N*HO*WO, depth = C*KH*KW)
struct Shape {
    int dt = DT_F32;
    int conv = 0;
    int64_t M = 0, N = 0, K = 0;
    int accumulate = 1;
    int out16 = 0;        // 1: C holds bf16 (matmul only)
    int64_t conv_c = 0;   // conv: input channels
    int64_t conv_in = 0;  // conv: input elements N*C*H*W
    int conv_kh = 0, conv_kw = 0, conv_sh = 0, conv_sw = 0;  // conv: filter taps and strides
};

// one-pass e4m3 quantisation (elementwise.hip): the whole input held in the
// registers of a resident grid across a grid-wide exchange of the workgroups'
// maxima.  hipErrorNotSupported, with nothing enqueued, when the input does
// not fit or is not aligned (the two-pass form then runs).  Callers serialise
// through the scratch lock (held around the launch).
hipError_t launch_quant_e4m3_fused(const float* x, int64_t n, uint8_t* q, float* scale, hipStream_t s);

// registry of compiled kernels
const std::vector<const KernelEntry*>& registry();
// the fp32 conv tiles that gather whole K chunks (k_conv_f32.hip)
const KernelEntry* kernels_conv_chunk(int* n);
// such a tile (fp32 conv, stages 1) and the limits of its 32-bit gather
// offsets and reciprocal divisions: C*H*W per image below 2^31 and
// C*KH*KW * KH*KW below 2^32
bool is_chunk_conv(const KernelEntry* e);
bool chunk_conv_ok(const Shape& s);
const KernelEntry* find_kernel(int dt, int conv, const mlk_tile_config& c);

int dt_of(mlk_dtype in, mlk_dtype out, int conv, bool* ok);

// problem -> Shape (validating the problem's own fields); MLK_OK or an error
mlk_status shape_of_problem(const mlk_problem* p, Shape* s);

// the legal configuration space of a problem, in enumeration order
std::vector<mlk_tile_config> enumerate_configs(const mlk_problem* p, const Shape& s);
mlk_status check_config(const Shape& s, int op, const mlk_tile_config& c);
// conv_gather = false leaves out the channel-gather conv tile (whose filter
// transpose takes scratch memory in an unbound call)
mlk_tile_config heuristic_config(const Shape& s, int op, bool conv_gather = true);
std::string problem_key(const mlk_problem* p);

// tuned defaults consulted by launches that pass no configuration
bool lookup_default(const std::string& key, mlk_tile_config* c);
void store_default(const std::string& key, const mlk_tile_config& c);

// launch one contraction with a resolved configuration
mlk_status launch_dense(const Shape& s, const void* A, int64_t lda, const void* B, int64_t ldb,
                        void* C, int64_t ldc, const float* sa, const float* sb,
                        const mlk_tile_config& cfg, hipStream_t st, const float* bias = nullptr,
                        void* ext_ws = nullptr, size_t ext_bytes = 0);
// bytes of packed operand copies launch_dense needs for this launch (0: none)
int64_t dense_workspace_bytes(const Shape& s, const void* A, int64_t lda, const void* B, int64_t ldb,
                              const mlk_tile_config& cfg);
// Buffers a bound convolution owns for the channels-last layout: the NHWC
// copy of the input (written by each call) and the filter already laid out
// F x KH x KW x C.  With them launch_conv takes no scratch memory.
struct ConvPrep {
    void* xn;
    const void* w_cl;
};
mlk_status launch_conv(const Shape& s, int64_t n, int64_t c, int64_t h, int64_t w, int64_t f,
                       int64_t kh, int64_t kw, int sh, int sw, int ph, int pw, int64_t ho,
                       int64_t wo, const void* x, const void* wt, void* y,
                       const mlk_tile_config& cfg, hipStream_t st, const ConvPrep* prep = nullptr);

int64_t conv_out(int64_t in, int64_t k, int64_t stride, int64_t pad);

// the MFMA rate probe (probe.hip): `blocks` workgroups of four waves, each
// wave `iters` steps of eight independent MFMAs (dt DT_BF16 or DT_F8)
hipError_t launch_mfma_rate(int dt, int64_t iters, int blocks, float* out, hipStream_t s);

// One use of the library's scratch memory (scratch.cpp).  begin() returns
// with the device's buffer (at least `bytes`) locked for this call and the
// stream ordered after the buffer's previous use; end(), or the destructor,
// records the release once the call's work is enqueued.  On a capturing
// stream begin() refuses with MLK_ERR_CONFIG.
class ScratchUse {
  public:
    ScratchUse() = default;
    ScratchUse(const ScratchUse&) = delete;
    ScratchUse& operator=(const ScratchUse&) = delete;
    ~ScratchUse();
    mlk_status begin(size_t bytes, hipStream_t st, const char* what);
    mlk_status end();
    void* ptr() const { return ptr_; }

  private:
    std::unique_lock<std::mutex> lock_;
    hipStream_t stream_ = nullptr;
    void* ptr_ = nullptr;
    void* own_ = nullptr;  // an uncached (oversized) allocation of this use
    int dev_ = 0;
};
void release_scratch();

// cost model internals used by the tuner
int model_feature_count();
void model_features(const Shape& s, const mlk_tile_config& c, int cus, float* out);
mlk_status model_predict_shape(mlk_cost_model* m, const Shape& s,
                               const std::vector<mlk_tile_config>& cfgs, std::vector<float>* us);

// analytic stand-in for a GPU timing (used by mlk_tune's fake_timer mode)
double fake_time_us(const Shape& s, int op, const mlk_tile_config& c, int index, uint64_t seed);

}  // namespace mlk
