// elementwise.hip -- the HBM-bound kernels around the contractions:
// quantisation to bf16 / OCP e4m3 (per-tensor amax scaling), clearing an
// output, seeded fills for tuner scratch inputs, and the FP64 error
// reduction against a double-precision reference.
//
// All are streaming kernels: 16-byte coalesced loads, grid-stride loops,
// a grid sized to a few workgroups per CU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "internal.hpp"
#include "kernels.hpp"

namespace mlk {

namespace {

constexpr int kThreads = 256;

inline int grid_for(int64_t items, int per_block_items) {
    int64_t g = (items + per_block_items - 1) / per_block_items;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

// ------------------------------------------------------------------ bf16
// (bf16_rne, the rounding shared with the GEMM epilogues, is in gemm_tile.hpp)

__global__ __launch_bounds__(kThreads) void k_quant_bf16(const float* __restrict__ x, int64_t n,
                                                         uint16_t* __restrict__ q) {
    // 8 values per thread per step: two 16-byte loads, one 16-byte store
    const int64_t nvec = n / 8;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) {
        const f4_t a = *(const f4_t*)(x + 8 * i);
        const f4_t b = *(const f4_t*)(x + 8 * i + 4);
        u4_t o;
        o[0] = bf16_rne(a[0]) | ((uint32_t)bf16_rne(a[1]) << 16);
        o[1] = bf16_rne(a[2]) | ((uint32_t)bf16_rne(a[3]) << 16);
        o[2] = bf16_rne(b[0]) | ((uint32_t)bf16_rne(b[1]) << 16);
        o[3] = bf16_rne(b[2]) | ((uint32_t)bf16_rne(b[3]) << 16);
        *(u4_t*)(q + 8 * i) = o;
    }
    // tail
    if (blockIdx.x == 0)
        for (int64_t i = nvec * 8 + threadIdx.x; i < n; i += blockDim.x) q[i] = bf16_rne(x[i]);
}

__global__ __launch_bounds__(kThreads) void k_quant_bf16_scalar(const float* __restrict__ x,
                                                                int64_t n, uint16_t* __restrict__ q) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        q[i] = bf16_rne(x[i]);
}

// ------------------------------------------------------------------ e4m3

// fp32 -> OCP E4M3, round to nearest even, saturating to +-448; NaN -> 0x7F.
__device__ inline uint32_t e4m3_rne_sat(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t mag = u & 0x7FFFFFFFu;
    if (mag > 0x7F800000u) return 0x7Fu;              // NaN
    if (mag >= 0x43E00000u) return sign | 0x7Eu;      // |v| >= 448 (incl. inf)
    if (mag < 0x3C800000u) {                          // |v| < 2^-6: subnormal grid 2^-9
        // |v| * 2^9 is exact; round half to even onto 0..8 (8 = smallest normal)
        const float s = __uint_as_float(mag) * 512.0f;
        return sign | (uint32_t)__builtin_rintf(s);
    }
    const uint32_t e = (mag >> 23) - 127 + 7;         // biased e4m3 exponent, 1..15
    const uint32_t m = mag & 0x7FFFFFu;
    uint32_t r = m >> 20;                             // keep 3 fraction bits
    const uint32_t rest = m & 0xFFFFFu, half = 0x80000u;
    uint32_t code = (e << 3) | r;
    if (rest > half || (rest == half && (r & 1u))) code += 1;  // carry may bump exponent
    return sign | code;                               // < 448 never reaches 0x7F
}

// Two passes.  k_amax writes one maximum |x| per workgroup (kAmaxBlocks of
// them, as non-negative floats); k_quant_e4m3 has every workgroup reduce those
// partials to amax first (a few KB from L2: no atomics, no device-wide
// counter), derive the scale, and workgroup 0 stores it.
constexpr int kAmaxBlocks = quant_e4m3_parts();

template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_amax(const float* __restrict__ x, int64_t n,
                                                   float* __restrict__ part) {
    float m = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (VEC) {
        const int64_t nvec = n / 4;
        int64_t i = first;
        // eight independent 16-byte loads in flight per thread
        for (; i + 7 * stride < nvec; i += 8 * stride) {
            f4_t a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = *(const f4_t*)(x + 4 * (i + u * stride));
#pragma unroll
            for (int u = 0; u < 8; ++u)
                m = fmaxf(m, fmaxf(fmaxf(fabsf(a[u][0]), fabsf(a[u][1])), fmaxf(fabsf(a[u][2]), fabsf(a[u][3]))));
        }
        for (; i < nvec; i += stride) {
            const f4_t a = *(const f4_t*)(x + 4 * i);
            m = fmaxf(m, fmaxf(fmaxf(fabsf(a[0]), fabsf(a[1])), fmaxf(fabsf(a[2]), fabsf(a[3]))));
        }
        if (blockIdx.x == 0)
            for (int64_t j = nvec * 4 + threadIdx.x; j < n; j += blockDim.x) m = fmaxf(m, fabsf(x[j]));
    } else {
        for (int64_t i = first; i < n; i += stride) m = fmaxf(m, fabsf(x[i]));
    }
    // fmaxf drops NaN operands, so NaNs never reach the maximum
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    __shared__ float wmax[kThreads / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) m = fmaxf(m, wmax[w]);
        part[blockIdx.x] = m;
    }
}

__device__ inline float e4m3_scale_from_amax(float amax) {
    if (!(amax > 0.0f) || !__builtin_isfinite(amax)) return 1.0f;
    return __fdiv_rn(amax, 448.0f);
}

// amax over the partials of k_amax, by the whole workgroup; thread 0 of
// workgroup 0 also stores the scale
__device__ inline float e4m3_block_scale(const float* __restrict__ part, int nparts, float* scale) {
    float m = 0.0f;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmaxf(m, part[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    __shared__ float wmax[kThreads / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = wmax[0];
    for (int w = 1; w < kThreads / 64; ++w) m = fmaxf(m, wmax[w]);
    const float s = e4m3_scale_from_amax(m);
    if (blockIdx.x == 0 && threadIdx.x == 0) *scale = s;
    return s;
}

// e4m3 code of RN(x / s) without a division for almost every element: y =
// x * RN(1/s) is within 2.5 fp32 ulps of RN(x / s) (two roundings of 2^-24
// relative each, plus the quotient's own half ulp), and the e4m3 code is a
// step function of its input whose steps in the normal range sit where the
// 20 fraction bits below the kept three equal 0x80000.  So when y is a normal
// e4m3 input (2^-6 <= |y| < 448) at least 5 ulps from such a step, y and
// RN(x / s) give the same code; otherwise (near a step, subnormal,
// saturating, non-finite, or 1/s not finite) the quotient is formed exactly.
__device__ inline uint32_t e4m3_of_quotient(float x, float s, float r, bool fast) {
    if (fast) {
        const float y = x * r;
        const uint32_t mag = __float_as_uint(y) & 0x7FFFFFFFu;
        const uint32_t rest = mag & 0xFFFFFu;
        const uint32_t d = rest > 0x80000u ? rest - 0x80000u : 0x80000u - rest;
        if (mag >= 0x3C800000u && mag < 0x43E00000u && d > 4u) return e4m3_rne_sat(y);
    }
    return e4m3_rne_sat(__fdiv_rn(x, s));
}

// Four codes packed in a word, through the gfx950 packed conversion
// v_cvt_pk_fp8_f32 (round to nearest even into OCP e4m3, two values per
// instruction): it gives e4m3_rne_sat's code for every fp32 value below 464
// in magnitude (checked on the GPU over all 2,278,555,648 such bit patterns
// of both signs), and it is monotonic.  y = x * RN(1/s) is within 1.5 * 2^-23
// of RN(x / s) relatively (see e4m3_of_quotient), so when y * (1 - 2^-21)
// and y * (1 + 2^-21) (which bracket that interval) encode to y's own code,
// no rounding step lies between y and RN(x / s) and the code is RN(x / s)'s.
// Values of 448 or more in magnitude (or NaN), or a bracket that straddles a
// step, take e4m3_of_quotient per value.
// The packed conversion's code for four values into *code; true when the
// bracket test settles all four (every |y| below 448 and neither bracket end
// changes the code).
__device__ inline bool e4m3_try_pack4(const f4_t& a, float r, uint32_t* code) {
    const float y0 = a[0] * r, y1 = a[1] * r, y2 = a[2] * r, y3 = a[3] * r;
    // (a NaN compares false)
    if (!(fabsf(y0) < 448.0f && fabsf(y1) < 448.0f && fabsf(y2) < 448.0f && fabsf(y3) < 448.0f)) return false;
    const float up = 1.0f + 0x1p-21f, dn = 1.0f - 0x1p-21f;
    const uint32_t c = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(
        y2, y3, __builtin_amdgcn_cvt_pk_fp8_f32(y0, y1, 0, false), true);
    const uint32_t cu = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(
        y2 * up, y3 * up, __builtin_amdgcn_cvt_pk_fp8_f32(y0 * up, y1 * up, 0, false), true);
    const uint32_t cd = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(
        y2 * dn, y3 * dn, __builtin_amdgcn_cvt_pk_fp8_f32(y0 * dn, y1 * dn, 0, false), true);
    *code = c;
    return cu == c && cd == c;
}

// four codes value by value
__device__ inline uint32_t e4m3_slow4(const f4_t& a, float s, float r, bool fast) {
    return e4m3_of_quotient(a[0], s, r, fast) | (e4m3_of_quotient(a[1], s, r, fast) << 8) |
           (e4m3_of_quotient(a[2], s, r, fast) << 16) | (e4m3_of_quotient(a[3], s, r, fast) << 24);
}

__device__ inline uint32_t e4m3_encode4(const f4_t& a, float s, float r, bool fast) {
    uint32_t c;
    if (fast && e4m3_try_pack4(a, r, &c)) return c;
    return e4m3_slow4(a, s, r, fast);
}

__global__ __launch_bounds__(kThreads) void k_quant_e4m3(const float* __restrict__ x, int64_t n,
                                                         const float* __restrict__ part, int nparts,
                                                         uint8_t* __restrict__ q, float* scale) {
    const float s = e4m3_block_scale(part, nparts, scale);
    const float r = __frcp_rn(s);
    const bool fast = __builtin_isfinite(r) && r > 0.0f;
    // consecutive lanes take consecutive groups of 4 values (each load and store
    // instruction of a wave covers one contiguous block), four groups in flight
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto encode4 = [&](const f4_t& a) { return e4m3_encode4(a, s, r, fast); };
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        f4_t a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = *(const f4_t*)(x + 4 * (i + u * stride));
#pragma unroll
        for (int u = 0; u < 4; ++u) *(uint32_t*)(q + 4 * (i + u * stride)) = encode4(a[u]);
    }
    for (; i < n4; i += stride) *(uint32_t*)(q + 4 * i) = encode4(*(const f4_t*)(x + 4 * i));
    if (blockIdx.x == 0)
        for (int64_t j = n4 * 4 + threadIdx.x; j < n; j += blockDim.x)
            q[j] = (uint8_t)e4m3_of_quotient(x[j], s, r, fast);
}

__global__ __launch_bounds__(kThreads) void k_quant_e4m3_scalar(const float* __restrict__ x, int64_t n,
                                                                const float* __restrict__ part, int nparts,
                                                                uint8_t* __restrict__ q, float* scale) {
    const float s = e4m3_block_scale(part, nparts, scale);
    const float r = __frcp_rn(s);
    const bool fast = __builtin_isfinite(r) && r > 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        q[i] = (uint8_t)e4m3_of_quotient(x[i], s, r, fast);
}

__global__ __launch_bounds__(kThreads) void k_scale_one(float* scale) { *scale = 1.0f; }

// One-pass e4m3 quantisation.  Every workgroup of the grid is resident (the
// launcher sizes the grid by the kernel's occupancy), each thread holds up to
// kFusedVec groups of four inputs in registers, and the scale, which depends
// on every element, comes from a grid-wide exchange of single 64-bit words:
// each workgroup publishes (epoch << 32 | bits of its maximum |x|) in its own
// word; workgroup 0 reads every word of this call's epoch, forms amax, and
// publishes (epoch << 32 | bits of amax) in each workgroup's own release word,
// which that workgroup polls.  A value and its epoch travel in one atomic
// word, so the exchange needs no fences (fences here are cache write-backs
// and invalidations, thousands of them at once); the input is read-only and
// each workgroup writes only its own codes.  Epochs only grow from call to
// call (calls are serialised), so nothing is reset.  Every wait is bounded: a
// workgroup that gives up computes the maximum over the whole input itself
// (slow, and the same value), so the kernel always ends, with the right codes.
constexpr int kFusedVec = 16;
constexpr int kFusedMaxGrid = 1024;  // 4 words per thread of workgroup 0 (16.8 M elements)
__device__ unsigned long long g_quant_part[kFusedMaxGrid];
__device__ unsigned long long g_quant_release[kFusedMaxGrid];

// the low 32 bits of *word once its high 32 bits equal epoch (relaxed polls);
// false after spin_limit polls
__device__ inline bool wait_for_epoch(const unsigned long long* word, unsigned int epoch,
                                      unsigned int spin_limit, uint32_t* value) {
    unsigned int spins = 0;
    for (;;) {
        const unsigned long long v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned int)(v >> 32) == epoch) {
            *value = (uint32_t)v;
            return true;
        }
        if (++spins > spin_limit) return false;
        __builtin_amdgcn_s_sleep(8);
    }
}

__device__ inline float block_max(float m, float* wmax) {
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = wmax[0];
    for (int w = 1; w < kThreads / 64; ++w) m = fmaxf(m, wmax[w]);
    return m;
}

__global__ __launch_bounds__(kThreads) void k_quant_e4m3_fused(const float* __restrict__ x, int64_t n,
                                                               uint8_t* __restrict__ q, float* scale,
                                                               unsigned int epoch, unsigned int spin_limit) {
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t first = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    f4_t a[kFusedVec];
    float m = 0.0f;
#pragma unroll
    for (int u = 0; u < kFusedVec; ++u) {
        const int64_t i = first + u * stride;
        a[u] = i < n4 ? *(const f4_t*)(x + 4 * i) : f4_t{0.0f, 0.0f, 0.0f, 0.0f};
        m = fmaxf(m, fmaxf(fmaxf(fabsf(a[u][0]), fabsf(a[u][1])), fmaxf(fabsf(a[u][2]), fabsf(a[u][3]))));
    }
    if (blockIdx.x == 0)
        for (int64_t j = n4 * 4 + threadIdx.x; j < n; j += blockDim.x) m = fmaxf(m, fabsf(x[j]));
    // (fmaxf drops NaN operands, so NaNs never reach the maximum)
    __shared__ float wmax[kThreads / 64];
    __shared__ float shared_amax;
    __shared__ int released;
    m = block_max(m, wmax);
    const unsigned long long tag = (unsigned long long)epoch << 32;
    if (threadIdx.x == 0)
        __hip_atomic_store(&g_quant_part[blockIdx.x], tag | __float_as_uint(m), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (blockIdx.x == 0) {
        // each thread gathers its (up to kFusedMaxGrid / kThreads) words, all of
        // them polled together so that every round waits one memory latency
        constexpr int kWords = kFusedMaxGrid / kThreads;
        uint32_t pending = 0;
#pragma unroll
        for (int k = 0; k < kWords; ++k)
            if (threadIdx.x + k * kThreads < (int)gridDim.x) pending |= 1u << k;
        float mm = 0.0f;
        unsigned int spins = 0;
        while (pending != 0 && spins <= spin_limit) {
            unsigned long long v[kWords];
#pragma unroll
            for (int k = 0; k < kWords; ++k)
                v[k] = (pending >> k) & 1u ? __hip_atomic_load(&g_quant_part[threadIdx.x + k * kThreads],
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                           : 0ull;
#pragma unroll
            for (int k = 0; k < kWords; ++k)
                if (((pending >> k) & 1u) && (unsigned int)(v[k] >> 32) == epoch) {
                    mm = fmaxf(mm, __uint_as_float((uint32_t)v[k]));
                    pending &= ~(1u << k);
                }
            if (pending != 0) {
                ++spins;
                __builtin_amdgcn_s_sleep(2);
            }
        }
        const bool all = __syncthreads_and(pending == 0);
        mm = block_max(mm, wmax);
        if (all)
            for (int b = threadIdx.x + 1; b < (int)gridDim.x; b += blockDim.x)
                __hip_atomic_store(&g_quant_release[b], tag | __float_as_uint(mm), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x == 0) {
            released = all;
            shared_amax = mm;
        }
    } else if (threadIdx.x == 0) {
        uint32_t bits = 0;
        released = wait_for_epoch(&g_quant_release[blockIdx.x], epoch, spin_limit, &bits);
        shared_amax = __uint_as_float(bits);
    }
    __syncthreads();
    float amax = shared_amax;
    if (!released) {
        float mm = 0.0f;
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) mm = fmaxf(mm, fabsf(x[j]));
        amax = block_max(mm, wmax);
    }
    const float s = e4m3_scale_from_amax(amax);
    if (blockIdx.x == 0 && threadIdx.x == 0) *scale = s;
    const float r = __frcp_rn(s);
    const bool fast = __builtin_isfinite(r) && r > 0.0f;
    // Codes that the packed conversion settles are stored at once; the other
    // groups (the one holding the maximum, values next to a rounding step) are
    // read again and take the per-value path in one loop, so the kernel holds
    // one copy of that long path rather than one per register group (inlined
    // into all sixteen, it made the kernel four times larger).
    uint32_t rest = 0;
#pragma unroll
    for (int u = 0; u < kFusedVec; ++u) {
        const int64_t i = first + u * stride;
        uint32_t c;
        if (i < n4) {
            if (fast && e4m3_try_pack4(a[u], r, &c))
                *(uint32_t*)(q + 4 * i) = c;
            else
                rest |= 1u << u;
        }
    }
    while (rest != 0) {
        const int u = __builtin_ctz(rest);
        rest &= rest - 1;
        const int64_t i = first + u * stride;
        *(uint32_t*)(q + 4 * i) = e4m3_slow4(*(const f4_t*)(x + 4 * i), s, r, fast);
    }
    if (blockIdx.x == 0)
        for (int64_t j = n4 * 4 + threadIdx.x; j < n; j += blockDim.x)
            q[j] = (uint8_t)e4m3_of_quotient(x[j], s, r, fast);
}

// ------------------------------------------------------------------ fills

__global__ __launch_bounds__(kThreads) void k_zero_matrix(uint8_t* C, int64_t M, int64_t rowbytes,
                                                          int64_t ldbytes) {
    const int64_t total = M * rowbytes;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total / 4; i += stride) {
        const int64_t r = (4 * i) / rowbytes, c = (4 * i) % rowbytes;
        *(uint32_t*)(C + r * ldbytes + c) = 0u;
    }
}

__device__ inline uint64_t splitmix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Seeded scratch values for timing runs: uniform in [-1, 1) for f32 / bf16,
// finite e4m3 codes of magnitude <= 1 for e4m3, and any int8.
__global__ __launch_bounds__(kThreads) void k_fill_random(uint8_t* p, int64_t n, int dt,
                                                          uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t h = splitmix(seed ^ (uint64_t)i * 0x632BE59BD9B4E019ull);
        const float u = (float)(h >> 40) * (1.0f / 8388608.0f) - 1.0f;
        if (dt == DT_F32) ((float*)p)[i] = u;
        else if (dt == DT_BF16) ((uint16_t*)p)[i] = bf16_rne(u);
        else if (dt == DT_F8) p[i] = (uint8_t)((h & 0x80u) | ((h >> 8) % 0x38u));
        else p[i] = (uint8_t)h;
    }
}

// ------------------------------------------------------------------ operand packing

// Every job's destination block (rows_dst x ld_dst elements, contiguous) is
// cut into segments of kPackSeg consecutive elements, across row ends, so a
// narrow operand moves as much per wave as a wide one; seg_start[j] counts the
// segments of the jobs before j.  One wave per segment: lane l moves elements
// l, l + 64, l + 128, ... of the segment, so each wave-wide load (within a
// row) and store is one contiguous run, and all of the segment's loads are
// issued before its stores.  Elements outside the copied block are zero.
template <typename T>
__device__ inline void pack_segment(const PackJob& jb, int64_t q, int lane) {
    // lane l moves the 16-byte destination chunks l, l + 64, ... of the segment
    // (a chunk never crosses a destination row: ld_dst is a whole number of
    // chunks); the source row is read with dword-aligned 16-byte loads
    constexpr int EPV = 16 / (int)sizeof(T);
    constexpr int U = kPackSeg / (64 * EPV);
    const uint32_t n = (uint32_t)jb.rows_dst * (uint32_t)jb.ld_dst;  // < 2^31 (2 GiB operands)
    const uint32_t ld = (uint32_t)jb.ld_dst;
    const gbytes src = (gbytes)jb.src;
    u4_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t e = (uint32_t)q * kPackSeg + (uint32_t)(u * 64 + lane) * EPV;
        const uint32_t r = e / ld, c = e - r * ld;
        v[u] = u4_t{0u, 0u, 0u, 0u};
        if (e < n && r < (uint32_t)jb.rows && c < (uint32_t)jb.cols) {
            const gbytes row = src + (int64_t)r * jb.ld_src * (int64_t)sizeof(T);
            if (c + EPV <= (uint32_t)jb.cols) v[u] = load16_any<(int)sizeof(T)>(row + (int64_t)c * sizeof(T));
            else v[u] = load_unaligned<(int)sizeof(T)>(row, c, (int)(jb.cols - c));
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t e = (uint32_t)q * kPackSeg + (uint32_t)(u * 64 + lane) * EPV;
        if (e < n) *(u4_t*)((T*)jb.dst + e) = v[u];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_pack(const PackJob* __restrict__ jobs,
                                                   const int64_t* __restrict__ seg_start, int njobs,
                                                   int64_t total) {
    // wave w takes the contiguous segments [q0, q1): one search for its first
    // job, then the job index only moves forward
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t per = (total + nwaves - 1) / nwaves;
    const int64_t q0 = w * per, q1 = min(total, q0 + per);
    if (q0 >= q1) return;
    int j = 0, hi = njobs - 1;  // the last j with seg_start[j] <= q0
    while (j < hi) {
        const int mid = (j + hi + 1) >> 1;
        if (seg_start[mid] <= q0) j = mid;
        else hi = mid - 1;
    }
    int64_t s0 = seg_start[j], s1 = seg_start[j + 1];
    PackJob jb = jobs[j];
    for (int64_t q = q0; q < q1; ++q) {
        while (q >= s1) {
            ++j;
            s0 = s1;
            s1 = seg_start[j + 1];
            jb = jobs[j];
        }
        pack_segment<T>(jb, q - s0, lane);
    }
}

// the same for at most two jobs passed by value (one GEMM's A and B)
struct PackPair {
    PackJob job[2];
    int64_t segs0, total;  // segments of job 0, of both
};

template <typename T>
__global__ __launch_bounds__(kThreads) void k_pack_pair(PackPair pp) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; q < pp.total; q += nwaves) {
        if (q < pp.segs0) pack_segment<T>(pp.job[0], q, lane);
        else pack_segment<T>(pp.job[1], q - pp.segs0, lane);
    }
}

// ------------------------------------------------------------------ layout transform

// out[b][c][r] = in[b][r][c] for a batch of rows x cols matrices.  One tile
// of one batch entry per workgroup.  Generic form: a 32 x 32 LDS tile (one
// padding column keeps the column reads conflict-free).
template <typename T>
__device__ inline void transpose_tile32(const T* __restrict__ src, T* __restrict__ dst, int64_t rows,
                                        int64_t cols, int64_t bx, int64_t by, uint8_t* lds) {
    T (*tile)[33] = (T (*)[33])lds;
    const int64_t c0 = bx * 32, r0 = by * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = src[r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows) dst[c * rows + r] = tile[tx][i];
    }
}

// 2-byte elements with rows and columns multiples of 8 and 16-byte aligned
// rows: each thread moves one 8 x 8 block through registers, no LDS.  It reads
// the block's 8 rows as 16-byte loads (8 columns each), pairs the rows'
// halves into 32-bit words (column p of rows 2a and 2a + 1), and writes the
// block's 8 columns as 16-byte stores (8 rows each).  Lanes take the row
// groups fastest, so one load instruction of a wave reads 8 row segments of
// 128 bytes and one store instruction writes 8 output segments of 128 bytes.
// A workgroup covers 64 rows x 256 columns; a block is either whole or
// outside the matrix.
__device__ inline void transpose_blocks8_16(const uint16_t* __restrict__ src, uint16_t* __restrict__ dst,
                                            int64_t rows, int64_t cols, int64_t bx, int64_t by) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = by * 64 + 8 * (lane & 7);
    const int64_t c = bx * 256 + 8 * ((lane >> 3) + 8 * wave);
    if (r >= rows || c >= cols) return;
    u4_t in[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) in[e] = *(const u4_t*)(src + (r + e) * cols + c);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int w = j >> 1;
        u4_t out;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const uint32_t x = in[2 * a][w], y = in[2 * a + 1][w];
            out[a] = (j & 1) ? (x >> 16) | (y & 0xFFFF0000u) : (x & 0xFFFFu) | (y << 16);
        }
        *(u4_t*)(dst + (c + j) * rows + r) = out;
    }
}

// One batched transpose: tiles x-major, then y, then batch entry.
struct TransposeJob {
    const void* in;
    void* out;
    int64_t rows, cols;
    int64_t tiles_x, tiles_y;
    int64_t blocks;  // tiles_x * tiles_y * batch
    int wide;        // 2-byte elements moved as 8 x 8 blocks through registers
};

// Two batched transposes in one launch (the conv's input and filter to
// channels-last): workgroups [0, j0.blocks) take the first job, the rest the
// second.  The job choice is uniform per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_pair(TransposeJob j0, TransposeJob j1) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[32 * 33 * sizeof(T)];
    int64_t id = blockIdx.x;
    const bool second = id >= j0.blocks;
    const TransposeJob j = second ? j1 : j0;
    if (second) id -= j0.blocks;
    const int64_t bx = id % j.tiles_x, by = (id / j.tiles_x) % j.tiles_y, bz = id / (j.tiles_x * j.tiles_y);
    const int64_t off = bz * j.rows * j.cols;
    if constexpr (sizeof(T) == 2) {
        if (j.wide) {
            transpose_blocks8_16((const uint16_t*)j.in + off, (uint16_t*)j.out + off, j.rows, j.cols, bx, by);
            return;
        }
    }
    transpose_tile32<T>((const T*)j.in + off, (T*)j.out + off, j.rows, j.cols, bx, by, lds);
}

// ------------------------------------------------------------------ error statistics

constexpr int kErrBlocks = err_stats_parts();

// per-block partials: [sum d^2, sum r^2, max |d|, max |d|/bound]
__global__ __launch_bounds__(kThreads) void k_err_partial(int c_is_int, int64_t n,
                                                          const void* __restrict__ c,
                                                          const double* __restrict__ r,
                                                          const double* __restrict__ bound,
                                                          double* __restrict__ part) {
    double s2 = 0.0, r2 = 0.0, mx = 0.0, ratio = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double cv = c_is_int ? (double)((const int32_t*)c)[i] : (double)((const float*)c)[i];
        const double d = cv - r[i];
        s2 += d * d;
        r2 += r[i] * r[i];
        mx = fmax(mx, fabs(d));
        if (bound && bound[i] > 0.0) ratio = fmax(ratio, fabs(d) / bound[i]);
    }
    __shared__ double sh[4][kThreads];
    sh[0][threadIdx.x] = s2;
    sh[1][threadIdx.x] = r2;
    sh[2][threadIdx.x] = mx;
    sh[3][threadIdx.x] = ratio;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + w]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kThreads) void k_err_final(const double* __restrict__ part, int nb,
                                                        double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s2 = 0.0, r2 = 0.0, mx = 0.0, ratio = 0.0;
    for (int b = 0; b < nb; ++b) {
        s2 += part[4 * b];
        r2 += part[4 * b + 1];
        mx = fmax(mx, part[4 * b + 2]);
        ratio = fmax(ratio, part[4 * b + 3]);
    }
    out[0] = s2;
    out[1] = r2;
    out[2] = mx;
    out[3] = ratio;
}

}  // namespace

hipError_t launch_zero_matrix(void* C, int64_t M, int64_t N, int64_t ldc, int esize,
                              hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t rowbytes = N * esize;
    hipLaunchKernelGGL(k_zero_matrix, dim3(grid_for(M * rowbytes / 4, kThreads * 4)),
                       dim3(kThreads), 0, s, (uint8_t*)C, M, rowbytes, ldc * esize);
    return hipGetLastError();
}

hipError_t launch_quant_bf16(const float* x, int64_t n, uint16_t* q, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const bool vec = ((uintptr_t)x % 16 == 0) && ((uintptr_t)q % 16 == 0);
    if (vec)
        hipLaunchKernelGGL(k_quant_bf16, dim3(grid_for(n / 8 + 1, kThreads * 4)), dim3(kThreads), 0,
                           s, x, n, q);
    else
        hipLaunchKernelGGL(k_quant_bf16_scalar, dim3(grid_for(n, kThreads * 8)), dim3(kThreads), 0, s,
                           x, n, q);
    return hipGetLastError();
}

// The one-pass form when the whole input fits the resident grid's registers
// (16.8 M elements take 1,024 workgroups of 256 threads); hipErrorNotSupported,
// with nothing enqueued, otherwise.  Callers serialise through the library's
// scratch lock, so one launch at a time uses the exchange words of a device;
// the host keeps the last epoch it used there.
namespace {
struct FusedQuant {
    int grid_cap = 0;
    unsigned int epoch = 0;  // the last call's (device flags start at 0)
};
std::mutex g_fused_mu;
std::map<int, FusedQuant> g_fused;
}  // namespace

hipError_t launch_quant_e4m3_fused(const float* x, int64_t n, uint8_t* q, float* scale, hipStream_t s) {
    if (n <= 0 || (uintptr_t)x % 16 != 0 || (uintptr_t)q % 4 != 0) return hipErrorNotSupported;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_fused_mu);
    FusedQuant& st = g_fused[dev];
    if (st.grid_cap == 0) {
        int per_cu = 0, cus = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_quant_e4m3_fused, kThreads, 0)) !=
            hipSuccess)
            return e;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        st.grid_cap = std::max(1, std::min(per_cu * cus, kFusedMaxGrid));
    }
    const int64_t need = (n / 4 + (int64_t)kThreads * kFusedVec - 1) / ((int64_t)kThreads * kFusedVec);
    if (need > st.grid_cap) return hipErrorNotSupported;
    const int grid = (int)std::max<int64_t>(1, need);
    // (an epoch of 0 would match the flags' initial value: skip it on wrap)
    const unsigned int epoch = st.epoch + 1 == 0 ? 1 : st.epoch + 1;
    // ~1 << 18 sleeps of ~512 cycles: tens of milliseconds before a workgroup
    // stops waiting and computes the maximum itself.  MLK_QUANT_WAIT_POLLS
    // sets the bound instead (0: one round of polls), so that a test can
    // drive the fallback from the host.
    unsigned int polls = 1u << 18;
    if (const char* env = getenv("MLK_QUANT_WAIT_POLLS")) polls = (unsigned int)strtoul(env, nullptr, 10);
    hipLaunchKernelGGL(k_quant_e4m3_fused, dim3(grid), dim3(kThreads), 0, s, x, n, q, scale, epoch, polls);
    e = hipGetLastError();
    if (e == hipSuccess) st.epoch = epoch;
    return e;
}

hipError_t launch_quant_e4m3(const float* x, int64_t n, uint8_t* q, float* scale, float* part,
                             hipStream_t s) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_scale_one, dim3(1), dim3(1), 0, s, scale);
        return hipGetLastError();
    }
    const bool vec = ((uintptr_t)x % 16 == 0) && ((uintptr_t)q % 16 == 0);
    const int nparts = (int)std::min<int64_t>(kAmaxBlocks, grid_for(vec ? n / 4 + 1 : n, kThreads));
    if (vec) {
        hipLaunchKernelGGL(k_amax<true>, dim3(nparts), dim3(kThreads), 0, s, x, n, part);
        hipLaunchKernelGGL(k_quant_e4m3, dim3(grid_for(n / 16 + 1, kThreads * 2)), dim3(kThreads), 0, s, x,
                           n, (const float*)part, nparts, q, scale);
    } else {
        hipLaunchKernelGGL(k_amax<false>, dim3(nparts), dim3(kThreads), 0, s, x, n, part);
        hipLaunchKernelGGL(k_quant_e4m3_scalar, dim3(grid_for(n, kThreads * 8)), dim3(kThreads), 0, s, x, n,
                           (const float*)part, nparts, q, scale);
    }
    return hipGetLastError();
}

static TransposeJob transpose_job(const void* in, void* out, int64_t batch, int64_t rows, int64_t cols,
                                  int esize) {
    TransposeJob j{in, out, rows, cols, 0, 0, 0, 0};
    if (batch <= 0 || rows <= 0 || cols <= 0) return j;
    j.wide = esize == 2 && rows % 8 == 0 && cols % 8 == 0 && (uintptr_t)in % 16 == 0 && (uintptr_t)out % 16 == 0;
    // the wide form: 64 rows x 256 columns per workgroup; else 32 x 32 tiles
    j.tiles_x = (cols + (j.wide ? 255 : 31)) / (j.wide ? 256 : 32);
    j.tiles_y = (rows + (j.wide ? 63 : 31)) / (j.wide ? 64 : 32);
    j.blocks = j.tiles_x * j.tiles_y * batch;
    return j;
}

hipError_t launch_transpose_pair(const void* in0, void* out0, int64_t batch0, int64_t rows0, int64_t cols0,
                                 const void* in1, void* out1, int64_t batch1, int64_t rows1, int64_t cols1,
                                 int esize, hipStream_t s) {
    const TransposeJob j0 = transpose_job(in0, out0, batch0, rows0, cols0, esize);
    const TransposeJob j1 = transpose_job(in1, out1, batch1, rows1, cols1, esize);
    const int64_t blocks = j0.blocks + j1.blocks;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (esize == 4)
        hipLaunchKernelGGL(k_transpose_pair<uint32_t>, grid, dim3(256), 0, s, j0, j1);
    else if (esize == 2)
        hipLaunchKernelGGL(k_transpose_pair<uint16_t>, grid, dim3(256), 0, s, j0, j1);
    else
        hipLaunchKernelGGL(k_transpose_pair<uint8_t>, grid, dim3(256), 0, s, j0, j1);
    return hipGetLastError();
}

hipError_t launch_pack(const PackJob* jobs, const int64_t* seg_start, int njobs, int64_t total_segs,
                       int esize, hipStream_t s) {
    if (njobs <= 0 || total_segs <= 0) return hipSuccess;
    const int grid = grid_for(total_segs, kThreads / 64);
    if (esize == 4)
        hipLaunchKernelGGL(k_pack<uint32_t>, dim3(grid), dim3(kThreads), 0, s, jobs, seg_start, njobs, total_segs);
    else if (esize == 2)
        hipLaunchKernelGGL(k_pack<uint16_t>, dim3(grid), dim3(kThreads), 0, s, jobs, seg_start, njobs, total_segs);
    else
        hipLaunchKernelGGL(k_pack<uint8_t>, dim3(grid), dim3(kThreads), 0, s, jobs, seg_start, njobs, total_segs);
    return hipGetLastError();
}

hipError_t launch_pack_pair(const PackJob* jobs, int njobs, int esize, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    PackPair pp;
    memset(&pp, 0, sizeof pp);
    pp.job[0] = jobs[0];
    if (njobs > 1) pp.job[1] = jobs[1];
    pp.segs0 = pack_segments(jobs[0]);
    pp.total = pp.segs0 + (njobs > 1 ? pack_segments(jobs[1]) : 0);
    if (pp.total <= 0) return hipSuccess;
    const int grid = grid_for(pp.total, kThreads / 64);
    if (esize == 4) hipLaunchKernelGGL(k_pack_pair<uint32_t>, dim3(grid), dim3(kThreads), 0, s, pp);
    else if (esize == 2) hipLaunchKernelGGL(k_pack_pair<uint16_t>, dim3(grid), dim3(kThreads), 0, s, pp);
    else hipLaunchKernelGGL(k_pack_pair<uint8_t>, dim3(grid), dim3(kThreads), 0, s, pp);
    return hipGetLastError();
}

hipError_t launch_fill_random(void* p, int64_t n, int dt, uint64_t seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_random, dim3(grid_for(n, kThreads * 8)), dim3(kThreads), 0, s,
                       (uint8_t*)p, n, dt, seed);
    return hipGetLastError();
}

hipError_t launch_err_stats(int c_is_int, int64_t n, const void* c, const double* r,
                            const double* bound, double* out, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_err_partial, dim3(kErrBlocks), dim3(kThreads), 0, s, c_is_int, n, c, r,
                       bound, part);
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(64), 0, s, (const double*)part, kErrBlocks, out);
    return hipGetLastError();
}

}  // namespace mlk
