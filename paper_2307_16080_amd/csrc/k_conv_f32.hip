// k_conv_f32.hip -- fp32 implicit-GEMM convolution (Sec. 4.1 `2dnchwconv`,
// y[n, f, oh, ow] += sum_{c, kh, kw} w[f, c, kh, kw] x[n, c, oh*s + kh - p, ow*s + kw - p])
// with deep K chunks gathered whole from the NCHW input.
//
// The output tile is BM filters x BN output pixels (pixels p = (n, oh, ow)
// flattened); the contraction runs over k = (c, kh, kw) in chunks of BK.  A
// whole chunk of both operands is requested at once (every thread holds
// BM*BK/NT + BN*BK/NT floats in registers), and up to PF chunks are in flight
// in a ring of register sets (PF as many as about 96 VGPRs hold, at most 6);
// each chunk is stored into one LDS buffer and multiplied.  Small layers (a
// batch-1 56 x 56 x 64 3 x 3 layer has 49 tiles of 64 x 64) split K so that
// each workgroup holds at most PF chunks: all of its loads are issued before
// the first is waited for, so the launch costs one round trip to memory, a
// few hundred MFMAs per wave and the partial sums' atomic adds, where the
// 16-deep stages of the general tile kernel cost one round trip each.
//
// The gather is wave-uniform in k: a thread's 4-element groups are
// (pixel = lane-consecutive, k group = the same for the whole wave), so the
// decomposition k -> (c, kh, kw) is scalar work (division by the filter's
// tap counts through a multiply-high by a reciprocal computed once per
// workgroup), and each element costs one bounds test and one 4-byte load of
// consecutive pixels across the wave.
//
// LDS holds A as [BM][BK] and B as [BN][BK] (k contiguous, rows padded by 16
// bytes so that 16 consecutive rows start in distinct banks).  Each lane reads
// 16 bytes = four consecutive k of one row; the four MFMAs 16x16x4 f32 that
// consume them take, in MFMA s, k = 4 * (lane / 16) + s of each 16-deep group
// from A and B alike, so the sum covers every k of the group once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace mlk {

namespace {

typedef float fv4 __attribute__((ext_vector_type(4)));

// floor(k / d) for k * d < 2^32 by a multiply-high with ceil(2^32 / d)
struct Divider {
    uint32_t d, m;
    __device__ explicit Divider(uint32_t dd) : d(dd), m(dd <= 1 ? 0u : 0xFFFFFFFFu / dd + 1u) {}
    __device__ uint32_t div(uint32_t k) const { return d <= 1 ? k : __umulhi(k, m); }
};

template <int BM, int BN, int BK, int WM, int WN>
struct ChunkConv {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int WTM = BM / WM, WTN = BN / WN;
    static constexpr int TM = WTM / 16, TN = WTN / 16;
    static constexpr int PITCH = BK * 4 + 16;          // LDS row pitch (bytes)
    static constexpr int LDS_BYTES = (BM + BN) * PITCH;
    static constexpr int KQ = BK / 4;                   // 4-element k groups per row
    static constexpr int NA = BM * KQ / NT;             // A groups per thread
    static constexpr int NB = BN * KQ / NT;             // B groups per thread
    static constexpr int NPIX = BN > NT ? BN / NT : 1;  // distinct pixels per thread
    // register sets in flight: as many chunks as about 96 VGPRs hold, 1 to 6
    static constexpr int SET_REGS = 4 * (NA + NB);
    static constexpr int PF = 96 / SET_REGS < 1 ? 1 : 96 / SET_REGS > 6 ? 6 : 96 / SET_REGS;

    static_assert(BN % 64 == 0, "a wave's B groups share one k group: BN a multiple of 64");
    static_assert(NT % BN == 0 || BN % NT == 0, "pixel slots");
    static_assert((BM * KQ) % NT == 0 && (BN * KQ) % NT == 0, "whole groups per thread");
    static_assert(WTM % 16 == 0 && WTN % 16 == 0 && BK % 16 == 0, "MFMA tiles");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");

    struct Pix {
        int64_t base;  // element offset of tap (0, 0, 0): img*C*H*W + ih0*W + iw0 (negative
                       // when the window starts in the padding; used only for taps inside)
        int ih0, iw0;  // window origin; far outside the image for a pixel past P
    };

    __device__ static inline void load(const GemmArgs& g, int64_t k0, int tid, uint32_t wb, const Pix* px,
                                       const Divider& dtap, const Divider& dkw, fv4* ra, fv4* rb,
                                       int64_t m0) {
        // A: the filter, F x K row-major (pitch lda)
        const float* W = (const float*)g.A;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int L = tid + i * NT;
            const int m = L / KQ, kq = L % KQ;
            const int64_t f = m0 + m, k = k0 + 4 * kq;
            fv4 v = fv4{0.f, 0.f, 0.f, 0.f};
            if (f < g.M) {
                const float* row = W + f * g.lda;
                if (g.vec_a && k + 4 <= g.K) {
                    v = *(const fv4*)(row + k);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (k + e < g.K) v[e] = row[k + e];
                }
            }
            ra[i] = v;
        }
        // B: implicit im2col; this wave's groups all have the same k
        const float* X = (const float*)g.B;
        const int hw = g.ch * g.cw;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const uint32_t Lw = wb + (uint32_t)(i * NT);  // the wave's first group index (uniform)
            const uint32_t kg = Lw / BN;
            const Pix& p = px[NT >= BN ? 0 : i % NPIX];
            fv4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = k0 + 4 * (int64_t)kg + e;
                const uint32_t ku = (uint32_t)k;
                const uint32_t c = dtap.div(ku);
                const uint32_t r = ku - c * dtap.d;
                const uint32_t kh = dkw.div(r);
                const uint32_t kw = r - kh * dkw.d;
                const int off = (int)c * hw + (int)kh * g.cw + (int)kw;
                const bool in = k < g.K && (unsigned)(p.ih0 + (int)kh) < (unsigned)g.ch &&
                                (unsigned)(p.iw0 + (int)kw) < (unsigned)g.cw;
                v[e] = in ? X[p.base + off] : 0.f;
            }
            rb[i] = v;
        }
    }

    __device__ static inline void store(uint8_t* lds, int tid, const fv4* ra, const fv4* rb) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int L = tid + i * NT;
            *(fv4*)(lds + (L / KQ) * PITCH + (L % KQ) * 16) = ra[i];
        }
        uint8_t* sb = lds + BM * PITCH;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int L = tid + i * NT;
            *(fv4*)(sb + (L % BN) * PITCH + (L / BN) * 16) = rb[i];
        }
    }

    __device__ static inline void run(const GemmArgs& g, int tm, int tn, int kz, uint8_t* lds) {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wy = wave / WN, wx = wave % WN;
        const int lr = lane & 15, lg = lane >> 4;
        const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

        const int64_t kstages = (g.K + BK - 1) / BK;
        const int64_t per = (kstages + g.split_k - 1) / g.split_k;
        const int64_t s_beg = (int64_t)kz * per;
        const int nk = (int)max<int64_t>(0, min<int64_t>(kstages, s_beg + per) - s_beg);
        // a part of a K split with nothing to add leaves the (pre-zeroed or
        // accumulated) output alone
        if (nk == 0 && g.atomic) return;

        const Divider dtap((uint32_t)(g.ckh * g.ckw)), dkw((uint32_t)g.ckw);
        const uint32_t wb = (uint32_t)__builtin_amdgcn_readfirstlane(tid & ~63);

        // this thread's output pixels (fixed for the tile)
        Pix px[NPIX];
        {
            const int64_t P = (int64_t)g.cn * g.cho * g.cwo;
            const int hwo = g.cho * g.cwo;
#pragma unroll
            for (int s = 0; s < NPIX; ++s) {
                const int pn = NT >= BN ? tid % BN : tid + NT * s;
                const int64_t pp = n0 + pn;
                if (pp < P) {
                    const int img = (int)(pp / hwo), q = (int)(pp - (int64_t)img * hwo);
                    const int oh = q / g.cwo, ow = q - oh * g.cwo;
                    px[s].ih0 = oh * g.csh - g.cph;
                    px[s].iw0 = ow * g.csw - g.cpw;
                    px[s].base = (int64_t)img * g.cc * g.ch * g.cw + (int64_t)px[s].ih0 * g.cw + px[s].iw0;
                } else {
                    px[s].ih0 = -(1 << 28);
                    px[s].iw0 = -(1 << 28);
                    px[s].base = 0;
                }
            }
        }

        fv4 acc[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = fv4{0.f, 0.f, 0.f, 0.f};

        // a ring of PF register sets: chunks c .. c+PF-1 are in flight while
        // chunk c is stored and multiplied (a part of one to PF chunks issues
        // every load before its first store)
        fv4 ra[PF][NA], rb[PF][NB];
#pragma unroll
        for (int u = 0; u < PF; ++u)
            if (u < nk) load(g, (s_beg + u) * BK, tid, wb, px, dtap, dkw, ra[u], rb[u], m0);
        const uint8_t* sa = lds + (wy * WTM + lr) * PITCH + lg * 16;
        const uint8_t* sb = lds + BM * PITCH + (wx * WTN + lr) * PITCH + lg * 16;
        for (int it = 0; it < nk; it += PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int c = it + u;
                if (c < nk) {
                    if (c > 0) __syncthreads();  // every wave is done with the previous chunk
                    store(lds, tid, ra[u], rb[u]);
                    __syncthreads();
                    if (c + PF < nk) load(g, (s_beg + c + PF) * BK, tid, wb, px, dtap, dkw, ra[u], rb[u], m0);
#pragma unroll
                    for (int q = 0; q < BK / 16; ++q) {
                        fv4 af[TM];
#pragma unroll
                        for (int i = 0; i < TM; ++i) af[i] = *(const fv4*)(sa + i * 16 * PITCH + q * 64);
#pragma unroll
                        for (int j = 0; j < TN; ++j) {
                            const fv4 bj = *(const fv4*)(sb + j * 16 * PITCH + q * 64);
#pragma unroll
                            for (int i = 0; i < TM; ++i)
#pragma unroll
                                for (int s = 0; s < 4; ++s)
                                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bj[s], acc[i][j], 0, 0, 0);
                        }
                    }
                }
            }
        }

        // output (f, p) of NFHW: y[img(p) * F * HWO + f * HWO + pix(p)]
        const int64_t P = (int64_t)g.cn * g.cho * g.cwo;
        const int64_t hwo = (int64_t)g.cho * g.cwo;
        float* Y = (float*)g.C;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t p = n0 + wx * WTN + j * 16 + lr;
            if (p >= P) continue;
            const int64_t img = p / hwo;
            float* col = Y + img * g.M * hwo + (p - img * hwo);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t f = m0 + wy * WTM + i * 16 + lg * 4 + r;
                    if (f >= g.M) continue;
                    float* o = col + f * hwo;
                    const float v = acc[i][j][r];
                    if (g.atomic) __hip_atomic_fetch_add(o, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    else if (g.accumulate) *o = *o + v;
                    else *o = v;
                }
        }
    }
};

template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_conv_chunk_f32(GemmArgs g) {
    typedef ChunkConv<BM, BN, BK, WM, WN> CC;
    __shared__ __attribute__((aligned(16))) uint8_t lds[CC::LDS_BYTES];
    int tm, tn, kz;
    tile_coords(g, blockIdx.x, gridDim.x, tm, tn, kz);
    CC::run(g, tm, tn, kz, lds);
}

template <int BM, int BN, int BK, int WM, int WN>
hipError_t launch_conv_chunk(const GemmArgs& g, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_conv_chunk_f32<BM, BN, BK, WM, WN>), dim3(nblk), dim3(64 * WM * WN), 0, s, g);
    return hipGetLastError();
}

}  // namespace

// Registry entries: fp32 conv, stages 1 (operands loaded through registers),
// layout 0 (gathered from NCHW); bk = the chunk depth.
#define MLK_ENTRY_CHUNK(BM, BN, BK, WM, WN)                                                              \
    KernelEntry {                                                                                        \
        DT_F32, 1, 1, BM, BN, BK, WM, WN, ChunkConv<BM, BN, BK, WM, WN>::LDS_BYTES, 64 * (WM) * (WN),    \
            &launch_conv_chunk<BM, BN, BK, WM, WN>, nullptr, nullptr, nullptr, nullptr, nullptr, 16,     \
            nullptr, nullptr, nullptr                                                                    \
    }

const KernelEntry* kernels_conv_chunk(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY_CHUNK(64, 64, 16, 2, 2),  MLK_ENTRY_CHUNK(64, 64, 32, 2, 2),  MLK_ENTRY_CHUNK(64, 64, 64, 2, 2),
        MLK_ENTRY_CHUNK(64, 64, 128, 2, 2), MLK_ENTRY_CHUNK(32, 64, 32, 1, 2),
        MLK_ENTRY_CHUNK(32, 64, 64, 1, 2),  MLK_ENTRY_CHUNK(32, 64, 128, 1, 2), MLK_ENTRY_CHUNK(64, 128, 64, 2, 2),
        MLK_ENTRY_CHUNK(32, 128, 64, 1, 2), MLK_ENTRY_CHUNK(16, 64, 64, 1, 1),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}

}  // namespace mlk
