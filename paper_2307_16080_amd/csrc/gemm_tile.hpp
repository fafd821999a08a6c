// gemm_tile.hpp -- the workgroup-tiled MFMA contraction shared by every dense
// kernel of the library (matmul in fp32 / bf16 / e4m3 / int8, the implicit-GEMM
// conv2d, and the persistent batched GEMM).
//
// What is computed is linalg.matmul, C[M,N] (+)= A[M,K] * B[K,N] (paper
// Sec. 2.1, listing "linalg-matmul"), or, with the conv operand policy,
// linalg.conv_2d_nchw_fchw (Sec. 4.1, listing "2dnchwconv") viewed as
// rows = output channels, columns = output pixels, depth = (c, kh, kw).
// The paper maps each output element to a GPU block and notes that tiling
// introduces a block x thread distribution; here one workgroup owns a BM x BN
// output tile, each 64-lane wave a (BM/WM) x (BN/WN) sub-tile made of 16x16
// MFMA tiles, and the contraction runs through LDS in stages of KB bytes per
// row.
//
// LDS layout: both operands are stored "K-contiguous": row r of the A stage
// holds A[m0 + r, k0 ...] and row n of the B stage holds B[k0 ..., n0 + n],
// each row KB bytes plus 16 bytes of padding (which spreads consecutive rows
// over different banks).  A is copied as is; B (row-major, N-contiguous in
// HBM) is transposed in registers on its way from HBM to LDS, in blocks of
// EPV x EPV elements (EPV = elements per 16 bytes), so that every lane then
// reads its MFMA operand with one 16-byte LDS load.
//
// MFMA operand convention (16x16 output tile, 64 lanes): lane l supplies row
// (l % 16) of the A tile and column (l % 16) of the B tile; the 16 or 32 bytes
// it supplies along K are bytes [g*KS/4, (g+1)*KS/4) of the current K step,
// g = l / 16.  A and B use the same (lane group, byte) -> k assignment, so the
// MFMA sums exactly the products of matching k.  The result lane l, register
// r holds output (4*(l/16) + r, l % 16).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mlk {

enum : int { DT_F32 = 0, DT_BF16 = 1, DT_F8 = 2, DT_I8 = 3 };

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i4_t __attribute__((ext_vector_type(4)));
typedef int i8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

// fp32 -> bf16 code: round to nearest, ties to even; a NaN stays a quiet NaN
// with its sign, overflow rounds to inf.  Adding 0x7FFF plus the kept part's
// lowest bit and truncating rounds half-way cases to the even neighbour.
__device__ inline uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0)
        return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
// bf16 code -> its (exact) fp32 value
__device__ inline float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int DT> struct Traits;
template <> struct Traits<DT_F32> {
    static constexpr int ES = 4;   // element size (bytes)
    static constexpr int KS = 64;  // bytes of one row consumed per K step
    typedef f4_t acc_t;
    typedef float out_t;
};
template <> struct Traits<DT_BF16> {
    static constexpr int ES = 2;
    static constexpr int KS = 64;
    typedef f4_t acc_t;
    typedef float out_t;
};
template <> struct Traits<DT_I8> {
    static constexpr int ES = 1;
    static constexpr int KS = 64;
    typedef i4_t acc_t;
    typedef int32_t out_t;
};
template <> struct Traits<DT_F8> {
    static constexpr int ES = 1;
    static constexpr int KS = 128;
    typedef f4_t acc_t;
    typedef float out_t;
};

// Everything a tile needs to know about one GEMM (or one convolution).
struct GemmArgs {
    int64_t M, N, K;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    void* C;
    int64_t ldc;
    const float* scale_a;  // e4m3 only; may be null (= 1)
    const float* scale_b;
    int32_t accumulate;    // 1: C += result
    int32_t atomic;        // 1: add partial results with atomics (split K)
    int32_t split_k;
    int32_t vec_a;         // 1: A rows are 16-byte aligned (vector loads allowed)
    int32_t vec_b;
    int32_t tiles_m, tiles_n;
    int32_t group_m, xcd_remap;
    // convolution view (conv policy only)
    int32_t cn, cc, ch, cw, ckh, ckw, csh, csw, cph, cpw, cho, cwo;
    // Linear layer: bias[n] added to every row of the product (float outputs,
    // GEMM policy only); null for a plain product.  Under split K only the
    // first split adds it.
    const float* bias;
    // 1: C holds bf16 codes (float results rounded once, to nearest even;
    // GEMM policy only, split_k 1); accumulate reads them back as fp32
    int32_t out_bf16;
};

// ---------------------------------------------------------------- MFMA step

template <int DT> struct Mma;
template <> struct Mma<DT_F32> {
    __device__ static inline void run(f4_t& c, const u4_t* a, const u4_t* b) {
        // one 16-byte operand = 4 consecutive k per lane = 4 MFMA 16x16x4
#pragma unroll
        for (int s = 0; s < 4; ++s)
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[0][s]),
                                                     __uint_as_float(b[0][s]), c, 0, 0, 0);
    }
};
template <> struct Mma<DT_BF16> {
    __device__ static inline void run(f4_t& c, const u4_t* a, const u4_t* b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a[0]),
                                                    __builtin_bit_cast(bf8_t, b[0]), c, 0, 0, 0);
    }
};
template <> struct Mma<DT_I8> {
    __device__ static inline void run(i4_t& c, const u4_t* a, const u4_t* b) {
        c = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i4_t, a[0]),
                                                  __builtin_bit_cast(i4_t, b[0]), c, 0, 0, 0);
    }
};
template <> struct Mma<DT_F8> {
    __device__ static inline void run(f4_t& c, const u4_t* a, const u4_t* b) {
        i8_t av = {(int)a[0][0], (int)a[0][1], (int)a[0][2], (int)a[0][3],
                   (int)a[1][0], (int)a[1][1], (int)a[1][2], (int)a[1][3]};
        i8_t bv = {(int)b[0][0], (int)b[0][1], (int)b[0][2], (int)b[0][3],
                   (int)b[1][0], (int)b[1][1], (int)b[1][2], (int)b[1][3]};
        // format code 0 = OCP E4M3 for both operands; block scales 2^(127-127) = 1
        c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    }
};

// ---------------------------------------------------------------- helpers

// Global-memory views.  Accesses through these compile to global_load /
// global_store; through a generic pointer they would be flat accesses, which
// also count against the LDS wait counter and so serialise with LDS traffic.
#define MLK_GLOBAL __attribute__((address_space(1)))
typedef const MLK_GLOBAL uint8_t* gbytes;
typedef uint32_t u4a_t __attribute__((ext_vector_type(4), aligned(4)));

__host__ __device__ inline uint32_t funnel32(uint32_t lo, uint32_t hi, int byteshift) {
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * byteshift));
}

// The 16 bytes at p, all of them wanted, for a p that is a multiple of the
// element size but not necessarily of 4 or 16: one dword-aligned 16-byte load
// and, when p is not dword aligned, the dword after it, joined by byte shifts.
// Every dword read holds a wanted byte (when p is dword aligned the last dword
// is read again instead of the next one).
template <int ES>
__device__ inline u4_t load16_any(gbytes p) {
    const uintptr_t a = (uintptr_t)p;
    const int sh = (int)(a & 3);
    const gbytes q = (gbytes)(a - (uintptr_t)sh);
    const u4a_t lo = *(const MLK_GLOBAL u4a_t*)q;
    if constexpr (ES == 4) {
        return u4_t{lo[0], lo[1], lo[2], lo[3]};
    } else {
        const uint32_t hi = *(const MLK_GLOBAL uint32_t*)(q + (sh ? 16 : 12));
        return u4_t{funnel32(lo[0], lo[1], sh), funnel32(lo[1], lo[2], sh),
                    funnel32(lo[2], lo[3], sh), funnel32(lo[3], hi, sh)};
    }
}

// The 16 bytes holding elements [e0, e0 + nvalid) of a row (zero beyond):
// the tail of a row, where reading past the wanted bytes could leave the
// operand.  Reads the (at most two) aligned 16-byte blocks that contain the
// wanted bytes and shifts them into place; an aligned block that holds a
// wanted byte lies in the same page as that byte.
template <int ES>
__device__ inline u4_t load_unaligned(gbytes row, int64_t e0, int nvalid) {
    const uintptr_t a = (uintptr_t)(row + e0 * ES);
    const MLK_GLOBAL u4_t* blk = (const MLK_GLOBAL u4_t*)(a & ~(uintptr_t)15);
    const int sh = (int)(a & 15);
    const int nbytes = nvalid * ES;
    const u4_t lo = blk[0];
    const u4_t hi = (sh + nbytes > 16) ? blk[1] : u4_t{0u, 0u, 0u, 0u};
    const uint32_t w[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    const int q = sh >> 2, r = sh & 3;
    u4_t v;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        // dwords d + q and d + q + 1 of the 32-byte window, selected without
        // dynamic register indexing
        uint32_t x0 = w[d], x1 = w[d + 1];
        if (q == 1) { x0 = w[d + 1]; x1 = w[d + 2]; }
        if (q == 2) { x0 = w[d + 2]; x1 = w[d + 3]; }
        if (q == 3) { x0 = w[d + 3]; x1 = w[d + 4]; }
        uint32_t x = funnel32(x0, x1, r);
        const int keep = nbytes - 4 * d;  // valid bytes in this dword
        if (keep <= 0) x = 0u;
        else if (keep < 4) x &= (1u << (8 * keep)) - 1u;
        v[d] = x;
    }
    return v;
}

// Transpose an EPV x EPV block of ES-byte elements held as EPV rows of 16 bytes.
template <int ES>
__device__ inline void transpose_block(const u4_t* in, u4_t* out) {
    if constexpr (ES == 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[j][i] = in[i][j];
    } else if constexpr (ES == 2) {
        // out[j] holds element j of rows 0..7; dword p of out[j] = rows 2p, 2p+1
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t lo = in[2 * p][j >> 1], hi = in[2 * p + 1][j >> 1];
                out[j][p] = (j & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u))
                                    : ((lo & 0xFFFFu) | (hi << 16));
            }
    } else {
        // 16 x 16 bytes: dword p of out[j] = byte j of rows 4p .. 4p+3
#pragma unroll
        for (int j = 0; j < 16; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int sh = 8 * (j & 3);
                const uint32_t b0 = (in[4 * p + 0][j >> 2] >> sh) & 0xFFu;
                const uint32_t b1 = (in[4 * p + 1][j >> 2] >> sh) & 0xFFu;
                const uint32_t b2 = (in[4 * p + 2][j >> 2] >> sh) & 0xFFu;
                const uint32_t b3 = (in[4 * p + 3][j >> 2] >> sh) & 0xFFu;
                out[j][p] = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
            }
    }
}

// Logical tile of workgroup `bid` (of `nblk`): XCD remap, then grouped raster.
__device__ inline void tile_coords(const GemmArgs& g, int bid, int nblk, int& tm, int& tn,
                                   int& kz) {
    if (g.xcd_remap && (nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
    kz = bid % g.split_k;
    int t = bid / g.split_k;
    const int gm = g.group_m < 1 ? 1 : g.group_m;
    const int width = gm * g.tiles_n;
    const int first_m = (t / width) * gm;
    const int rows = min(g.tiles_m - first_m, gm);
    tm = first_m + (t % width) % rows;
    tn = (t % width) / rows;
}

// ---------------------------------------------------------------- the tile

// Operand policies.  CONV = 0: dense row-major A, B, C.  CONV = 1: A = filter
// (F x C*KH*KW, row-major), B = implicit im2col of the NCHW input, k ordered
// (c, kh, kw), C = NFHW output.  CONV = 2: the channels-last form: A = filter
// laid out F x KH x KW x C, B gathered from an NHWC copy of the input, k
// ordered (kh, kw, c); with C a multiple of the 16-byte vector, every B load
// is one aligned 16-byte read of consecutive channels, stored into LDS as is
// (no transpose).  The output is NFHW in both conv policies.
// Output stage: EPI = 0 the plain product; 1 adds the Linear layer's bias to
// an fp32 C; 2 writes a bf16 C (bias optional).  Each is its own instantiation.
template <int DT, int BM, int BN, int KB, int WM, int WN, int CONV, int EPI = 0>
struct Tile {
    typedef Traits<DT> T;
    typedef typename T::acc_t acc_t;
    typedef typename T::out_t out_t;
    static constexpr int ES = T::ES;
    static constexpr int KS = T::KS;
    static constexpr int EPV = 16 / ES;          // elements per 16 bytes
    static constexpr int NT = 64 * WM * WN;      // threads
    static constexpr int PITCH = KB + 16;         // LDS row pitch (bytes)
    static constexpr int STAGE = (BM + BN) * PITCH;
    static constexpr int LDS_BYTES = 2 * STAGE;
    static constexpr int BK = KB / ES;           // elements of K per stage
    static constexpr int WTM = BM / WM, WTN = BN / WN;
    static constexpr int TM = WTM / 16, TN = WTN / 16;
    static constexpr int CPR = KB / 16;          // 16-byte chunks per row
    static constexpr int NA = (BM * CPR + NT - 1) / NT;      // A chunks per thread
    static constexpr int NBLK = (BK / EPV) * (BN / EPV);     // B transpose blocks
    static constexpr int NB = CONV == 2 ? 0 : (NBLK + NT - 1) / NT;  // B blocks per thread
    static constexpr int NB2 = CONV == 2 ? (BN * CPR + NT - 1) / NT : 0;  // channels-last B chunks
    static constexpr int KV = KS / 64;                       // 16-byte regs per MFMA operand

    static_assert(KB % KS == 0, "stage depth must hold whole K steps");
    static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "wave tile must be 16-aligned");
    static_assert(BK % EPV == 0 && BN % EPV == 0, "B blocks must tile the stage");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");

    // ---- global -> registers
    __device__ static inline void load_a(const GemmArgs& g, int64_t m0, int64_t k0, u4_t* ra,
                                         int tid) {
        const gbytes A = (gbytes)g.A;
        const bool kfull = k0 + BK <= g.K;  // every chunk of this stage lies inside K
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int c = tid + i * NT;
            ra[i] = u4_t{0u, 0u, 0u, 0u};
            if ((BM * CPR) % NT != 0 && c >= BM * CPR) continue;
            const int r = c / CPR, cc = c % CPR;
            const int64_t m = m0 + r, k = k0 + cc * EPV;
            if (m >= g.M) continue;
            const gbytes row = A + m * g.lda * ES;
            if (kfull || k + EPV <= g.K)
                ra[i] = g.vec_a ? *(const MLK_GLOBAL u4_t*)(row + k * ES) : load16_any<ES>(row + k * ES);
            else if (k < g.K)
                ra[i] = load_unaligned<ES>(row, k, (int)(g.K - k));
        }
    }

    struct NoCols {};
    template <class Cols>
    __device__ static inline void load_b(const GemmArgs& g, int64_t n0, int64_t k0, u4_t* rb,
                                         int tid, const Cols* cols) {
        if constexpr (CONV == 2) {
            nhwc_gather(g, k0, rb, tid, cols);
            return;
        }
        const bool kfull = k0 + BK <= g.K;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int blk = tid + i * NT;
            u4_t* v = rb + i * EPV;
#pragma unroll
            for (int e = 0; e < EPV; ++e) v[e] = u4_t{0u, 0u, 0u, 0u};
            if (NBLK % NT != 0 && blk >= NBLK) continue;
            const int kr = blk / (BN / EPV), nc = blk % (BN / EPV);
            const int64_t kb = k0 + kr * EPV, n = n0 + nc * EPV;
            if constexpr (CONV == 0) {
                if (n >= g.N) continue;
                const gbytes B = (gbytes)g.B;
                const int64_t pitch = g.ldb * ES;
                const int nval = (int)min<int64_t>(EPV, g.N - n);
                if (nval == EPV && (kfull || kb + EPV <= g.K)) {
                    const gbytes p = B + kb * pitch + n * ES;
                    if (g.vec_b) {
#pragma unroll
                        for (int e = 0; e < EPV; ++e) v[e] = *(const MLK_GLOBAL u4_t*)(p + e * pitch);
                    } else {
#pragma unroll
                        for (int e = 0; e < EPV; ++e) v[e] = load16_any<ES>(p + e * pitch);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < EPV; ++e) {
                        const int64_t k = kb + e;
                        if (k < g.K) v[e] = load_unaligned<ES>(B + k * pitch, n, nval);
                    }
                }
            } else if constexpr (CONV == 1) {
                conv_gather(g, cols[i], kb, v);
            }
        }
    }

    // Implicit im2col for the conv policy.  Columns p = (img, oh, ow) of a
    // transpose block are fixed for the whole tile, so their input offsets
    // are computed once (ConvCols); the rows k = (c, kh, kw) of a block are
    // decomposed once per stage and then stepped (kw fastest).  A block whose
    // columns are all valid and whose windows lie inside the image needs no
    // bounds checks at all.
    struct ConvCols {
        int cbase[EPV];  // img*C*H*W + ih0*W + iw0 (element offset of tap (0,0,0))
        int ih0[EPV], iw0[EPV];
        int interior;    // every column valid and its whole window inside the image
        int any;         // at least one valid column
    };

    __device__ static inline void conv_cols(const GemmArgs& g, int64_t n0, int tid, ConvCols* cols) {
        const int64_t P = (int64_t)g.cn * g.cho * g.cwo;
        const int hw = g.cho * g.cwo;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int blk = tid + i * NT;
            const int nc = blk % (BN / EPV);
            ConvCols& cc = cols[i];
            cc.interior = (NBLK % NT != 0 && blk >= NBLK) ? 0 : 1;
            cc.any = 0;
#pragma unroll
            for (int j = 0; j < EPV; ++j) {
                const int64_t p = n0 + nc * EPV + j;
                if (p < P && !(NBLK % NT != 0 && blk >= NBLK)) {
                    const int img = (int)(p / hw), q = (int)(p % hw);
                    cc.ih0[j] = (q / g.cwo) * g.csh - g.cph;
                    cc.iw0[j] = (q % g.cwo) * g.csw - g.cpw;
                    cc.cbase[j] = img * g.cc * g.ch * g.cw + cc.ih0[j] * g.cw + cc.iw0[j];
                    cc.any = 1;
                    if (cc.ih0[j] < 0 || cc.ih0[j] + g.ckh > g.ch || cc.iw0[j] < 0 || cc.iw0[j] + g.ckw > g.cw)
                        cc.interior = 0;
                } else {
                    cc.ih0[j] = -(1 << 28);  // never inside the image
                    cc.iw0[j] = -(1 << 28);
                    cc.cbase[j] = 0;
                    cc.interior = 0;
                }
            }
        }
    }

    __device__ static inline void conv_gather(const GemmArgs& g, const ConvCols& cc, int64_t kb,
                                              u4_t* v) {
        if (!cc.any || kb >= g.K) return;
        const gbytes X = (gbytes)g.B;
        const int KHW = g.ckh * g.ckw, HW = g.ch * g.cw;
        // (K = C*KH*KW < 2^31: 32-bit divisions)
        int c = (int)kb / KHW;
        const int rem = (int)kb - c * KHW;
        int kh = rem / g.ckw, kw = rem - (rem / g.ckw) * g.ckw;
#pragma unroll
        for (int e = 0; e < EPV; ++e) {
            if (kb + e < g.K) {
                const int coff = c * HW + kh * g.cw + kw;
                const int bit = e * ES * 8;
#pragma unroll
                for (int j = 0; j < EPV; ++j) {
                    const bool in = cc.interior ||
                                    ((unsigned)(cc.ih0[j] + kh) < (unsigned)g.ch &&
                                     (unsigned)(cc.iw0[j] + kw) < (unsigned)g.cw);
                    if (in) {
                        const int64_t off = (int64_t)cc.cbase[j] + coff;
                        uint32_t x;
                        if constexpr (ES == 4) x = *(const MLK_GLOBAL uint32_t*)(X + off * 4);
                        else if constexpr (ES == 2) x = *(const MLK_GLOBAL uint16_t*)(X + off * 2);
                        else x = X[off];
                        v[j][bit >> 5] |= x << (bit & 31);
                    }
                }
            }
            if (++kw == g.ckw) {
                kw = 0;
                if (++kh == g.ckh) {
                    kh = 0;
                    ++c;
                }
            }
        }
    }

    // Channels-last gather (CONV = 2): chunk i of this thread covers column
    // n = n0 + c / CPR and k-chunk c % CPR; its pixel window origin is fixed
    // for the tile.
    struct NhwcCols {
        int pbase[NB2 > 0 ? NB2 : 1];  // img * H * W
        int ih0[NB2 > 0 ? NB2 : 1], iw0[NB2 > 0 ? NB2 : 1];
    };

    __device__ static inline void nhwc_cols(const GemmArgs& g, int64_t n0, int tid, NhwcCols* nc) {
        const int64_t P = (int64_t)g.cn * g.cho * g.cwo;
        const int hw = g.cho * g.cwo;
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
            const int c = tid + i * NT;
            const int64_t p = n0 + c / CPR;
            if ((BN * CPR) % NT == 0 || c < BN * CPR) {
                if (p < P) {
                    const int img = (int)(p / hw), q = (int)(p % hw);
                    nc->pbase[i] = img * g.ch * g.cw;
                    nc->ih0[i] = (q / g.cwo) * g.csh - g.cph;
                    nc->iw0[i] = (q % g.cwo) * g.csw - g.cpw;
                    continue;
                }
            }
            nc->pbase[i] = 0;
            nc->ih0[i] = -(1 << 28);  // never inside the image
            nc->iw0[i] = -(1 << 28);
        }
    }

    template <class Cols>
    __device__ static inline void nhwc_gather(const GemmArgs& g, int64_t k0, u4_t* rb, int tid,
                                              const Cols* cols) {
        if constexpr (CONV == 2) {
            const NhwcCols& nc = cols[0];
            const gbytes X = (gbytes)g.B;
#pragma unroll
            for (int i = 0; i < NB2; ++i) {
                const int c = tid + i * NT;
                rb[i] = u4_t{0u, 0u, 0u, 0u};
                const int64_t k = k0 + (c % CPR) * EPV;
                if (k >= g.K) continue;
                const int tap = (int)k / g.cc, ch = (int)k - tap * g.cc;  // K < 2^31
                const int kh = tap / g.ckw, kw = tap - (tap / g.ckw) * g.ckw;
                const int ih = nc.ih0[i] + kh, iw = nc.iw0[i] + kw;
                if ((unsigned)ih >= (unsigned)g.ch || (unsigned)iw >= (unsigned)g.cw) continue;
                const int64_t off = ((int64_t)nc.pbase[i] + ih * g.cw + iw) * g.cc + ch;
                rb[i] = *(const MLK_GLOBAL u4_t*)(X + off * ES);
            }
        }
    }

    // ---- registers -> LDS
    __device__ static inline void store_a(uint8_t* sa, const u4_t* ra, int tid) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int c = tid + i * NT;
            if ((BM * CPR) % NT != 0 && c >= BM * CPR) continue;
            const int r = c / CPR, cc = c % CPR;
            *(u4_t*)(sa + r * PITCH + cc * 16) = ra[i];
        }
    }

    __device__ static inline void store_b(uint8_t* sb, const u4_t* rb, int tid) {
        if constexpr (CONV == 2) {
#pragma unroll
            for (int i = 0; i < NB2; ++i) {
                const int c = tid + i * NT;
                if ((BN * CPR) % NT != 0 && c >= BN * CPR) continue;
                *(u4_t*)(sb + (c / CPR) * PITCH + (c % CPR) * 16) = rb[i];
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int blk = tid + i * NT;
            if (NBLK % NT != 0 && blk >= NBLK) continue;
            const int kr = blk / (BN / EPV), nc = blk % (BN / EPV);
            u4_t t[EPV];
            if constexpr (CONV == 0) transpose_block<ES>(rb + i * EPV, t);
            else {
#pragma unroll
                for (int e = 0; e < EPV; ++e) t[e] = rb[i * EPV + e];
            }
#pragma unroll
            for (int j = 0; j < EPV; ++j)
                *(u4_t*)(sb + (nc * EPV + j) * PITCH + kr * 16) = t[j];
        }
    }

    // ---- one tile: C[m0:m0+BM, n0:n0+BN] (+)= A[m0:, kbeg:kend] B[kbeg:kend, n0:]
    __device__ static inline void run(const GemmArgs& g, int tm, int tn, int kz, uint8_t* lds) {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wy = wave / WN, wx = wave % WN;
        const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

        // contraction range of this split
        const int64_t kstages = (g.K + BK - 1) / BK;
        const int64_t per = (kstages + g.split_k - 1) / g.split_k;
        const int64_t s_beg = (int64_t)kz * per;
        const int64_t s_end = min<int64_t>(kstages, s_beg + per);
        const int nk = (int)max<int64_t>(0, s_end - s_beg);

        acc_t acc[TM][TN];
        const int lr = lane & 15, lg = lane >> 4;
        MLK_GLOBAL out_t* C = (MLK_GLOBAL out_t*)g.C;
        // C += A B: start the accumulators from C (read here, next to the first
        // loads, rather than in a read-add-write epilogue).  e4m3 scales the
        // product and int8 must wrap modulo 2^32 exactly, so both keep C apart.
        // (a bf16 C is read in the epilogue instead)
        const bool c_in_acc = DT != DT_F8 && DT != DT_I8 && g.accumulate && !g.atomic && EPI != 2;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            int64_t cbase = 0, rstride = 0;
            const int64_t n = n0 + wx * WTN + j * 16 + lr;
            if constexpr (CONV != 0) {
                const int64_t hw = (int64_t)g.cho * g.cwo;
                const int64_t img = (uint32_t)n / (uint32_t)hw;  // n < N*HO*WO + tile < 2^32
                cbase = img * g.M * hw + (n - img * hw);
                rstride = hw;
            } else {
                cbase = n;
                rstride = g.ldc;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t m = m0 + wy * WTM + i * 16 + lg * 4 + r;
                    acc[i][j][r] = (c_in_acc && m < g.M && n < g.N) ? C[m * rstride + cbase] : 0;
                }
        }

        u4_t ra[NA > 0 ? NA : 1];
        u4_t rb[(NB * EPV > NB2 ? NB * EPV : NB2) > 0 ? (NB * EPV > NB2 ? NB * EPV : NB2) : 1];

        typedef typename std::conditional<CONV == 1, ConvCols,
                typename std::conditional<CONV == 2, NhwcCols, NoCols>::type>::type ColsT;
        ColsT cols[CONV == 1 ? NB : 1];
        if constexpr (CONV == 1) conv_cols(g, n0, tid, cols);
        if constexpr (CONV == 2) nhwc_cols(g, n0, tid, cols);
        if (nk > 0) {
            load_a(g, m0, s_beg * BK, ra, tid);
            load_b(g, n0, s_beg * BK, rb, tid, cols);
            store_a(lds, ra, tid);
            store_b(lds + BM * PITCH, rb, tid);
        }
        __syncthreads();

        for (int it = 0; it < nk; ++it) {
            const bool more = it + 1 < nk;
            if (more) {
                load_a(g, m0, (s_beg + it + 1) * BK, ra, tid);
                load_b(g, n0, (s_beg + it + 1) * BK, rb, tid, cols);
            }
            const uint8_t* sa = lds + (it & 1) * STAGE;
            const uint8_t* sb = sa + BM * PITCH;
#pragma unroll
            for (int ks = 0; ks < KB / KS; ++ks) {
                u4_t af[TM][KV];
                const int off = ks * KS + lg * (KS / 4);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int v = 0; v < KV; ++v)
                        af[i][v] = *(const u4_t*)(sa + (wy * WTM + i * 16 + lr) * PITCH + off + v * 16);
                // B fragments are used as they arrive (one column tile at a
                // time), which keeps few of them live next to the staged loads
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    u4_t bj[KV];
#pragma unroll
                    for (int v = 0; v < KV; ++v)
                        bj[v] = *(const u4_t*)(sb + (wx * WTN + j * 16 + lr) * PITCH + off + v * 16);
#pragma unroll
                    for (int i = 0; i < TM; ++i) Mma<DT>::run(acc[i][j], af[i], bj);
                }
            }
            if (more) {
                uint8_t* na = lds + ((it + 1) & 1) * STAGE;
                store_a(na, ra, tid);
                store_b(na + BM * PITCH, rb, tid);
            }
            __syncthreads();
        }

        // ---- epilogue
        float alpha = 1.0f;
        if constexpr (DT == DT_F8) {
            if (g.scale_a) alpha *= *g.scale_a;
            if (g.scale_b) alpha *= *g.scale_b;
        }
        if constexpr (EPI == 2 && DT != DT_I8 && CONV == 0) {
            // bf16 C (never split): fp32 result, plus the bf16 C when
            // accumulating, rounded once
            MLK_GLOBAL uint16_t* const Cb = (MLK_GLOBAL uint16_t*)g.C;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int64_t n = n0 + wx * WTN + j * 16 + lr;
                if (n >= g.N) continue;
                const float bn = g.bias && kz == 0 ? g.bias[n] : 0.0f;
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t m = m0 + wy * WTM + i * 16 + lg * 4 + r;
                        if (m >= g.M) continue;
                        MLK_GLOBAL uint16_t* q = Cb + m * g.ldc + n;
                        const float v = ((DT == DT_F8) ? alpha * acc[i][j][r] : acc[i][j][r]) + bn;
                        *q = bf16_rne(g.accumulate ? bf16_value(*q) + v : v);
                    }
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t n = n0 + wx * WTN + j * 16 + lr;
            if (n >= g.N) continue;
            float bn = 0.0f;
            if constexpr (EPI && DT != DT_I8 && CONV == 0)
                if (g.bias && kz == 0) bn = g.bias[n];
            int64_t cbase = n;   // offset of column n (row 0)
            int64_t rstride = g.ldc;
            if constexpr (CONV != 0) {
                const int64_t hw = (int64_t)g.cho * g.cwo;
                const int64_t img = (uint32_t)n / (uint32_t)hw, q = n - img * hw;
                cbase = img * g.M * hw + q;
                rstride = hw;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t m = m0 + wy * WTM + i * 16 + lg * 4 + r;
                    if (m >= g.M) continue;
                    MLK_GLOBAL out_t* p = C + m * rstride + cbase;
                    if constexpr (DT == DT_I8) {
                        const uint32_t v = (uint32_t)acc[i][j][r];
                        if (g.atomic) __hip_atomic_fetch_add((MLK_GLOBAL uint32_t*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else *p = (int32_t)(g.accumulate ? (uint32_t)*p + v : v);
                    } else {
                        const float v0 = (DT == DT_F8) ? alpha * acc[i][j][r] : acc[i][j][r];
                        const float v = EPI ? v0 + bn : v0;
                        if (g.atomic) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else if (c_in_acc || !g.accumulate) *p = v;
                        else *p = *p + v;
                    }
                }
        }
    }
};

}  // namespace mlk
