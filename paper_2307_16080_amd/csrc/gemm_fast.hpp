// gemm_fast.hpp -- the bf16 / e4m3 / int8 matmul main loop for large, aligned
// problems on gfx950: operands go from HBM straight into LDS (buffer loads
// with the LDS destination bit, no register staging), B stays in its
// row-major (N-contiguous) layout in LDS and is transposed on the way out by
// the gfx950 LDS transpose reads (ds_read_b64_tr_b16 for bf16,
// ds_read_b64_tr_b8 for e4m3 and int8), and the K loop keeps STAGES-1 stages
// of loads in flight behind the MFMAs.
//
// What is computed is still linalg.matmul, C[M,N] (+)= A[M,K] * B[K,N]
// (paper Sec. 2.1, listing "linalg-matmul"), with fp32 accumulation (int8:
// sign-extended products summed in int32, wrapping modulo 2^32).
//
// Requirements of the direct-to-LDS form (checked on the host): K % BK == 0,
// A, B 16-byte aligned with row pitches that are multiples of 16 bytes, N a
// multiple of the 16-byte chunk (B's rows are read in whole chunks up to the
// last row's padded end), each operand < 2 GiB.  M is arbitrary: rows past the
// end of A read as zero (buffer range check); columns past N only feed outputs
// that are never stored.
//
// STAGES == 1 selects the register-loaded form of the same kernel: every
// thread loads the 16-byte chunks that the DMA would have moved (with the
// same swizzles) into registers, up to three stages ahead (register sets
// permitting), and writes them to one of two LDS buffers.  It takes any shape and alignment (rows aligned only to
// the element size, K not a multiple of BK) and is the tile that the
// persistent batched launch runs.
//
// LDS layout per stage: A as BM rows of 128 bytes (BK = 64 bf16, or 128
// e4m3 or int8), the 16-byte chunk c of row r stored at chunk c ^ fa(r); B as BK rows
// of BN elements, the 16-byte chunk c of row k stored at chunk c ^ fb(k).  The
// XOR patterns spread the lanes of one LDS read over distinct banks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_tile.hpp"


namespace mlk {

typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef int i2_t __attribute__((ext_vector_type(2)));
typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));
typedef float f16v_t __attribute__((ext_vector_type(16)));

// 16-byte buffer load per lane whose data goes to LDS at m0 + 16 * lane.
// Written as inline asm so that the compiler does not treat it as a pending
// write to every LDS location (it would otherwise wait for the whole prefetch
// before the next LDS read); the kernel waits on vmcnt itself.  One wait
// state separates the m0 write from the load.  m0 is listed as clobbered
// (the compiler warns that it is a reserved register); in these kernels
// nothing else keeps a value in m0 (the generated code writes m0 only here).
__device__ inline void dma_load16(uint32_t lds_addr, int voffset, const i32x4_t& rsrc, int soffset) {
    asm volatile(
        "s_mov_b32 m0, %0\n\t"
        "s_nop 0\n\t"
        "buffer_load_dwordx4 %1, %2, %3 offen lds"
        :
        : "s"(lds_addr), "v"(voffset), "s"(rsrc), "s"(soffset)
        : "memory", "m0");
}

__device__ inline i32x4_t make_rsrc(const void* base, uint32_t bytes) {
    const uint64_t b = (uint64_t)base;
    i32x4_t r;
    r[0] = (int32_t)(uint32_t)(b & 0xFFFFFFFFu);
    r[1] = (int32_t)(uint32_t)(b >> 32);  // stride 0
    r[2] = (int32_t)bytes;                // range: larger offsets read zero
    r[3] = 0x00020000;                    // raw buffer, 32-bit data format
    return r;
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding)
template <int N>
__device__ inline void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

// A swizzle: chosen by measurement among XOR patterns (a ds_read_b128 sweep
// in which 16 lanes read 16 consecutive 128-byte rows at one logical chunk:
// this one streams 181 B/clk/CU, the plain layout 59).
__device__ inline int fa(int r) { return (r & 7) ^ ((r >> 2) & 2); }

// CONV = 2: the channels-last implicit-GEMM convolution (bf16): A is the
// filter as F x (KH*KW*C), C contiguous; B is never formed: its transpose --
// one row per output pixel n = (img, oh, ow), columns k = (kh, kw, c) -- is
// gathered from the NHWC input in 16-byte chunks of 8 channels (C a multiple
// of 8), through registers (STAGES = 1) or as direct-to-LDS copies (STAGES >=
// 2, C*KH*KW a multiple of BK), and kept in LDS like A (rows of BK k), so the
// MFMA's B operand is read as A's is.  The output is NFHW.
// CONV = 3: the same tile fed from the NCHW input itself (no channels-last
// copy): each 16-byte chunk -- 8 channels of one input pixel -- is assembled
// in registers from 8 two-byte loads H*W elements apart (STAGES = 1 only).
// Output stage: EPI = 0 the plain product; 1 adds the Linear layer's bias to
// an fp32 C; 2 writes a bf16 C (bias optional).  Each is its own instantiation,
// so no kernel carries a branch between them.
// MF: the MFMA tile, 16 (16x16 outputs per instruction; every dtype) or 32
// (bf16 v_mfma_f32_32x32x16_bf16: twice the flops per instruction, so half
// the MFMA and LDS read instructions -- the LDS bytes per k a wave reads are
// set by its tile, not the MFMA shape -- and 16 accumulators per lane per
// tile; GEMM policy, fp32 or bias output stages).
template <int DT, int BM, int BN, int WM, int WN, int STAGES, int CONV = 0, int EPI = 0, int MF = 16>
struct FastGemm {
    static_assert(DT == DT_BF16 || DT == DT_F8 || DT == DT_I8, "direct-layout kernel: bf16, e4m3 or int8");
    static_assert(CONV == 0 || ((CONV == 2 || CONV == 3) && DT == DT_BF16), "implicit convolution: bf16");
    static_assert(CONV != 3 || STAGES == 1, "the NCHW channel gather is register-loaded");
    static_assert(DT != DT_I8 || EPI == 0, "int8: plain int32 output stage only");
    static_assert(MF == 16 || (MF == 32 && DT == DT_BF16 && CONV == 0 && EPI != 2),
                  "32x32 MFMA tiles: bf16 GEMM policy, fp32 or bias output");
    static constexpr int KB = 128;                 // bytes of K per A row per stage
    static constexpr int ES = DT == DT_BF16 ? 2 : 1;
    static constexpr int BK = KB / ES;             // elements per A row per stage
    // k per MFMA: 16x16x32 bf16, 16x16x128 f8f6f4, 16x16x64 i8
    static constexpr int KSTEP = DT == DT_BF16 ? (MF == 32 ? 16 : 32) : DT == DT_F8 ? 128 : 64;
    // accumulator registers per lane per MFMA tile
    static constexpr int NR = MF == 32 ? 16 : 4;
    // int8: int32 accumulators and output (sums wrap modulo 2^32)
    typedef typename std::conditional<DT == DT_I8, i4_t,
                                      typename std::conditional<MF == 32, f16v_t, f4_t>::type>::type acc_t;
    typedef typename std::conditional<DT == DT_I8, int32_t, float>::type out_t;
    static constexpr int NW = WM * WN;
    static constexpr int NT = 64 * NW;
    static constexpr int A_ROW = KB;               // bytes
    static constexpr int A_CPR = KB / 16;          // 16-byte chunks per A row
    static constexpr int B_ROW = CONV ? KB : BN * ES;  // B^T rows of BK k for conv
    static constexpr int A_STAGE = BM * A_ROW;
    static constexpr int B_STAGE = CONV ? BN * B_ROW : BK * B_ROW;
    static constexpr int STAGE = A_STAGE + B_STAGE;
    static constexpr bool REG = STAGES == 1;      // register-loaded form
    static constexpr int NBUF = REG ? 2 : STAGES;  // LDS stage buffers
    static constexpr int EPV = 16 / ES;            // elements per 16-byte chunk
    static constexpr int LDS_BYTES = NBUF * STAGE;
    static constexpr int A_SLABS = A_STAGE / 1024;  // one wave-wide 16-byte load fills a slab
    static constexpr int B_SLABS = B_STAGE / 1024;
    static constexpr int NA = A_SLABS / NW;         // per wave per stage
    static constexpr int NB = B_SLABS / NW;
    static constexpr int LOADS = NA + NB;
    static constexpr int WTM = BM / WM, WTN = BN / WN;
    static constexpr int TM = WTM / MF, TN = WTN / MF;
    static constexpr int A_ROWS_PER_SLAB = 1024 / A_ROW;
    static constexpr int B_ROWS_PER_SLAB = 1024 / B_ROW;
    static constexpr int B_CHUNKS = B_ROW / 16;
    // register-loaded form: stages loaded ahead into PF register sets (2..4,
    // as many as fit beside the accumulators in ~192 VGPRs), so that PF - 1
    // stages of loads are in flight while one is multiplied
    static constexpr int SET_REGS = (NA + NB) * 4;
    static constexpr int ACC_REGS = TM * TN * NR;
    static constexpr int PF_FIT = (192 - ACC_REGS) / SET_REGS;
    static constexpr int PF = PF_FIT < 2 ? 2 : PF_FIT > 4 ? 4 : PF_FIT;

    static_assert(A_SLABS % NW == 0 && B_SLABS % NW == 0, "slabs must divide among waves");
    static_assert(CONV || B_CHUNKS >= (DT == DT_BF16 ? 16 : DT == DT_F8 ? 8 : 4), "B rows too short for the swizzle");

    // B swizzle: the rows read together by one transpose read land in distinct
    // 16-byte bank groups.  bf16 reads 4 rows x 32 bytes per lane group, e4m3
    // 8 rows x 16 bytes.  int8 reads 8 rows x 16 bytes per lane group, the
    // groups 16 rows apart, so the 16 rows a half-wave reads are k = 0..7 and
    // 16..23 (plus a multiple of 8): with 64 banks of 4 bytes a row pitch of 256
    // bytes maps every row to the same banks (chunks 0..15 must differ), 128
    // bytes alternates two halves by k & 1, 64 bytes four quarters by k & 3.
    __device__ static inline int fb(int k) {
        // 32x32 tiles: a half-wave's transpose read covers 4 rows x 4 chunks
        if constexpr (DT == DT_BF16 && MF == 32) return (k & 3) << 2;
        else if constexpr (DT == DT_BF16) return ((k & 3) << 1) | (((k >> 3) & 1) << 3);
        else if constexpr (DT == DT_F8) return (k & 7) | (B_CHUNKS >= 16 ? (((k >> 5) & 1) << 3) : 0);
        else if constexpr (B_CHUNKS >= 16) return (k & 7) | (((k >> 4) & 1) << 3);
        else if constexpr (B_CHUNKS == 8) return ((k >> 1) & 3) | (((k >> 4) & 1) << 2);
        else return ((k >> 2) & 1) | (((k >> 4) & 1) << 1);
    }
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(WTM % MF == 0 && WTN % MF == 0, "wave tile");
    static_assert(STAGES >= 1 && (STAGES - 1) * LOADS < 64, "pipeline depth");

    // wait until stage `it` has landed: at most `later` stages (issued after
    // it) may still be in flight, LOADS buffer loads each per lane
    template <int L>
    __device__ static inline void wait_stage(int later) {
        if constexpr (L == 0) {
            wait_vmcnt<0>();
        } else {
            if (later >= L) wait_vmcnt<L * LOADS>();
            else wait_stage<L - 1>(later);
        }
    }

    __device__ static inline void issue_stage(const i32x4_t& ra, const i32x4_t& rb,
                                              const int* voff_a, const int* voff_b, int64_t k0,
                                              int64_t ldb, uint8_t* stage, int wave) {
        const int sa = __builtin_amdgcn_readfirstlane((int)(k0 * ES));
        const int sb = __builtin_amdgcn_readfirstlane((int)(k0 * ldb * ES));
        const uint32_t base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)stage;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int slab = wave + i * NW;
            dma_load16(__builtin_amdgcn_readfirstlane(base + slab * 1024), voff_a[i], ra, sa);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int slab = wave + i * NW;
            dma_load16(__builtin_amdgcn_readfirstlane(base + A_STAGE + slab * 1024), voff_b[i], rb, sb);
        }
    }

    // conv, direct-to-LDS form: A as issue_stage; each B^T slab is gathered
    // from the NHWC input, one 16-byte chunk per lane (8 channels of one pixel
    // and filter tap) landing where the register-loaded form would store it;
    // chunks outside the image or past the last pixel read zero (offset past
    // the buffer's range).  Stages are issued in order and every call steps the
    // chunks' k by BK (C * KH * KW is a multiple of BK for this form).
    template <typename Slots>
    __device__ static inline void issue_stage_conv(const GemmArgs& g, const i32x4_t& ra, const i32x4_t& rb,
                                                   const int* voff_a, Slots& rs, int64_t k0, uint8_t* stage,
                                                   int wave) {
        const int sa = __builtin_amdgcn_readfirstlane((int)(k0 * ES));
        const uint32_t base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)stage;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int slab = wave + i * NW;
            dma_load16(__builtin_amdgcn_readfirstlane(base + slab * 1024), voff_a[i], ra, sa);
        }
        if (rs.tap_uniform) {
            const int dk = (rs.t_kh * g.cw + rs.t_kw) * g.cc + rs.t_c0;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int slab = wave + i * NW;
                const bool in = rs.p_ok[i] && (unsigned)(rs.p_ih0[i] + rs.t_kh) < (unsigned)g.ch &&
                                (unsigned)(rs.p_iw0[i] + rs.t_kw) < (unsigned)g.cw;
                const int off = in ? (rs.p_base[i] + dk) * ES : 0x7FFFFFF0;
                dma_load16(__builtin_amdgcn_readfirstlane(base + A_STAGE + slab * 1024), off, rb, 0);
            }
            tap_step(g, rs);
            return;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int slab = wave + i * NW;
            int off = 0x7FFFFFF0;
            if (rs.p_ok[i]) {
                const int ih = rs.p_ih0[i] + rs.k_kh[i], iw = rs.p_iw0[i] + rs.k_kw[i];
                if ((unsigned)ih < (unsigned)g.ch && (unsigned)iw < (unsigned)g.cw)
                    off = (int)(((rs.p_img[i] + (int64_t)ih * g.cw + iw) * g.cc + rs.k_ci[i]) * ES);
            }
            dma_load16(__builtin_amdgcn_readfirstlane(base + A_STAGE + slab * 1024), off, rb, 0);
            rs.k_ci[i] += BK;
            while (rs.k_ci[i] >= g.cc) {
                rs.k_ci[i] -= g.cc;
                if (++rs.k_kw[i] == g.ckw) {
                    rs.k_kw[i] = 0;
                    ++rs.k_kh[i];
                }
            }
        }
    }

    // ---- register-loaded form: per-thread chunk state, fixed for a tile
    struct RegSlots {
        int64_t a_off[NA];   // byte offset of the chunk's row (clamped to row 0 when invalid)
        int a_el[NA];        // element offset of the chunk inside its row (swizzled source chunk)
        bool a_ok[NA];       // row < M
        int64_t b_off[NB];   // byte offset of (row r of the stage, first column of the chunk)
        int b_r[NB];         // row of the stage
        int b_col[NB];       // first column of the chunk
        int b_nv[NB];        // valid columns in the chunk (0..EPV)
        // conv: the pixel of B^T row r (base of its image in NHWC, window origin),
        // and the chunk's current k = (kh, kw, ci), stepped by BK per stage
        int64_t p_img[NB];
        int p_ih0[NB], p_iw0[NB];
        int p_ok[NB];
        int k_ci[NB], k_kh[NB], k_kw[NB];
        // C a multiple of BK (every stage inside one filter tap, the same for all
        // lanes): the tap (kh, kw) and first channel c0 of the next stage to
        // load, stepped once per stage as wave-uniform values, and per chunk the
        // element offset of its first channel at tap (0, 0) (NHWC: pixel * C +
        // channel; NCHW: image base + window origin + channel * H * W)
        bool tap_uniform;
        int t_c0, t_kh, t_kw;
        int p_base[NB];
    };

    // step the uniform tap state past one stage (C a multiple of BK)
    __device__ static inline void tap_step(const GemmArgs& g, RegSlots& rs) {
        rs.t_c0 += BK;
        if (rs.t_c0 >= g.cc) {
            rs.t_c0 = 0;
            if (++rs.t_kw == g.ckw) {
                rs.t_kw = 0;
                ++rs.t_kh;
            }
        }
    }

    __device__ static inline void reg_slots(const GemmArgs& g, int64_t m0, int64_t n0, int64_t kfirst,
                                            int wave, int lane, RegSlots& rs) {
        if constexpr (CONV) {
            rs.tap_uniform = g.cc % BK == 0;
            const int k = __builtin_amdgcn_readfirstlane((int)kfirst);
            const int tap = k / g.cc;
            rs.t_c0 = k - tap * g.cc;
            rs.t_kh = tap / g.ckw;
            rs.t_kw = tap - rs.t_kh * g.ckw;
        }
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int slab = wave + i * NW;
            const int r = slab * A_ROWS_PER_SLAB + lane / A_CPR;
            const int c = (lane % A_CPR) ^ fa(r);
            const int64_t row = m0 + r;
            rs.a_ok[i] = row < g.M;
            rs.a_off[i] = (rs.a_ok[i] ? row : 0) * g.lda * ES;
            rs.a_el[i] = c * EPV;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int slab = wave + i * NW;
            if constexpr (CONV) {
                // B^T row r = output pixel n0 + r, chunk c of its k range.  The
                // NCHW gather (CONV 3) gives a wave 64 consecutive rows of one
                // chunk, so each of its two-byte loads reads 64 neighbouring
                // pixels of one channel plane; reg_store puts the chunk where
                // this layout's slab would have it.
                const int slot = i * NT + wave * 64 + lane;
                const int r = CONV == 3 ? slot % BN : slab * A_ROWS_PER_SLAB + lane / A_CPR;
                const int c = CONV == 3 ? slot / BN : (lane % A_CPR) ^ fa(r);
                const int64_t p = n0 + r;
                const int hw = g.cho * g.cwo;
                rs.b_r[i] = r;
                rs.b_col[i] = c * EPV;  // element offset of the chunk in the stage's k range
                rs.p_ok[i] = p < g.N;
                // pixel and depth indices fit 32 bits (N*HO*WO and C*KH*KW are
                // below 2^31): 32-bit divisions
                const int img = rs.p_ok[i] ? (int)((uint32_t)p / (uint32_t)hw) : 0;
                const int q = rs.p_ok[i] ? (int)p - img * hw : 0;
                // image base in elements: NHWC (CONV 2) counts pixels, scaled by C
                // at the load; NCHW (CONV 3) is the image's first element
                rs.p_img[i] = CONV == 3 ? (int64_t)img * g.cc * g.ch * g.cw : (int64_t)img * g.ch * g.cw;
                rs.p_ih0[i] = (q / g.cwo) * g.csh - g.cph;
                rs.p_iw0[i] = (q % g.cwo) * g.csw - g.cpw;
                const int k = (int)kfirst + rs.b_col[i];
                const int tap = (int)((uint32_t)k / (uint32_t)g.cc);
                rs.k_ci[i] = k - tap * g.cc;
                rs.k_kh[i] = tap / g.ckw;
                rs.k_kw[i] = tap - rs.k_kh[i] * g.ckw;
                // (operands below 2 GiB: element offsets fit 32 bits; a window
                // origin above or left of the image makes the base negative,
                // and it is used only for taps inside the image)
                rs.p_base[i] = CONV == 3 ? (int)rs.p_img[i] + rs.p_ih0[i] * g.cw + rs.p_iw0[i] + rs.b_col[i] * g.ch * g.cw
                                         : ((int)rs.p_img[i] + rs.p_ih0[i] * g.cw + rs.p_iw0[i]) * g.cc + rs.b_col[i];
            } else {
                const int r = slab * B_ROWS_PER_SLAB + lane / B_CHUNKS;
                const int c = (lane % B_CHUNKS) ^ fb(r);
                const int64_t col = n0 + c * EPV;
                rs.b_r[i] = r;
                rs.b_col[i] = (int)min<int64_t>(col, g.N);
                rs.b_nv[i] = (int)max<int64_t>(0, min<int64_t>(EPV, g.N - col));
                rs.b_off[i] = (int64_t)r * g.ldb * ES + (int64_t)rs.b_col[i] * ES;
            }
        }
    }

    // the chunks of the stage starting at k0 (zero outside the operands)
    __device__ static inline void reg_load(const GemmArgs& g, RegSlots& rs, int64_t k0,
                                           u4_t* ra, u4_t* rb) {
        const gbytes A = (gbytes)g.A, B = (gbytes)g.B;
        const bool kfull = k0 + BK <= g.K;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int64_t k = k0 + rs.a_el[i];
            const gbytes row = A + rs.a_off[i];
            u4_t v = u4_t{0u, 0u, 0u, 0u};
            if (rs.a_ok[i]) {
                if (kfull) v = g.vec_a ? *(const MLK_GLOBAL u4_t*)(row + k * ES) : load16_any<ES>(row + k * ES);
                else if (k < g.K) v = load_unaligned<ES>(row, k, (int)min<int64_t>(EPV, g.K - k));
            }
            ra[i] = v;
        }
        if constexpr (CONV) {
            if (rs.tap_uniform) {
                // the whole stage lies in tap (t_kh, t_kw), channels t_c0 ..
                const int dk = CONV == 3 ? rs.t_c0 * g.ch * g.cw + rs.t_kh * g.cw + rs.t_kw
                                         : (rs.t_kh * g.cw + rs.t_kw) * g.cc + rs.t_c0;
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    u4_t v = u4_t{0u, 0u, 0u, 0u};
                    if (rs.p_ok[i] && (unsigned)(rs.p_ih0[i] + rs.t_kh) < (unsigned)g.ch &&
                        (unsigned)(rs.p_iw0[i] + rs.t_kw) < (unsigned)g.cw) {
                        if constexpr (CONV == 3) {
                            const int plane = g.ch * g.cw;
                            const MLK_GLOBAL uint16_t* src = (const MLK_GLOBAL uint16_t*)B + (rs.p_base[i] + dk);
                            uint32_t h[8];
#pragma unroll
                            for (int e = 0; e < 8; ++e) h[e] = src[e * plane];
                            v = u4_t{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                     h[6] | (h[7] << 16)};
                        } else {
                            v = *(const MLK_GLOBAL u4_t*)(B + (int64_t)(rs.p_base[i] + dk) * ES);
                        }
                    }
                    rb[i] = v;
                }
                tap_step(g, rs);
                return;
            }
            // chunk k..k+7 lies in one filter tap (C is a multiple of 8): channels
            // ci..ci+7 of input pixel (ih, iw), zero outside the image
            // (stages are loaded in order, so each call steps every chunk by BK)
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                u4_t v = u4_t{0u, 0u, 0u, 0u};
                const int64_t k = k0 + rs.b_col[i];
                if (rs.p_ok[i] && k < g.K) {
                    const int ih = rs.p_ih0[i] + rs.k_kh[i], iw = rs.p_iw0[i] + rs.k_kw[i];
                    if ((unsigned)ih < (unsigned)g.ch && (unsigned)iw < (unsigned)g.cw) {
                        if constexpr (CONV == 3) {
                            // channels ci..ci+7 of pixel (ih, iw): one plane (H*W elements) apart
                            const int64_t plane = (int64_t)g.ch * g.cw;
                            const MLK_GLOBAL uint16_t* src = (const MLK_GLOBAL uint16_t*)B + rs.p_img[i] +
                                                             (int64_t)rs.k_ci[i] * plane + (int64_t)ih * g.cw + iw;
                            uint32_t h[8];
#pragma unroll
                            for (int e = 0; e < 8; ++e) h[e] = src[e * plane];
                            v = u4_t{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                     h[6] | (h[7] << 16)};
                        } else {
                            v = *(const MLK_GLOBAL u4_t*)(B + ((rs.p_img[i] + (int64_t)ih * g.cw + iw) * g.cc +
                                                               rs.k_ci[i]) * ES);
                        }
                    }
                }
                rb[i] = v;
                rs.k_ci[i] += BK;
                while (rs.k_ci[i] >= g.cc) {
                    rs.k_ci[i] -= g.cc;
                    if (++rs.k_kw[i] == g.ckw) {
                        rs.k_kw[i] = 0;
                        ++rs.k_kh[i];
                    }
                }
            }
            return;
        }
        const int64_t kb = k0 * g.ldb * ES;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            u4_t v = u4_t{0u, 0u, 0u, 0u};
            if (rs.b_nv[i] > 0 && (kfull || k0 + rs.b_r[i] < g.K)) {
                const gbytes p = B + kb + rs.b_off[i];
                if (rs.b_nv[i] == EPV) v = g.vec_b ? *(const MLK_GLOBAL u4_t*)p : load16_any<ES>(p);
                else v = load_unaligned<ES>(p - (int64_t)rs.b_col[i] * ES, rs.b_col[i], rs.b_nv[i]);
            }
            rb[i] = v;
        }
    }

    // registers -> the LDS positions the DMA would have filled
    __device__ static inline void reg_store(uint8_t* stage, const u4_t* ra, const u4_t* rb, int wave,
                                            int lane, const RegSlots& rs) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
            *(u4_t*)(stage + (wave + i * NW) * 1024 + lane * 16) = ra[i];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if constexpr (CONV == 3) {
                // row-major lane layout: logical chunk c of row r sits at c ^ fa(r)
                const int r = rs.b_r[i], c = rs.b_col[i] / EPV;
                *(u4_t*)(stage + A_STAGE + r * B_ROW + ((c ^ fa(r)) * 16)) = rb[i];
            } else {
                *(u4_t*)(stage + A_STAGE + (wave + i * NW) * 1024 + lane * 16) = rb[i];
            }
        }
    }

    // the MFMAs of one LDS stage (sa: A rows, sb: B rows or, for conv, B^T rows)
    // `mid` issues the next stage's copies.  bf16 stages hold two k-steps and
    // issue them between the two (measured ~10% faster at 4096^3 than issuing
    // before the first); e4m3 stages hold one k-step and issue before it (an
    // issue after any of its MFMAs measured ~20% slower).
    template <typename Mid>
    __device__ static inline void mma_stage(const uint8_t* sa, const uint8_t* sb, acc_t (&acc)[TM][TN], int wy,
                                            int wx, int lr, int lg, Mid&& mid) {
        constexpr int KSTEPS = BK / KSTEP;
        constexpr int MID_AT = (DT != DT_F8 && KSTEPS >= 2) ? KSTEPS / 2 : 0;
        typedef __attribute__((address_space(3))) bf4_t* tp;
        typedef __attribute__((address_space(3))) i2_t* t8p;
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            if (ks == MID_AT) mid();
            if constexpr (DT == DT_BF16 && MF == 32) {
                // 32x32x16: lane l supplies row (or column) l % 32 and k
                // 8 * (l / 32) .. +7 of the 16-deep step: A as one 16-byte read,
                // B as two transpose reads of 4 rows x 16 columns per 16-lane group
                const int l32 = lg * 16 + lr, half = lg >> 1;
                u4_t af[TM];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int r = wy * WTM + i * 32 + (l32 & 31);
                    af[i] = *(const u4_t*)(sa + r * A_ROW + (((ks * 2 + half) ^ fa(r)) * 16));
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int nb = wx * WTN + j * 32 + (lg & 1) * 16 + 4 * (lr & 3);
                    bf4_t h[2];
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        const int k = ks * 16 + half * 8 + hh * 4 + (lr >> 2);
                        const int c = (nb >> 3) ^ fb(k);
                        h[hh] = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((tp)(sb + k * B_ROW + c * 16 + (nb & 7) * 2));
                    }
                    const bf8_t bj = bf8_t{h[0][0], h[0][1], h[0][2], h[0][3], h[1][0], h[1][1], h[1][2], h[1][3]};
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8_t, af[i]), bj,
                                                                            acc[i][j], 0, 0, 0);
                }
            } else if constexpr (DT == DT_BF16) {
                u4_t af[TM];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int r = wy * WTM + i * 16 + lr;
                    const int c = (ks * 4 + lg) ^ fa(r);
                    af[i] = *(const u4_t*)(sa + r * A_ROW + c * 16);
                }
                // B fragments are consumed as soon as they arrive, column tile by
                // column tile, so only one or two are live at a time
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    // lane lr of the group supplies row lr/4, columns 4*(lr%4)..+3 of a
                    // 4 x 16 block; the transpose read returns column lr to it
                    bf8_t bj;
                    if constexpr (CONV) {
                        // B^T rows hold k contiguous: read like A
                        const int r = wx * WTN + j * 16 + lr;
                        bj = __builtin_bit_cast(bf8_t, *(const u4_t*)(sb + r * B_ROW + (((ks * 4 + lg) ^ fa(r)) * 16)));
                    } else {
                        const int nb = wx * WTN + j * 16 + 4 * (lr & 3);
                        bf4_t h[2];
#pragma unroll
                        for (int half = 0; half < 2; ++half) {
                            const int k = ks * 32 + lg * 8 + half * 4 + (lr >> 2);
                            const int c = (nb >> 3) ^ fb(k);
                            const uint8_t* p = sb + k * B_ROW + c * 16 + (nb & 7) * 2;
                            h[half] = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((tp)(p));
                        }
                        bj = bf8_t{h[0][0], h[0][1], h[0][2], h[0][3], h[1][0], h[1][1], h[1][2], h[1][3]};
                    }
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf8_t, af[i]), bj, acc[i][j], 0, 0, 0);
                }
            } else if constexpr (DT == DT_I8) {
                // lane (lr, lg) supplies row / column lr and k bytes
                // ks*64 + lg*16 .. +15 of the stage, as the 16x16x64 i8 MFMA takes them
                u4_t af[TM];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int r = wy * WTM + i * 16 + lr;
                    af[i] = *(const u4_t*)(sa + r * A_ROW + (((ks * 4 + lg) ^ fa(r)) * 16));
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    // two transpose reads: lane lr supplies row lr/2, bytes
                    // 8*(lr%2)..+7 of an 8 x 16 block and gets column lr (8 k) back
                    const int nb = wx * WTN + j * 16 + 8 * (lr & 1);
                    i2_t q[2];
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq) {
                        const int k = ks * 64 + lg * 16 + qq * 8 + (lr >> 1);
                        const int c = (nb >> 4) ^ fb(k);
                        const uint8_t* p = sb + k * B_ROW + c * 16 + (nb & 15);
                        q[qq] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((t8p)(p));
                    }
                    const i4_t bj = i4_t{q[0][0], q[0][1], q[1][0], q[1][1]};
#pragma unroll
                    for (int i = 0; i < TM; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i4_t, af[i]), bj,
                                                                           acc[i][j], 0, 0, 0);
                }
            } else {
                i8_t af[TM], bfr[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int r = wy * WTM + i * 16 + lr;
                    const u4_t lo = *(const u4_t*)(sa + r * A_ROW + ((2 * lg) ^ fa(r)) * 16);
                    const u4_t hi = *(const u4_t*)(sa + r * A_ROW + ((2 * lg + 1) ^ fa(r)) * 16);
                    af[i] = i8_t{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                                 (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    // lane lr supplies row lr/2, bytes 8*(lr%2)..+7 of an 8 x 16 block;
                    // the transpose read returns column lr (8 consecutive k) to it
                    const int nb = wx * WTN + j * 16 + 8 * (lr & 1);
                    i2_t q[4];
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const int k = lg * 32 + qq * 8 + (lr >> 1);
                        const int c = (nb >> 4) ^ fb(k);
                        const uint8_t* p = sb + k * B_ROW + c * 16 + (nb & 15);
                        q[qq] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((t8p)(p));
                    }
                    bfr[j] = i8_t{q[0][0], q[0][1], q[1][0], q[1][1], q[2][0], q[2][1], q[3][0], q[3][1]};
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                            af[i], bfr[j], acc[i][j], 0, 0, 0, 127, 0, 127);
            }
        }
    }

    __device__ static inline void run(const GemmArgs& g, int tm, int tn, int kz, uint8_t* lds) {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wy = wave / WN, wx = wave % WN;
        const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
        const int64_t kstages = REG ? (g.K + BK - 1) / BK : g.K / BK;
        const int64_t per = (kstages + g.split_k - 1) / g.split_k;
        const int64_t s_beg = (int64_t)kz * per;
        const int nk = (int)max<int64_t>(0, min<int64_t>(kstages, s_beg + per) - s_beg);

        // direct-to-LDS form: buffer resources and per-lane byte offsets of this
        // wave's load slabs (k0 added as the scalar offset)
        i32x4_t ra = {0, 0, 0, 0}, rb = {0, 0, 0, 0};
        int voff_a[NA], voff_b[NB];
        // register-loaded form: chunk state and the stage in flight
        RegSlots rs;
        u4_t qa[REG ? PF : 1][NA], qb[REG ? PF : 1][NB];
        if constexpr (!REG) {
            ra = make_rsrc(g.A, (uint32_t)(((g.M - 1) * g.lda + g.K) * ES));
            if constexpr (CONV) {
                rb = make_rsrc(g.B, (uint32_t)((int64_t)g.cn * g.ch * g.cw * g.cc * ES));
                reg_slots(g, m0, n0, s_beg * BK, wave, lane, rs);
            } else {
                // B rows are read in whole 16-byte chunks, so the range ends at the
                // last row's chunk-padded end: the host packs B whenever N is not a
                // multiple of the chunk (a 16-byte load that crosses the range end
                // would read back as zero, dropping the last row's products)
                const int64_t np = (g.N + EPV - 1) / EPV * EPV;
                rb = make_rsrc(g.B, (uint32_t)(((g.K - 1) * g.ldb + np) * ES));
            }
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int slab = wave + i * NW;
                const int r = slab * A_ROWS_PER_SLAB + lane / A_CPR;
                const int c = (lane % A_CPR) ^ fa(r);
                int64_t row = m0 + r;
                // rows past the operand read zero: push their offset past the range
                voff_a[i] = row < g.M ? (int)(row * g.lda * ES + c * 16) : 0x7FFFFFF0;
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                if constexpr (CONV) {
                    voff_b[i] = 0;
                } else {
                    const int slab = wave + i * NW;
                    const int r = slab * B_ROWS_PER_SLAB + lane / B_CHUNKS;
                    const int c = (lane % B_CHUNKS) ^ fb(r);
                    const int64_t col = n0 + c * (16 / ES);
                    voff_b[i] = col < g.N ? (int)((r * g.ldb + col) * ES) : 0x7FFFFFF0;
                }
            }
        } else {
            reg_slots(g, m0, n0, s_beg * BK, wave, lane, rs);
        }

        acc_t acc[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (MF == 32) acc[i][j] = acc_t{};
                else acc[i][j] = acc_t{0, 0, 0, 0};
            }

        // prologue: STAGES-1 stages in flight (direct), or stage 0 in LDS (registers)
        if constexpr (!REG) {
#pragma unroll
            for (int s = 0; s < STAGES - 1; ++s) {
                if (s >= nk) continue;
                if constexpr (CONV) issue_stage_conv(g, ra, rb, voff_a, rs, (s_beg + s) * BK, lds + s * STAGE, wave);
                else issue_stage(ra, rb, voff_a, voff_b, (s_beg + s) * BK, g.ldb, lds + s * STAGE, wave);
            }
        } else {
            // stages 0 .. PF-1 requested here; stage 0 is waited for and stored
            // after C's read below has been issued too
#pragma unroll
            for (int s = 0; s < PF; ++s)
                if (s < nk) reg_load(g, rs, (s_beg + s) * BK, qa[s], qb[s]);
        }

        const int lr = lane & 15, lg = lane >> 4;
        // This lane's outputs: rows wy*WTM + i*16 + lg*4 + r, columns
        // wx*WTN + j*16 + lr of the tile whose corner is Ct (a uniform base);
        // with 32x32 MFMA tiles rows wy*WTM + i*32 + 8*(r/4) + 4*(lane/32) + r%4,
        // columns wx*WTN + j*32 + lane%32;
        // offsets inside the tile are 32-bit.
        MLK_GLOBAL out_t* const Ct = (MLK_GLOBAL out_t*)g.C + (CONV ? 0 : m0 * g.ldc + n0);
        // bf16 output (GEMM policy only): the same tile of C as 16-bit codes
        MLK_GLOBAL uint16_t* const Cb = (MLK_GLOBAL uint16_t*)g.C + (CONV ? 0 : m0 * g.ldc + n0);
        const int ldc = (int)g.ldc;
        const int row0 = wy * WTM + (MF == 32 ? 4 * (lane >> 5) : lg * 4);
        const int col0 = wx * WTN + (MF == 32 ? (lane & 31) : lr);
        auto rowof = [&](int i, int r) { return MF == 32 ? row0 + i * 32 + 8 * (r >> 2) + (r & 3) : row0 + i * 16 + r; };
        const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
        const int mrem = (int)min<int64_t>(BM, g.M - m0), nrem = (int)min<int64_t>(BN, g.N - n0);
        // conv: output (f, n) of NFHW lives at img(n)*F*HW + f*HW + pix(n); this
        // lane's column tiles j start at cbase[j] (row f = 0), rows step by HW
        int64_t cbase[CONV ? TN : 1];
        const int64_t hw = CONV ? (int64_t)g.cho * g.cwo : 0;
        if constexpr (CONV) {
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int64_t n = n0 + col0 + j * MF;
                const int64_t img = (uint32_t)n / (uint32_t)hw;  // n < N*HO*WO < 2^31
                cbase[j] = img * g.M * hw + (n - img * hw) + m0 * hw;
            }
        }
        // C += A B: start the accumulators from C itself, so that its read
        // happens here, beside the first stage's loads, instead of in a
        // read-add-write epilogue after the last MFMA.  e4m3 multiplies the
        // sum by alpha = scale_a * scale_b at the end, so it starts from
        // C / alpha (one extra rounding of C); when alpha is far from 1, or a
        // wave finds a C / alpha that overflows, that wave keeps C apart.
        float alpha = 1.0f, inv_alpha = 1.0f;
        bool c_in_acc = g.accumulate && !g.atomic && EPI != 2;  // a bf16 C is read in the epilogue
        if constexpr (DT == DT_F8) {
            if (g.scale_a) alpha *= *(const MLK_GLOBAL float*)g.scale_a;
            if (g.scale_b) alpha *= *(const MLK_GLOBAL float*)g.scale_b;
            const float aa = fabsf(alpha);
            c_in_acc = c_in_acc && aa >= 0x1p-60f && aa <= 0x1p60f;
            inv_alpha = 1.0f / alpha;
        }
        if (c_in_acc) {
            bool over = false;
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const int row = rowof(i, r), col = col0 + j * MF;
                        const bool in = full || (row < mrem && col < nrem);
                        out_t x = 0;
                        if constexpr (CONV) {
                            // column pointer at this lane's first row, plus the
                            // row's distance from it times H*W (wave-uniform)
                            if (in) x = Ct[cbase[j] + (int64_t)row0 * hw + (int64_t)(row - row0) * hw];
                        } else {
                            x = in ? Ct[row * ldc + col] : (out_t)0;
                        }
                        if constexpr (DT == DT_F8) {
                            const float y = x * inv_alpha;
                            over |= __builtin_isinf(y) && !__builtin_isinf(x);
                            acc[i][j][r] = y;
                        } else {
                            acc[i][j][r] = x;
                        }
                    }
            if constexpr (DT == DT_F8) {
                if (__any(over)) {
                    c_in_acc = false;
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) {
                        if constexpr (MF == 32) acc[i][j] = acc_t{};
                        else acc[i][j] = acc_t{0, 0, 0, 0};
                    }
                }
            }
        }

        if constexpr (REG) {
            if (nk > 0) reg_store(lds, qa[0], qb[0], wave, lane, rs);
        }
        if constexpr (!REG) {
            for (int it = 0; it < nk; ++it) {
                // stage `it` has landed once at most (stages issued after it) loads remain
                wait_stage<(STAGES >= 2 ? STAGES - 2 : 0)>(min(STAGES - 2, nk - 1 - it));
                // all of this workgroup's waves: stage `it` visible, stage it-1 fully read
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                const uint8_t* sa = lds + (it % NBUF) * STAGE;
                mma_stage(sa, sa + A_STAGE, acc, wy, wx, lr, lg, [&] {
                    if (it + STAGES - 1 >= nk) return;
                    uint8_t* dst = lds + ((it + STAGES - 1) % STAGES) * STAGE;
                    if constexpr (CONV)
                        issue_stage_conv(g, ra, rb, voff_a, rs, (s_beg + it + STAGES - 1) * BK, dst, wave);
                    else
                        issue_stage(ra, rb, voff_a, voff_b, (s_beg + it + STAGES - 1) * BK, g.ldb, dst, wave);
                });
            }
        } else {
            // PF register sets, stage s in set s % PF, two LDS buffers: iteration
            // it loads stage it+PF into the set that held stage it (written to
            // LDS one iteration earlier), multiplies stage it, and writes stage
            // it+1 (loaded PF-1 iterations earlier) to the buffer stage it-1 used.
            // The body is unrolled PF times so that every set index is a constant.
            for (int it0 = 0; it0 < nk; it0 += PF) {
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int it = it0 + u;
                    if (it >= nk) break;
                    if (it + PF < nk) reg_load(g, rs, (s_beg + it + PF) * BK, qa[u], qb[u]);
                    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                    const uint8_t* sa = lds + (it & 1) * STAGE;
                    mma_stage(sa, sa + A_STAGE, acc, wy, wx, lr, lg, [] {});
                    if (it + 1 < nk)
                        reg_store(lds + ((it + 1) & 1) * STAGE, qa[(u + 1) % PF], qb[(u + 1) % PF], wave, lane,
                                  rs);
                }
            }
        }
        // epilogue: lane l, register r holds output row 4*(l/16) + r, column l % 16
        const MLK_GLOBAL float* const bias =
            !EPI || CONV || DT == DT_I8 || kz != 0 ? nullptr : (const MLK_GLOBAL float*)g.bias;
        // a bf16 C (direct-to-LDS forms only; never split) is read back, added in
        // fp32 and rounded once; the register-loaded form has no registers to spare
        constexpr bool OUT16 = EPI == 2 && !CONV && !REG;
        if constexpr (OUT16) {
            // Lanes l and l ^ 1 hold columns c and c + 1 (c even) of the same
            // four rows: they swap two values (DPP quad permute [1,0,3,2]) so that
            // the even lane writes rows 0-1 and the odd lane rows 2-3 of the
            // pair, each as one 32-bit store of two bf16 codes.  A pair cut by the
            // edge of C, or not 4-byte aligned (odd ldc), is written per element.
            const bool odd = (lr & 1) != 0;
            const bool al = (ldc & 1) == 0 && ((uintptr_t)g.C & 3) == 0;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int col = col0 + j * 16, cp = col & ~1;
                const float bn = bias && (full || col < nrem) ? bias[n0 + col] : 0.0f;
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    float v[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = (DT == DT_F8 ? alpha * acc[i][j][r] : acc[i][j][r]) + bn;
                    const float x0 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(odd ? v[0] : v[2]), 0xB1, 0xF, 0xF, true));
                    const float x1 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(odd ? v[1] : v[3]), 0xB1, 0xF, 0xF, true));
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int row = row0 + i * 16 + (odd ? 2 + h : h);
                        const float xh = h ? x1 : x0;
                        const float lo = odd ? xh : v[h];          // column cp
                        const float hi = odd ? v[2 + h] : xh;      // column cp + 1
                        const bool in_lo = full || (row < mrem && cp < nrem);
                        const bool in_hi = full || (row < mrem && cp + 1 < nrem);
                        if (!in_lo) continue;
                        MLK_GLOBAL uint16_t* q = Cb + row * ldc + cp;
                        if (in_hi && al) {
                            MLK_GLOBAL uint32_t* qd = (MLK_GLOBAL uint32_t*)q;
                            float a = lo, b = hi;
                            if (g.accumulate) {
                                const uint32_t c = *qd;
                                a = bf16_value((uint16_t)(c & 0xFFFFu)) + a;
                                b = bf16_value((uint16_t)(c >> 16)) + b;
                            }
                            *qd = (uint32_t)bf16_rne(a) | ((uint32_t)bf16_rne(b) << 16);
                        } else {
                            q[0] = bf16_rne(g.accumulate ? bf16_value(q[0]) + lo : lo);
                            if (in_hi) q[1] = bf16_rne(g.accumulate ? bf16_value(q[1]) + hi : hi);
                        }
                    }
                }
            }
        } else if constexpr (CONV) {
            // NFHW outputs: one pointer per column tile at this lane's first row,
            // rows at a compile-time distance times H*W; the store mode (plain,
            // read-add-write, atomic) is chosen once for the tile
            // (tiles wholly inside the output skip the bounds tests)
            auto conv_out = [&](auto mode, auto whole) {
                constexpr int MODE = decltype(mode)::value;
                constexpr bool WHOLE = decltype(whole)::value;
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int col = col0 + j * MF;
                    const bool colok = WHOLE || col < nrem;
                    MLK_GLOBAL out_t* const pj = Ct + cbase[j] + (int64_t)row0 * hw;
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int r = 0; r < NR; ++r) {
                            const int dr = rowof(i, r) - row0;
                            if (!(WHOLE || (colok && row0 + dr < mrem))) continue;
                            MLK_GLOBAL out_t* p = pj + (int64_t)dr * hw;
                            const out_t v = DT == DT_F8 ? alpha * acc[i][j][r] : acc[i][j][r];
                            if constexpr (MODE == 2) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            else if constexpr (MODE == 0) *p = v;
                            else *p = *p + v;
                        }
                }
            };
            auto by_extent = [&](auto mode) {
                if (full) conv_out(mode, std::true_type{});
                else conv_out(mode, std::false_type{});
            };
            if (g.atomic) by_extent(std::integral_constant<int, 2>{});
            else if (c_in_acc || !g.accumulate) by_extent(std::integral_constant<int, 0>{});
            else by_extent(std::integral_constant<int, 1>{});
        } else {
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int col = col0 + j * MF;
                const float bn = bias && (full || col < nrem) ? bias[n0 + col] : 0.0f;
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const int row = rowof(i, r);
                        if (!(full || (row < mrem && col < nrem))) continue;
                        MLK_GLOBAL out_t* p = CONV ? Ct + cbase[j] + row * hw : Ct + row * ldc + col;
                        out_t v;
                        if constexpr (DT == DT_I8) {
                            v = acc[i][j][r];
                        } else {
                            const float v0 = DT == DT_F8 ? alpha * acc[i][j][r] : acc[i][j][r];
                            v = EPI ? v0 + bn : v0;
                        }
                        if (g.atomic) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else if (c_in_acc || !g.accumulate) *p = v;
                        else *p = (out_t)((DT == DT_I8) ? (int32_t)((uint32_t)*p + (uint32_t)v) : *p + v);
                    }
            }
        }
    }
};

}  // namespace mlk
