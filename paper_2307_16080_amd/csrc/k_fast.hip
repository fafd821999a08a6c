// Configurations of the direct-layout kernel (bf16 and e4m3): tile, wave
// grid, LDS stages (2..4: direct-to-LDS ring; 1: loaded through registers),
// and its channels-last convolution form.
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_fast(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY_FAST(DT_BF16, 256, 256, 2, 2, 2),
        MLK_ENTRY_FAST(DT_BF16, 256, 256, 2, 4, 2),
        MLK_ENTRY_FAST(DT_BF16, 256, 256, 4, 2, 2),
        MLK_ENTRY_FAST(DT_BF16, 256, 128, 2, 2, 3),
        MLK_ENTRY_FAST(DT_BF16, 128, 256, 2, 2, 3),
        MLK_ENTRY_FAST(DT_BF16, 128, 128, 2, 2, 4),
        MLK_ENTRY_FAST(DT_BF16, 128, 128, 2, 2, 2),  // 64 KB of LDS: two workgroups per CU
        MLK_ENTRY_FAST(DT_BF16, 64, 128, 2, 2, 2),   // 48 KB: three per CU
        // operands loaded through registers: any shape and alignment, persistent batches
        MLK_ENTRY_FAST(DT_BF16, 128, 128, 2, 2, 1),
        MLK_ENTRY_FAST(DT_BF16, 256, 128, 2, 2, 1),
        // 32 x 32 MFMA tiles (half the MFMA and LDS read instructions)
        MLK_ENTRY_FAST32(256, 256, 2, 4, 2),
        MLK_ENTRY_FAST32(256, 256, 4, 2, 2),
        MLK_ENTRY_FAST32(256, 256, 2, 2, 2),
        MLK_ENTRY_FAST32(256, 128, 2, 2, 3),
        MLK_ENTRY_FAST32(128, 256, 2, 2, 3),
        MLK_ENTRY_FAST32(128, 128, 2, 2, 4),
        MLK_ENTRY_FAST(DT_F8, 256, 256, 2, 4, 2),
        MLK_ENTRY_FAST(DT_F8, 256, 256, 4, 2, 2),
        MLK_ENTRY_FAST(DT_F8, 256, 256, 2, 2, 2),
        MLK_ENTRY_FAST(DT_F8, 256, 128, 2, 2, 3),
        MLK_ENTRY_FAST(DT_F8, 128, 256, 2, 2, 3),
        MLK_ENTRY_FAST(DT_F8, 128, 128, 2, 2, 4),
        MLK_ENTRY_FAST(DT_F8, 128, 128, 2, 2, 2),
        MLK_ENTRY_FAST(DT_F8, 128, 128, 2, 2, 1),
        // channels-last implicit-GEMM convolution (bf16, C a multiple of 8);
        // these register-loaded tiles also gather straight from NCHW (layout 3)
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 64, 2, 2, 1),
        MLK_ENTRY_FASTCONV(DT_BF16, 128, 128, 2, 2, 1),
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 128, 2, 2, 1),
        MLK_ENTRY_FASTCONV(DT_BF16, 128, 256, 2, 2, 1),
        MLK_ENTRY_FASTCONV(DT_BF16, 256, 128, 2, 2, 1),
        // the same gather issued as direct-to-LDS copies: C * KH * KW a multiple of 64
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 64, 2, 2, 2),    // 32 KB of LDS: five workgroups per CU
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 64, 2, 2, 3),
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 128, 2, 2, 2),
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 128, 2, 2, 3),
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 128, 2, 2, 4),
        MLK_ENTRY_FASTCONV(DT_BF16, 128, 128, 2, 2, 3),
        MLK_ENTRY_FASTCONV(DT_BF16, 128, 128, 2, 2, 4),
        MLK_ENTRY_FASTCONV(DT_BF16, 256, 128, 2, 2, 3),
        MLK_ENTRY_FASTCONV(DT_BF16, 64, 256, 2, 2, 3),   // few filters, many pixels
        MLK_ENTRY_FASTCONV(DT_BF16, 128, 256, 2, 2, 3),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
