// Implicit-GEMM conv2d tile configurations: rows = output channels,
// columns = output pixels, depth = (c, kh, kw); fp32 and bf16 inputs.
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_conv(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY(DT_F32, 32, 32, 64, 1, 1, true),
        MLK_ENTRY(DT_F32, 32, 64, 64, 1, 2, true),
        MLK_ENTRY(DT_F32, 64, 32, 64, 2, 1, true),
        MLK_ENTRY(DT_F32, 64, 64, 64, 2, 2, true),
        MLK_ENTRY(DT_F32, 64, 128, 64, 2, 2, true),
        MLK_ENTRY(DT_F32, 128, 64, 64, 2, 2, true),
        MLK_ENTRY(DT_F32, 128, 128, 64, 2, 2, true),
        MLK_ENTRY(DT_BF16, 32, 32, 64, 1, 1, true),
        MLK_ENTRY(DT_BF16, 32, 64, 64, 1, 2, true),
        MLK_ENTRY(DT_BF16, 64, 32, 64, 2, 1, true),
        MLK_ENTRY(DT_BF16, 64, 64, 64, 2, 2, true),
        MLK_ENTRY(DT_BF16, 64, 128, 64, 2, 2, true),
        MLK_ENTRY(DT_BF16, 128, 64, 64, 2, 2, true),
        MLK_ENTRY(DT_BF16, 128, 128, 64, 2, 2, true),
        MLK_ENTRY(DT_BF16, 128, 128, 128, 2, 2, true),
        MLK_ENTRY(DT_BF16, 256, 128, 64, 2, 2, true),
        MLK_ENTRY(DT_BF16, 128, 256, 64, 2, 2, true),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
