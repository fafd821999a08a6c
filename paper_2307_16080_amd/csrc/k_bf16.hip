// bf16 matmul tile configurations (MFMA 16x16x32 bf16, fp32 accumulation).
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_bf16(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY_P(DT_BF16, 32, 32, 128, 1, 1),
        MLK_ENTRY_P(DT_BF16, 64, 32, 128, 2, 1),
        MLK_ENTRY_P(DT_BF16, 32, 64, 128, 1, 2),
        MLK_ENTRY_P(DT_BF16, 64, 64, 64, 2, 2),
        MLK_ENTRY_P(DT_BF16, 64, 64, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 128, 64, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 64, 128, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 128, 128, 64, 2, 2),
        MLK_ENTRY_P(DT_BF16, 128, 128, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 256, 128, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 128, 256, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 256, 256, 64, 2, 2),
        MLK_ENTRY_P(DT_BF16, 256, 256, 128, 2, 2),
        MLK_ENTRY_P(DT_BF16, 256, 256, 128, 2, 4),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
