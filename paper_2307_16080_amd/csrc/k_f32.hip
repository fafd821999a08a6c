// fp32 matmul tile configurations (MFMA 16x16x4 f32).
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_f32(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY_P(DT_F32, 32, 32, 64, 1, 1),
        MLK_ENTRY_P(DT_F32, 64, 32, 64, 2, 1),
        MLK_ENTRY_P(DT_F32, 32, 64, 64, 1, 2),
        MLK_ENTRY_P(DT_F32, 64, 64, 64, 2, 2),
        MLK_ENTRY_P(DT_F32, 64, 64, 128, 2, 2),
        MLK_ENTRY_P(DT_F32, 128, 64, 64, 2, 2),
        MLK_ENTRY_P(DT_F32, 64, 128, 64, 2, 2),
        MLK_ENTRY_P(DT_F32, 128, 128, 64, 2, 2),
        MLK_ENTRY_P(DT_F32, 128, 128, 128, 2, 2),
        MLK_ENTRY_P(DT_F32, 256, 128, 64, 2, 2),
        MLK_ENTRY_P(DT_F32, 128, 256, 64, 2, 2),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
