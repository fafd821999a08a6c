// OCP e4m3 matmul tile configurations (MFMA 16x16x128 f8f6f4, fp32 accumulation).
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_f8(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY(DT_F8, 32, 32, 128, 1, 1, false),
        MLK_ENTRY(DT_F8, 64, 64, 128, 2, 2, false),
        MLK_ENTRY(DT_F8, 128, 64, 128, 2, 2, false),
        MLK_ENTRY(DT_F8, 64, 128, 128, 2, 2, false),
        MLK_ENTRY(DT_F8, 128, 128, 128, 2, 2, false),
        MLK_ENTRY(DT_F8, 128, 128, 256, 2, 2, false),
        MLK_ENTRY(DT_F8, 256, 128, 128, 2, 2, false),
        MLK_ENTRY(DT_F8, 128, 256, 128, 2, 2, false),
        MLK_ENTRY(DT_F8, 256, 256, 128, 2, 2, false),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
