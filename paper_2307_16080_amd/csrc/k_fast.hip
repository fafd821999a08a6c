// bf16 matmul configurations of the direct-to-LDS kernel (large aligned problems).
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_fast(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY_FAST(256, 256, 2, 2, 2),
        MLK_ENTRY_FAST(256, 256, 2, 4, 2),
        MLK_ENTRY_FAST(256, 256, 4, 2, 2),
        MLK_ENTRY_FAST(256, 128, 2, 2, 3),
        MLK_ENTRY_FAST(128, 256, 2, 2, 3),
        MLK_ENTRY_FAST(128, 128, 2, 2, 4),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
