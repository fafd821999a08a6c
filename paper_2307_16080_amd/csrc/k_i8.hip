// int8 x int8 -> int32 matmul tile configurations (MFMA 16x16x64 i8): the
// register-staged tile and the direct-layout kernel.
#include "kernels.hpp"
namespace mlk {
const KernelEntry* kernels_i8(int* n) {
    static const KernelEntry t[] = {
        MLK_ENTRY(DT_I8, 32, 32, 128, 1, 1, false),
        MLK_ENTRY(DT_I8, 64, 64, 64, 2, 2, false),
        MLK_ENTRY(DT_I8, 64, 64, 128, 2, 2, false),
        MLK_ENTRY(DT_I8, 128, 64, 128, 2, 2, false),
        MLK_ENTRY(DT_I8, 64, 128, 128, 2, 2, false),
        MLK_ENTRY(DT_I8, 128, 128, 64, 2, 2, false),
        MLK_ENTRY(DT_I8, 128, 128, 128, 2, 2, false),
        MLK_ENTRY(DT_I8, 256, 128, 128, 2, 2, false),
        MLK_ENTRY(DT_I8, 256, 256, 128, 2, 2, false),
        // direct-layout kernel (MFMA 16x16x64 i8, B transposed by ds_read_b64_tr_b8):
        // direct-to-LDS rings of 2-4 stages, and the register-loaded form (any alignment)
        MLK_ENTRY_FAST_I8(32, 64, 1, 2, 3),   // 2 waves: twice the workgroups of 64 x 64
        MLK_ENTRY_FAST_I8(32, 64, 1, 2, 4),
        MLK_ENTRY_FAST_I8(64, 64, 1, 2, 4),
        MLK_ENTRY_FAST_I8(64, 64, 2, 4, 4),   // 8 waves: more in flight per CU
        MLK_ENTRY_FAST_I8(64, 64, 2, 2, 2),
        MLK_ENTRY_FAST_I8(64, 64, 2, 2, 3),
        MLK_ENTRY_FAST_I8(64, 64, 2, 2, 4),
        // deep rings: at K = 1024 every stage of a 64 x 64 tile is in flight
        // from the start (8 x 16 KB of LDS), so the loop waits once per stage
        // for data already requested instead of for a copy issued a few
        // stages earlier
        MLK_ENTRY_FAST_I8(64, 64, 2, 2, 6),
        MLK_ENTRY_FAST_I8(64, 64, 2, 2, 8),
        MLK_ENTRY_FAST_I8(64, 64, 1, 2, 8),
        MLK_ENTRY_FAST_I8(32, 64, 1, 2, 8),
        MLK_ENTRY_FAST_I8(128, 64, 2, 2, 3),
        MLK_ENTRY_FAST_I8(64, 128, 2, 2, 3),
        MLK_ENTRY_FAST_I8(128, 128, 2, 2, 2),
        MLK_ENTRY_FAST_I8(128, 128, 2, 2, 4),
        MLK_ENTRY_FAST_I8(256, 128, 2, 2, 3),
        MLK_ENTRY_FAST_I8(256, 256, 2, 4, 2),
        MLK_ENTRY_FAST_I8(128, 128, 2, 2, 1),
    };
    *n = (int)(sizeof(t) / sizeof(t[0]));
    return t;
}
}  // namespace mlk
