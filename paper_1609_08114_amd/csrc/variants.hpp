// Table of register-tile kernel variants.  Each entry fixes the thread grid
// of one kernel template:
//   BLP_LANE_VARIANT (name, R rows, C columns, waves per workgroup, waves
//     per SIMD): simplex_lane_kernel, one LP per lane (64 LPs per wave);
//   BLP_REG_VARIANT (name, waves, TC threads per tableau row, CT columns per
//     thread, waves per SIMD): simplex_reg_kernel, one LP per workgroup,
//     a tableau of 64*waves/TC rows by TC*CT columns;
//   BLP_BLK_VARIANT (name, waves, GC column groups, RB rows and CB columns
//     per thread, waves per SIMD): simplex_blk_kernel, one LP per workgroup;
//   BLP_COLS_VARIANT (name, waves, GCW lanes across a wave's columns, RB
//     rows and CB slots per lane, waves per SIMD, max rows, max columns):
//     simplex_cols_kernel, one LP per workgroup, the columns split between
//     the waves; it holds (64/GCW) RB constraint rows by waves GCW CB slots
//     and claims the stated shape.  It takes only LPs without artificial
//     rows under the largest-coefficient rule (type1_only).
// Shapes count the objective rows and the rhs column.  The scheduler sends
// each LP to the fitting variant of smallest area, the first in this order
// among equal areas: the lane variants come first, a column-split variant
// comes before the block tile of its shape (it takes the LPs it can), and
// the row-tile w4/w8 variants (the first design, kept for comparison and the
// autotuner) come after the block tiles of their shapes.
#pragma once

#include "blp_kernels.hpp"

namespace blp {

struct RegVariant {
    const char* name;
    int threads;
    int max_rows;
    int max_cols;
    hipError_t (*launch)(const KParams&, int grid, hipStream_t);
    const void* (*kernel)();
    int lps_per_block;  // LPs a workgroup takes at once (lane kernel: one per thread)
    int type1_only;     // 1: only LPs with no artificial rows, largest-coefficient rule
};

// Host-side table of the compiled variants.
const RegVariant* reg_variants(int* count);

// clang-format off
#define BLP_REG_VARIANT_LIST                                  \
    BLP_LANE_VARIANT("l64_r8_c8",    8, 8,  4, 2)            \
    BLP_LANE_VARIANT("l64_r7_c11",   7, 11, 4, 2)            \
    BLP_REG_VARIANT("w1_r8_c8",      1, 8,   1, 4)           \
    BLP_REG_VARIANT("w1_r16_c16",    1, 4,   4, 4)           \
    BLP_REG_VARIANT("w1_r32_c32",    1, 2,  16, 2)           \
    BLP_REG_VARIANT("w2_r64_c64",    2, 2,  32, 1)           \
    BLP_BLK_VARIANT("b4_r112_c112",  4, 16, 7, 7, 2)         \
    BLP_COLS_VARIANT("c4_r112_c112", 4, 4, 7, 7, 2, 112, 112) \
    BLP_BLK_VARIANT("b8_r128_c112",  8, 16, 4, 7, 2)         \
    BLP_BLK_VARIANT("b8_r128_c128",  8, 16, 4, 8, 2)         \
    BLP_BLK_VARIANT("b8_r160_c160",  8, 16, 5, 10, 2)        \
    BLP_REG_VARIANT("w4_r128_c112",  4, 2,  56, 2)           \
    BLP_REG_VARIANT("w8_r128_c128",  8, 4,  32, 2)
// clang-format on

}  // namespace blp
