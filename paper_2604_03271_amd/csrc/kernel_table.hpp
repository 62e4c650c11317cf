// kernel_table.hpp -- host-side table of the move / energy kernel instantiations.
//
// Tiles: lanes per chain (16, 32 or 64 lanes of one wavefront, or 4 whole
// wavefronts = 256 lanes) x points per lane (PPL, a compile-time register
// budget; the row loops stop at ceil(N / lanes)).
#pragma once

#include <hip/hip_runtime.h>

namespace smc {

constexpr int kNumLaneCfg = 4;            // 16x1, 32x1, 64x1, 64x4
constexpr int kLanesOf[kNumLaneCfg] = {16, 32, 64, 256};
constexpr int kNumPpl = 5;
constexpr int kPplOf[kNumPpl] = {2, 4, 8, 16, 32};

struct KernelTable {
    const void* move[2][2][kNumLaneCfg][kNumPpl];
    const void* energy[2][2][kNumLaneCfg][kNumPpl];
};

void register_kernels_00(KernelTable& t);
void register_kernels_01(KernelTable& t);
void register_kernels_10(KernelTable& t);
void register_kernels_11(KernelTable& t);

}  // namespace smc
