// kernel_table.hpp -- host-side table of the move / energy kernel instantiations.
//
// Tiles: lanes per chain (16, 32 or 64 lanes of one wavefront, or 2, 4 or 8 whole
// wavefronts = 128, 256 or 512 lanes) x points per lane (PPL, compile time; the smallest
// listed value >= ceil(N / lanes), points beyond N padded with zero-weight ones).
#pragma once

#include <hip/hip_runtime.h>

#include "smc_types.hpp"

namespace smc {

constexpr int kNumLaneCfg = 6;            // 16x1, 32x1, 64x1, 64x4, 64x8, 64x2
constexpr int kLanesOf[kNumLaneCfg] = {16, 32, 64, 256, 512, 128};
// the lane configurations by increasing lane count (the tile rule's search order)
constexpr int kLaneOrder[kNumLaneCfg] = {0, 1, 2, 5, 3, 4};
// the points-per-lane list (kNumPpl, kPplOf) is in smc_types.hpp: the kernels read it too

// [peak kind][noise kind][lane configuration][points per lane]; noise kind 2 (heteroscedastic,
// with the Shirley background) exists for pseudo-Voigt peaks, one-wavefront lane
// configurations and at most 16 points per lane only; peak kind 2 (XRD) for Poisson counts
// and at most 20 points per lane; 128 and 512 lanes (workgroups of 128 or 512 threads, one
// chain) for XRD only (other entries are null).
struct KernelTable {
    const void* move[3][3][kNumLaneCfg][kNumPpl];
    const void* energy[3][3][kNumLaneCfg][kNumPpl];
};

void register_kernels_00(KernelTable& t);
void register_kernels_01(KernelTable& t);
void register_kernels_10(KernelTable& t);
void register_kernels_11(KernelTable& t);
void register_kernels_xps(KernelTable& t);
void register_kernels_xrd(KernelTable& t);

}  // namespace smc
