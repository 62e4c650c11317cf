// Move / energy kernel instantiations of the XRD powder profile with Poisson counts: every lane
// configuration (512-lane chains included), at most 20 points per lane.
#include "chain_xrd.hpp"
#include "kernel_table.hpp"

namespace smc {
namespace {

template <int L, int WPC, int PPL>
void reg_xrd_one(KernelTable& t, int lc, int pi) {
    t.move[SMC_PEAK_XRD][SMC_NOISE_POISSON][lc][pi] = reinterpret_cast<const void*>(&k_move_xrd<L, WPC, PPL>);
    t.energy[SMC_PEAK_XRD][SMC_NOISE_POISSON][lc][pi] = reinterpret_cast<const void*>(&k_energy_xrd<L, WPC, PPL>);
}

template <int L, int WPC, int... PPLS>
void reg_xrd_list(KernelTable& t, int lc) {
    int pi = 0;
    (reg_xrd_one<L, WPC, PPLS>(t, lc, pi++), ...);
}

}  // namespace

void register_kernels_xrd(KernelTable& t) {
    reg_xrd_list<16, 1, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20>(t, 0);
    reg_xrd_list<32, 1, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20>(t, 1);
    reg_xrd_list<64, 1, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20>(t, 2);
    reg_xrd_list<64, 4, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20>(t, 3);
    reg_xrd_list<64, 8, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20>(t, 4);
    reg_xrd_list<64, 2, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20>(t, 5);
}

}  // namespace smc
