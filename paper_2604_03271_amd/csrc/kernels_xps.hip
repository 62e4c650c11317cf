// Move / energy kernel instantiations of the XPS model form (pseudo-Voigt peaks, Shirley
// background, heteroscedastic noise): one-wavefront lane configurations, at most 16 points
// per lane.
#include "chain_xps.hpp"
#include "kernel_table.hpp"

namespace smc {
namespace {

template <int L, int PPL>
void reg_xps_one(KernelTable& t, int lc, int pi) {
    t.move[SMC_PEAK_PVOIGT][SMC_NOISE_HETERO][lc][pi] = reinterpret_cast<const void*>(&k_move_xps<L, PPL>);
    t.energy[SMC_PEAK_PVOIGT][SMC_NOISE_HETERO][lc][pi] = reinterpret_cast<const void*>(&k_energy_xps<L, PPL>);
}

template <int L, int... PPLS>
void reg_xps_list(KernelTable& t, int lc) {
    int pi = 0;
    (reg_xps_one<L, PPLS>(t, lc, pi++), ...);
}

}  // namespace

void register_kernels_xps(KernelTable& t) {
    reg_xps_list<16, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16>(t, 0);
    reg_xps_list<32, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16>(t, 1);
    reg_xps_list<64, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16>(t, 2);
}

}  // namespace smc
