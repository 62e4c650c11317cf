// kernel_inst.hpp -- instantiates every tile of k_move / k_energy for one
// (peak kind, noise kind) pair; included once per translation unit so the
// instantiations compile in parallel.
#pragma once

#include "chain.hpp"
#include "kernel_table.hpp"

namespace smc {

template <int PK, int NZ, int L, int WPC, int PPL>
inline void reg_one(KernelTable& t, int lc, int pi) {
    t.move[PK][NZ][lc][pi] = reinterpret_cast<const void*>(&k_move<PK, NZ, L, WPC, PPL>);
    t.energy[PK][NZ][lc][pi] = reinterpret_cast<const void*>(&k_energy<PK, NZ, L, WPC, PPL>);
}

template <int PK, int NZ, int L, int WPC, int... PPLS>
inline void reg_list(KernelTable& t, int lc) {
    int pi = 0;
    (reg_one<PK, NZ, L, WPC, PPLS>(t, lc, pi++), ...);
}

template <int PK, int NZ, int L, int WPC>
inline void reg_ppl(KernelTable& t, int lc) {
    reg_list<PK, NZ, L, WPC, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32>(t, lc);
}

template <int PK, int NZ>
inline void reg_all(KernelTable& t) {
    reg_ppl<PK, NZ, 16, 1>(t, 0);
    reg_ppl<PK, NZ, 32, 1>(t, 1);
    reg_ppl<PK, NZ, 64, 1>(t, 2);
    reg_ppl<PK, NZ, 64, 4>(t, 3);
}

}  // namespace smc
