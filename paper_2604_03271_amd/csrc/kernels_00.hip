// Move / energy kernel instantiations: peak kind 0, noise kind 0.
#include "kernel_inst.hpp"
namespace smc {
void register_kernels_00(KernelTable& t) { reg_all<0, 0>(t); }
}  // namespace smc
