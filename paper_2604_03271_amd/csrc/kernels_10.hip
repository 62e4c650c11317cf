// Move / energy kernel instantiations: peak kind 1, noise kind 0.
#include "kernel_inst.hpp"
namespace smc {
void register_kernels_10(KernelTable& t) { reg_all<1, 0>(t); }
}  // namespace smc
