// Move / energy kernel instantiations: peak kind 0, noise kind 1.
#include "kernel_inst.hpp"
namespace smc {
void register_kernels_01(KernelTable& t) { reg_all<0, 1>(t); }
}  // namespace smc
