// Move / energy kernel instantiations: peak kind 1, noise kind 1.
#include "kernel_inst.hpp"
namespace smc {
void register_kernels_11(KernelTable& t) { reg_all<1, 1>(t); }
}  // namespace smc
