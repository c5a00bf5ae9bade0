// Whole-system NLTE kernels (k_nlte<NT, 0>), one per species-size bound.
#include "nlte_kernel.hpp"

namespace extrass {

bool launch_nlte_whole(int nt, unsigned blocks, size_t lds, hipStream_t st, const NArgs& A) {
  switch (nt) {
    case 16: hipLaunchKernelGGL((k_nlte<16, 0>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 24: hipLaunchKernelGGL((k_nlte<24, 0>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 32: hipLaunchKernelGGL((k_nlte<32, 0>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 40: hipLaunchKernelGGL((k_nlte<40, 0>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 50: hipLaunchKernelGGL((k_nlte<50, 0>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 64: hipLaunchKernelGGL((k_nlte<64, 0>), dim3(blocks), dim3(64), lds, st, A); return true;
    default: return false;
  }
}

}  // namespace extrass
