// Stage-block NLTE kernels with the fixed-point steps reduced in FP32
// (k_nlte<0, NTB, true>), one per block-size bound.
#include "nlte_kernel.hpp"

namespace extrass {

bool launch_nlte_blocks_mixed(int ntb, unsigned blocks, size_t lds, hipStream_t st, const NArgs& A) {
  switch (ntb) {
    case 12: hipLaunchKernelGGL((k_nlte<0, 12, true>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 16: hipLaunchKernelGGL((k_nlte<0, 16, true>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 21: hipLaunchKernelGGL((k_nlte<0, 21, true>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 22: hipLaunchKernelGGL((k_nlte<0, 22, true>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 24: hipLaunchKernelGGL((k_nlte<0, 24, true>), dim3(blocks), dim3(64), lds, st, A); return true;
    case 32: hipLaunchKernelGGL((k_nlte<0, 32, true>), dim3(blocks), dim3(64), lds, st, A); return true;
    default: return false;
  }
}

}  // namespace extrass
