// fused_k2b.hip -- instantiates the persistent batch kernel k_batch<2, F>
// for the feature sets F in [16, 32).
#include "fused_device.h"

namespace ptsg {

BatchKernel batch_kernel_2b(int feat) {
  return pick_kernel<2>(feat - 16, std::make_integer_sequence<int, 16>{}, std::integral_constant<int, 16>{});
}

}  // namespace ptsg
