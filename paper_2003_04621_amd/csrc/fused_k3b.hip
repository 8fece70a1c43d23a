// fused_k3b.hip -- instantiates the persistent batch kernel k_batch<3, F>
// for the feature sets F in [16, 32).
#include "fused_device.h"

namespace ptsg {

BatchKernel batch_kernel_3b(int feat) {
  return pick_kernel<3>(feat - 16, std::make_integer_sequence<int, 16>{}, std::integral_constant<int, 16>{});
}

}  // namespace ptsg
