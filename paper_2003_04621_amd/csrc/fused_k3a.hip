// fused_k3a.hip -- instantiates the persistent batch kernel k_batch<3, F>
// for the feature sets F in [0, 16).
#include "fused_device.h"

namespace ptsg {

BatchKernel batch_kernel_3a(int feat) {
  return pick_kernel<3>(feat - 0, std::make_integer_sequence<int, 16>{}, std::integral_constant<int, 0>{});
}

}  // namespace ptsg
