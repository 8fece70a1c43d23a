// fused_k2a.hip -- instantiates the persistent batch kernel k_batch<2, F>
// for the feature sets F in [0, 16).
#include "fused_device.h"

namespace ptsg {

BatchKernel batch_kernel_2a(int feat) {
  return pick_kernel<2>(feat - 0, std::make_integer_sequence<int, 16>{}, std::integral_constant<int, 0>{});
}

}  // namespace ptsg
