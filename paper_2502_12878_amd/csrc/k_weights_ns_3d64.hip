// Compiled sizes of the null-space weight kernel: 3D with 64-entry row arrays.
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_INSTANCE(3, 64)

}  // namespace rbf
