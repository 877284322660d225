// Compiled sizes of the null-space weight kernel: 3D with 24-entry row arrays, 3D with 40-entry row arrays.
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_INSTANCE(3, 24)
RBF_NS_INSTANCE(3, 40)

}  // namespace rbf
