// Compiled sizes of the null-space weight kernel: 2D with 16-entry row arrays, 2D with 24-entry row arrays, 2D with 40-entry row arrays, 2D with 64-entry row arrays.
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_INSTANCE(2, 16)
RBF_NS_INSTANCE(2, 24)
RBF_NS_INSTANCE(2, 40)
RBF_NS_INSTANCE(2, 64)

}  // namespace rbf
