// Compiled sizes of the null-space weight kernel (dimension, LU row entries, Cholesky row entries): (2, 16, 16), (2, 24, 24), (2, 40, 40), (2, 64, 64).
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_INSTANCE(2, 16, 16)
RBF_NS_INSTANCE(2, 24, 24)
RBF_NS_INSTANCE(2, 40, 40)
RBF_NS_INSTANCE(2, 64, 64)

}  // namespace rbf
