// Compiled sizes of the null-space weight kernel (dimension, LU row entries, Cholesky row entries): (3, 20, 32), (3, 36, 40).
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_INSTANCE(3, 20, 32)
RBF_NS_INSTANCE(3, 36, 40)

}  // namespace rbf
