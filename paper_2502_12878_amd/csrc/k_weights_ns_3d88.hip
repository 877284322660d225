// Compiled sizes of the null-space weight kernel (dimension, LU row entries, Cholesky row entries): (3, 84, 86).
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_INSTANCE(3, 84, 86)

}  // namespace rbf
