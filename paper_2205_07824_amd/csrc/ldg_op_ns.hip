// Operator kernels instantiated for one model kind (ns).
#include "ldg_operator_launch.hpp"

namespace ldg {
LDG_DEFINE_KIND_OPS(3)
}  // namespace ldg
