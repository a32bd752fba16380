// Operator kernels instantiated for one model kind (convdiff).
#include "ldg_operator_launch.hpp"

namespace ldg {
LDG_DEFINE_KIND_OPS(1)
}  // namespace ldg
