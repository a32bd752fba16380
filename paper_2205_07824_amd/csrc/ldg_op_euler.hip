// Operator kernels instantiated for one model kind (euler).
#include "ldg_operator_launch.hpp"

namespace ldg {
LDG_DEFINE_KIND_OPS(2)
}  // namespace ldg
