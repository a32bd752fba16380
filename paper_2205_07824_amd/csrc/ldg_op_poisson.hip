// Operator kernels instantiated for one model kind (poisson).
#include "ldg_operator_launch.hpp"

namespace ldg {
LDG_DEFINE_KIND_OPS(0)
}  // namespace ldg
