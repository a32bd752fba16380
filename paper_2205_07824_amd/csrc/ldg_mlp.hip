// Element-patch MLP preconditioner kernels (placeholder translation unit).
#include "ldg_internal.hpp"
