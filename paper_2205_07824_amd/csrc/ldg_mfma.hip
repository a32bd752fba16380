// Mixed-precision Jacobian-vector product of the linear models with the
// derivative and test contractions on MFMA (bf16 / fp16 operands, fp32
// accumulation).
#include "ldg_internal.hpp"

namespace ldg {

ldg_status op_mfma_jvp(const Model& md, const TimeDev& t, const double* v, double* out, bool fp16, hipStream_t s) {
  (void)md; (void)t; (void)v; (void)out; (void)fp16; (void)s;
  set_error("MFMA JVP not available for this configuration");
  return LDG_EUNSUPPORTED;
}

}  // namespace ldg
