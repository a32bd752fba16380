"""Physics sources for run-time compiled models in the tests: the package's model sources plus a source
that does not compile (for the error paths)."""
from paper_2205_07824_amd.physics import (EULER_2D, EULER_2D_SLIP, NONLINEAR_DIFFUSION,  # noqa: F401
                                          REACTION_DIFFUSION, REACTION_DIFFUSION_BOU, SHALLOW_WATER_2D, WAVE_2D,
                                          WAVE_2D_W)

BROKEN = r"""
struct LdgUser {
  static constexpr int NCU = 1;
  static constexpr bool HASQ = true;
  static constexpr int NAUX = 0;
  this is not C++;
};
"""
