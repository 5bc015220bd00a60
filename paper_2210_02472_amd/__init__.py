"""MI355X (gfx950) direct-summation pass of the HHS-FSI integrator (BIFROST, arXiv 2210.02472).

``paper_2210_02472_amd.Context`` wraps the C ABI of ``libbifrost_hip.so`` (include/bifrost.h);
``paper_2210_02472_amd.ics`` generates seeded synthetic cluster inputs.  The HIP library is
loaded on first use of a Context and there is no CPU fallback.
"""
from ._binding import (BF_A_VALID, BF_FLAG_BADINDEX, BF_FLAG_COINCIDENT, BF_FLAG_NONFINITE,  # noqa: F401
                       BF_OP_DTMIN, BF_OP_FORCES, BF_OP_GRADIENT, BifrostError, Context, Graph, LIB_PATH,
                       Particles, ParticleSet, load_library)

__all__ = ["Context", "Particles", "ParticleSet", "Graph", "BifrostError", "load_library", "LIB_PATH"]
