"""MI355X (gfx950) extrapolated GBS time stepper for method-of-lines wave
problems (Ellison & Fornberg, "A parallel-in-time approach for wave-type
PDEs").

    from paper_1907_11771_amd import GBSPlan, weights

The HIP library (lib/libgbs.so) is built by ``python -m paper_1907_11771_amd.build``;
the modules here only marshal arguments to its C ABI (include/gbs.h).
"""
from .binding import (ACOUSTIC2D, ACOUSTIC3D, ADVECT1D, F32, F64, GBSError, isb,  # noqa: F401
                      weights)
from .plan import GBSBatch, GBSPlan, scheme_weights  # noqa: F401
