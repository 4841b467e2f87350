"""MI355X (gfx950) implementation of the solve path of Multigrid Assisted
Reanalysis (MGAR) for SIMP heat-conduction topology optimisation.

The numerical work lives in libmgar.so (HIP, built by ``build.py``); this
package holds its thin ctypes binding (``mgar``) and the optimisation-loop
driver (``topopt``), which sequences library calls only.
"""
from . import mgar  # noqa: F401
