"""MI355X overset connectivity: direct cut of curved quadratic grids and
Newton donor search, as hand-written HIP for gfx950 behind a C ABI
(include/oc.h).  ``oc`` is the ctypes binding; ``pipeline`` runs the
connectivity step of a registered overset system."""
from . import oc  # noqa: F401
