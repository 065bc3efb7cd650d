"""MI355X (gfx950) fluctuating lattice Boltzmann: the D3Q19 collide-and-stream
update with detailed-balance thermal noise of Duenweg, Schiller & Ladd
(arXiv:0707.1581), as hand-written HIP kernels behind the C ABI of
include/lbf.h.  This package holds the kernels and the C ABI (csrc/), the
in-tree build (build.py) and the ctypes binding (lb.py)."""
from .lb import (Ensemble, LBError, Lattice, LbParams, LbSchedule, lib, make_params, physical_params,  # noqa: F401
                 STORAGE, STORAGE_DTYPE, INIT, THERMAL_MODES)
