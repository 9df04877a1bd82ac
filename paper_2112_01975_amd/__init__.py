"""MI355X-native two-phase lattice Boltzmann step (Hosseini, Dorschner & Karlin,
"Towards a consistent lattice Boltzmann model for two-phase fluid").

The simulation runs in liblbm2p.so (hand-written HIP for gfx950, C ABI in
include/lbm2p.h); `lbm` is the ctypes binding. There is no CPU fallback.
"""
from .lbm import *  # noqa: F401,F403
from .lbm import Params, Simulation, LbmError, lib  # noqa: F401
