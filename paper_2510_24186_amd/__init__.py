"""MI355X-native batched docking hot path (TRIDS, arXiv 2510.24186).

The computation lives in libdock.so (hand-written HIP for gfx950, C ABI in
include/dock.h); `binding` marshals arguments with the ABI's names.
"""
from .binding import *  # noqa: F401,F403
from .binding import lib, DockError, Pocket, Ligands, Run  # noqa: F401
from .autograd import DockScoreFn, dock_score  # noqa: F401
