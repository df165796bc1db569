"""MI355X-native Newton step of the barrier-free augmented-Lagrangian contact
solver: HIP kernels for gfx950 behind the C-ABI of include/bfal.h."""
from . import bfal  # noqa: F401
