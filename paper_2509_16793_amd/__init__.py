"""MI355X (gfx950) Galilean PIC step: a C-ABI HIP library and its ctypes binding."""
from .gempic import Sim, lib, LIB_PATH  # noqa: F401
