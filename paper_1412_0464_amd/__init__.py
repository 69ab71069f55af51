"""MI355X-native two-grid sweeping preconditioner for the Helmholtz equation
(Stolk, arXiv 1412.0464): HIP kernels for gfx950 behind the C ABI of
include/hsp.h, with a thin ctypes binding in ``hsp``."""
from .hsp import Group, Helmholtz, HspError, load, library_path, workspace_size  # noqa: F401
