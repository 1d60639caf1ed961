"""MI355X (gfx950) implementation of the CDI + GNBC time step of
arXiv:2412.16843: hand-written HIP kernels behind the C ABI of include/cdi.h,
with a thin ctypes binding.  PyTorch provides device memory and streams."""
from ._lib import CDIError, lib  # noqa: F401
