"""MI355X (gfx950) implementation of the 1D3V electrostatic PIC/MCC step of Becker et al.,
arXiv:1608.04601, behind the C ABI of include/pic1d.h (libpic1d.so, built by
``python -m paper_1608_04601_amd.build``).  ``binding`` is the ctypes layer over it."""
from . import binding  # noqa: F401
from .binding import Config, Discharge, PicError  # noqa: F401
