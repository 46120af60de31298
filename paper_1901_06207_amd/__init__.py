"""MI355X (gfx950) implementation of the CBAA super-host detector
(arXiv 1901.06207): HIP kernels behind the C ABI of include/cbaa.h, with a
ctypes binding in :mod:`paper_1901_06207_amd.cbaa`."""

from . import cbaa  # noqa: F401
from .cbaa import Config  # noqa: F401
