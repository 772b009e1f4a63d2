"""MI355X-native FFT estimator of redshift-space bispectrum multipoles.

The estimator (Gill & Bharadwaj, arXiv:2405.14513, Sec. II) runs in the HIP
kernels of ``libbk.so``; ``bk`` is a thin ctypes binding with the C ABI's
names (include/bk.h).  Build the library with ``python -m paper_2405_14513_amd.build``.
"""
from . import bk  # noqa: F401
from .bk import BK_F32, BK_F64, BkError, Estimator, make_binning  # noqa: F401
