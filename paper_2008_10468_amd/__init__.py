"""MI355X-native (gfx950) QED event generator for QED-PIC codes, after Volokitin et
al., "Optimized routines for event generators in QED-PIC codes" (arXiv:2008.10468).

The generator itself is the HIP library ``libqed.so`` (C ABI in ``include/qed.h``);
``paper_2008_10468_amd.qed`` is its ctypes binding.  Build with
``python -m paper_2008_10468_amd.build``.
"""
from . import qed  # noqa: F401
from .qed import (QED_F32, QED_F64, QED_PREC_F64, QED_PREC_MIXED, QED_SCHED_BINNED,  # noqa: F401
                  QED_SCHED_NAIVE, Generator, QedError, load, synchrotron)
