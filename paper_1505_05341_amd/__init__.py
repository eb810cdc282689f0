"""LOS-dependent power-spectrum multipoles (P0, P2, P4) with FFTs on AMD MI355X.

A from-scratch HIP implementation of the FFT-based Yamamoto estimator of Bianchi,
Gil-Marin, Ruggeri & Percival (2015). The C interface is include/pk.h (libpk.so);
this package is its Python binding plus the seeded synthetic catalogue generators.
"""
from .native import PkError, get_schedule, load, set_schedule  # noqa: F401
from .api import (DeviceCatalog, Workspace, autotune, pk_multipoles, pk_multipoles_batch,  # noqa: F401
                  hgrid_view, stage_contract, stage_fft, stage_xgrids, xgrid_row, xgrid_view)
