"""Exact graph N-point counts (triangles, parity 4-cliques) on AMD MI355X.

The computation lives in libgsn.so (HIP, gfx950), behind the C ABI declared in
include/gsn.h; gsn.py is its ctypes binding.
"""
from .gsn import (Context, Graph, GsError, Count3, Count4, Count6, Pairs, n_configs, n_configs6,  # noqa: F401
                  config6_table, load, EXPORTS, compute_3pcf, compute_4pcf, Result3pcf, Result4pcf,
                  GS_OK, GS_EINVAL, GS_EOVERFLOW, GS_ENOMEM, GS_EDEVMEM, GS_EHIP, GS_EAGAIN,
                  GS_ENOTFOUND, GS_EUNSUPPORTED, GS_ENOCOORDS, GS_WEIGHTED, GS_KEEP_COORDS,
                  GS_INPUT_ON_DEVICE, GS_NONPERIODIC, LIB_PATH, GS_DONE, GS_PENDING, GS_FAILED,
                  GS_CANCELLED, GS_3PCF, GS_4PCF_PARITY)
