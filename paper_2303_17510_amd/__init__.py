"""hdconv: hybrid-dealiased complex convolutions on MI355X (gfx950).

Murasko & Bowman, "Hybrid Dealiasing of Complex Convolutions" (arXiv
2303.17510), Sec. 2-6, built as a C-ABI HIP library (libhdconv.so, declared in
include/hdconv.h) with a thin Python front end.  Importing this package does
not load the library; the first plan does, and raises if it is not built.
"""
from .hdconv import BatchPlan, Plan, convolve, dtype_code, geometry  # noqa: F401

__all__ = ["Plan", "BatchPlan", "convolve", "geometry", "dtype_code"]
