"""MI355X-native curvilinear patch dynamics (arXiv 2405.08764).

The compute path lives in the HIP library ``libpd.so`` behind the C ABI declared in
``include/pd.h``; :mod:`paper_2405_08764_amd.pd` is its thin Python binding.  Importing
this package loads nothing; the binding loads the library on first use and raises if it
is missing.
"""

__all__ = ["workloads"]
