"""wig2: an MI355X-native two-body Wigner (phase-space 2-RDM) step.

The compute path is the HIP library ``libwig2.so`` behind the C ABI declared in
``include/wig2.h``; :mod:`paper_2511_11354_amd.wig2` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first use
and raises if it is missing.
"""
__all__ = ["inputs", "wig2"]
