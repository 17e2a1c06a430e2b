"""MI355X-native rank-profile-revealing PLDL^TP^T factorization over F_p.

The compute path lives in the HIP library ``libpldl.so`` built from ``csrc/``;
``pldl`` is its thin ctypes binding.  Importing this package loads nothing.
"""
