"""Plain CPU oracle for the rank-profile-revealing PLDL^TP^T factorization over F_p.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.
"""
