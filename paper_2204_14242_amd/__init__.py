"""MI355X-native analytic GPU metric estimator (Ernst et al., "Analytical
Performance Estimation during Code Generation on Modern GPUs").

The compute path is the HIP library ``libwsest.so`` (C-ABI in
``include/wsest.h``); ``wsest`` is its ctypes binding and ``workloads`` holds
the seeded input descriptions.  Importing the package loads nothing; the
binding raises if the library has not been built.
"""
__all__ = ["wsest", "workloads"]
