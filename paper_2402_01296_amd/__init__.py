"""MI355X-native ciphertext-branch engine for bi-CryptoNets (arXiv 2402.01296).

The HIP library (``lib/libbcn.so``, C ABI in ``include/bcn.h``) evaluates the
ciphertext branch in RNS-BFV on the GPU; ``bcn`` is its thin ctypes binding
and ``workload`` drives the synthetic workloads through it.
"""
from . import bcn  # noqa: F401
