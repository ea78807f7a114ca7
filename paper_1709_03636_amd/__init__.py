"""MI355X tensor-network contraction of quantum circuits (qTorch's method).

Host graph code (networks, orders, plans) and gfx950 HIP kernels live in the
native library libqtn.so (csrc/, C ABI in include/qtn.h); qtn.py is its
ctypes binding and qaoa.py the QAOA Max-Cut driver.
"""
from . import qtn  # noqa: F401
