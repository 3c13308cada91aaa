"""Batched projective-dynamics membrane solver for MI355X (gfx950).

The compute path is the HIP library ``libnpfem.so`` behind the C ABI in
``include/npfem.h``; ``solver`` wraps it with PyTorch-owned device memory.
Importing this package does not load the library; the first ``Mesh`` or
``Batch`` does, and raises if it is missing.
"""

__all__ = ["solver", "build"]
