"""qtp: QTT-accelerated PDIP Newton-step solver for frictional contact (MI355X).

The compute path is the HIP library ``libqtp.so`` built from ``csrc/``; the
Python module ``binding`` only marshals arguments (device pointers from torch
tensors, the current HIP stream) into its C ABI, declared in
``include/qtp.h``.  Importing the binding fails loudly when the library has
not been built.
"""
