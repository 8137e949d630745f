"""MI355X (gfx950) solver for the preconditioned Krylov solve of the Grunwald
discretisation of the space-fractional diffusion equation with the
symbol-based tau preconditioner P_F (Barakitis, Ekstrom, Vassalos).

The compute path is the HIP library ``libfde.so`` (C ABI in include/fde.h);
``paper_1912_13304_amd.fde`` is its ctypes binding.  Importing this package
loads nothing; importing ``.fde`` loads the library and raises if it is
missing.
"""
