"""MI355X (gfx950) FDTD step for attenuating, nonlinear acoustic waves with
multiple relaxation mechanisms (Sode & Pinton, Fullwave 2.5 method).

Modules
-------
native   ctypes binding of libfw25.so (the C ABI of include/fw25.h)
sim      Simulation: one fw_sim object with a torch-owned device workspace
relax    host FP64 calibration of relaxation parameters (Sec. 3)
build    hipcc build of libfw25.so for gfx950
"""
