"""MI355X-native voxel cardiac electrophysiology time-stepper.

The method (operator-split Mitchell-Schaeffer reaction, 19-point
anisotropic finite-volume diffusion, Jacobi-preconditioned CG and the
mixed-precision bidomain elliptic solve) runs in the HIP library
``libep_hip.so``; :mod:`paper_2302_12519_amd.ep` is its ctypes binding.
Importing the package loads the library and fails if it is not built.
"""
from .ep import EPError, Grid, lib  # noqa: F401
