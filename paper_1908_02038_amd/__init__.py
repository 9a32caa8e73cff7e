"""FIRE 2.0 energy minimisation on MI355X (gfx950): HIP kernels behind a C ABI.

Submodules:
  inputs    seeded synthetic FCC inputs (geometry only)
  api       ctypes binding of include/fire2.h (Context.fire_* methods)
  autograd  torch.autograd Functions whose backward passes are the force and
            Hessian-vector-product kernels
  build     hipcc build of libfire2.so

Importing the package loads nothing; the HIP library is loaded on first use
and there is no fallback if it is missing.
"""
__all__ = ["inputs", "api", "autograd", "build"]
