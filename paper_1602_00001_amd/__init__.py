"""Dense-inverse solves of the 5-point variable-permittivity Poisson operator on
AMD MI355X (gfx950): HIP kernels behind the C-ABI of include/pinv.h.

Submodules: ``pinv`` (the ctypes binding, loads the built library),
``autograd`` (torch.autograd.Function), ``workloads`` (seeded synthetic
inputs), ``build`` (compiles the library)."""

__version__ = "0.1.0"
