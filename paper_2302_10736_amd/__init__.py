"""MI355X (gfx950) nodal power injections and polar power-flow Jacobians.

Element-wise and Ybus methods of "Bus Admittance Matrix Revisited: Is It
Outdated on Modern Computers?" (arXiv 2302.10736) as hand-written HIP
kernels behind the C ABI in ``include/pf.h``.

Submodules: ``pf`` (binding of the C ABI), ``autograd`` (torch Function),
``gridgen`` (seeded synthetic inputs), ``build`` (compiles libpf.so).
Importing the package loads nothing; ``pf`` loads the library on first use.
"""
__all__ = ["pf", "autograd", "gridgen", "build"]
