"""MI355X (gfx950) implementation of the coupled step of the conservative
Allen-Cahn lattice Boltzmann method with geometric ghost-node wetting and
global phase-field volume correction.

The method runs in libcac.so (HIP kernels behind the C ABI of include/cac.h);
this package only binds it (``capi``) and builds it (``build``).  Importing the
package does not load the library; constructing a ``Sim`` does, and fails when
the library is not built or no GPU is present.
"""
__all__ = ["capi", "workloads", "build"]
