"""MI355X-native hybrid thermal pseudopotential lattice Boltzmann boiling solver.

The time step of Li, Kang, Francois, He and Luo (arXiv:1501.03857) runs in
hand-written HIP kernels for gfx950 behind the C-ABI library ``liblbboil.so``
(declared in ``include/lbboil.h``).  ``lbboil`` is the thin ctypes binding over
that library; ``workloads`` builds the seeded synthetic inputs.  Importing the
package loads nothing; ``lbboil`` raises if the built library is missing.
"""
__all__ = ["lbboil", "workloads"]
