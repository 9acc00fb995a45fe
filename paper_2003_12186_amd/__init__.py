"""MI355X (gfx950) implementation of the D2Q9 immersed interface-lattice
Boltzmann method (II-LBM) of Qin, Kolahdouz & Griffith, arXiv:2003.12186.

The method runs in the HIP kernels of ``libiilbm.so`` behind the C ABI of
``include/ii_lbm.h``; ``binding`` is its ctypes binding (``binding.Sim``) and
``workloads`` the seeded synthetic problem generator.  Nothing is loaded at
import time.
"""
__all__ = ["binding", "workloads", "build"]
