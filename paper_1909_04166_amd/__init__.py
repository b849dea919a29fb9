"""MI355X-native coupled cascaded central-moment lattice Boltzmann time step
(pressure-based two-phase hydrodynamics + conservative Allen-Cahn phase field,
D2Q9), after Hajabdollahi, Premnath & Welch, arXiv:1909.04166.

The compute path is the HIP library ``libcmlb.so`` behind the C-ABI declared in
``include/cmlb.h``; ``paper_1909_04166_amd.lb`` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first use
and raises if it has not been built.
"""
