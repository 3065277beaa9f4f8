"""MI355X (gfx950) steady discrete adjoint lattice Boltzmann solver.

Hot path of Luo, Chen, Yaji & Tao, "Improved adjoint lattice Boltzmann method
for topology optimization of laminar convective heat transfer" (arXiv
2501.02161): a Brinkman-penalised D3Q19 BGK flow lattice coupled to a D3Q7
thermal lattice, its fully consistent discrete adjoint and the dJ/dgamma
reduction, behind the C ABI of include/lbmadj.h.

Importing this package does not load the GPU library; :mod:`.lbm` does, and
raises if the library has not been built (see :mod:`.build`).
"""

__all__ = ["lbm", "build"]
