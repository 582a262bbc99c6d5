"""MI355X (gfx950) lattice Boltzmann MHD with a Smagorinsky-MHD closure.

Implements the per-site stream-and-collide update of Flint & Vahala,
"Lattice Boltzmann Large Eddy Simulation Model of MHD" (arXiv:1607.08675):
D2Q9 multi-relaxation-time collision for the density distribution, D2Q5
single-relaxation collision for the vector magnetic distribution, relaxation
times carrying the eddy viscosity and resistivity computed from each site's
non-equilibrium moments.  The hot path lives in ``liblbmhd.so`` (hand-written
HIP, C ABI in ``include/lbmhd.h``); this package only marshals arguments.

Submodules are imported lazily so that importing the package never loads the
GPU library: ``lattice.Lattice``, ``adjoint.LBMHDFunction``, ``build.build``.
"""

__all__ = ["Lattice", "LBMHDConfig", "LBMHDFunction"]


def __getattr__(name):
    if name in ("Lattice", "LBMHDConfig"):
        from . import lattice
        return getattr(lattice, name)
    if name == "LBMHDFunction":
        from . import adjoint
        return adjoint.LBMHDFunction
    raise AttributeError(name)
