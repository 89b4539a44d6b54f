"""MI355X-native coupled lattice-Boltzmann / rigid-body step for three-bead
swimmers (Pickl et al., arXiv:1108.0786).

The compute path is the HIP library built from ``csrc/`` into
``_lib/liblbmswim.so`` (C-ABI in ``include/lbmswim.h``); ``sim`` holds the
torch/ctypes binding.  Importing the package does not load the library."""

__all__ = ["Sim", "BatchSim"]


def __getattr__(name):
    if name in ("Sim", "BatchSim"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
