"""nmc: the convolution method for the gravitational potential on nested
Cartesian meshes (Vorobyov et al. 2023, arXiv:2301.06763), native on AMD
Instinct MI355X (gfx950).

The compute path is the HIP library libnmc.so (C ABI in include/nmc.h);
``paper_2301_06763_amd.nmc`` is its ctypes binding and
``paper_2301_06763_amd.inputs`` builds seeded synthetic densities.
Submodules are imported lazily so that building or reading inputs needs no GPU.
"""
import importlib

__all__ = ["nmc", "inputs", "build", "serve"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
