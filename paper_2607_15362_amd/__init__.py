"""MI355X-native GOC-LBM: the central-moment MRT lattice Boltzmann method in
general orthogonal coordinates (with the coupled D2Q5 induction scheme) as
hand-written HIP kernels for gfx950 behind the C-ABI library libgoclbm.so.

Submodules:
  binding    ctypes binding of include/goc_lbm.h (argument marshalling only)
  build      compiles the library in-tree with hipcc
  workloads  seeded synthetic workloads (problem descriptions only)
"""
__all__ = ["binding", "build", "workloads"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
