"""MI355X-native EMT nodal-analysis time loop (trapezoidal companion models,
nodal injections, prefactored conductance solves), FP64, hand-written HIP.

Submodules load lazily so that the input generator (`netgen`) can be imported
without the HIP library.
"""
__all__ = ["netgen", "sim", "autograd"]


def __getattr__(name):
    import importlib
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
