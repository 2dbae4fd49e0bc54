"""MI355X (gfx950) ensembles of active Brownian particles with an energy depot on a ratchet.

The compute path is libabp.so (HIP, built in-tree from csrc/); this package is its Python front
end. Submodules: ``api`` (integrate / reduce / run), ``workloads`` (seeded synthetic inputs),
``build`` (hipcc build of the library).
"""
from importlib import import_module

__all__ = ["api", "workloads", "build", "State", "init_state", "integrate", "reduce",
           "reduce_state", "run", "philox", "sweep", "AbpError"]

_API_NAMES = {"State", "init_state", "integrate", "reduce", "reduce_state", "run", "philox",
              "AbpError", "reduce_workspace", "Result", "sweep", "SweepResult", "reset_state"}


def __getattr__(name):
    if name in _API_NAMES:
        return getattr(import_module(".api", __name__), name)
    if name in ("api", "workloads", "build", "_lib"):
        return import_module("." + name, __name__)
    raise AttributeError(name)
