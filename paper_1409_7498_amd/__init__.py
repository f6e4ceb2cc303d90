"""MI355X-native reaction step for step- and chain-growth polymerization.

The compute path is the HIP library ``libpolyreact.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/polyreact.h``; ``binding`` marshals
arguments to it.  ``workload`` generates seeded synthetic inputs on the host.
"""
from . import workload  # noqa: F401

__all__ = ["workload", "binding"]


def __getattr__(name):
    if name == "binding":
        import importlib
        return importlib.import_module(__name__ + ".binding")
    raise AttributeError(name)
