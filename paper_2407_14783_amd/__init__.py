"""MI355X (gfx950) batched quadrotor step + BVH ray-cast renderer behind a C ABI.

The HIP library libvisfly_hip.so (built in-tree by ``paper_2407_14783_amd.build``)
does all the work; this package only marshals arguments (``capi``), wraps torch
device tensors and streams (``sim``), and adds the differentiable rollout
(``autograd``) and the serving loop (``serving``).  Importing ``capi`` without the
built library raises ImportError: there is no CPU fallback.
"""
__all__ = ["capi", "sim"]


def __getattr__(name):
    if name in ("capi", "sim", "autograd", "serving"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
