"""MI355X (gfx950) HIP implementation of R^2-Gaussian's differentiable X-ray
rasterizer and voxelizer (arXiv 2405.20693) behind the C ABI of include/gs.h.

The package holds the HIP sources (csrc/), their build (build.py), the ctypes
binding (_native.py), the PyTorch-facing calls and autograd functions (ops.py)
and the training-iteration driver (iteration.py).  Importing it does not load
the library; the first call does, and fails loudly if it is not built.
"""
__all__ = ["ops", "iteration", "build"]


def __getattr__(name):
    if name in ("ops", "iteration", "build", "_native"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
