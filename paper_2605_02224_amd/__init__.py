"""MI355X (gfx950) engine for Manifold k-NN queries over successor lists.

The compiled library (libmknn.so) is loaded on first use; importing the package does not
touch the GPU.  ``workloads`` holds the seeded input generators and imports nothing else.
"""
__all__ = ["Cloud", "MknnError"]


def __getattr__(name):
    if name == "Cloud":
        from .api import Cloud
        return Cloud
    if name == "MknnError":
        from ._lib import MknnError
        return MknnError
    raise AttributeError(name)
