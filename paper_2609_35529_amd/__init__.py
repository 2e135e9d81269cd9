"""MI355X-native (gfx950) VLBM stream-and-collide with conservative local grid refinement.

Importing the package loads nothing native; ``paper_2609_35529_amd.vlbm`` binds the
HIP library ``libvlbm.so`` and raises if it has not been built.
"""
__all__ = ["vlbm", "workloads"]
