"""MI355X-native Barnes-Hut gravitational potential on octree AMR meshes.

The compute path is the HIP library libbh.so (C ABI in include/bh.h); the
submodule ``binding`` marshals torch tensors into it and ``solver`` bundles the
handles of one grid.  Importing this package does not load the library; the
first use of ``binding`` does, and fails loudly when it is not built.
"""
__all__ = ["binding", "solver"]
